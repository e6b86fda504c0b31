// k_diag.hip -- FP64 diagnostics of the current state, deterministic two-stage reduction.
//
// Stage 1: each block accumulates a fixed, strided set of nodes in FP64 per thread,
// reduces across the 64-lane wavefront with cross-lane shuffles and across the block's
// waves through LDS, and writes one record of kDiagVals doubles.  Stage 2: one block
// sums the per-block records in a fixed order.  The result does not depend on timing.
//
// Record: [0] sum rho_A, [1] sum rho_B, [2..4] sum rho u, [5] W = sum w with
// w = max(phi, 0), [6..8] sum w x, [9..14] raw second moments sum w x_i x_j
// (xx, yy, zz, xy, xz, yz), [15] min(L^2 - tr C), [16] min leading minor of C,
// [17] max |u|, [18] sum m (tr C - 3), [19] sum m with m the polymer-phase weight
// (f+(phi), f-(phi), 1 or 0 as for the feedback).  Sec. 4.1 defines D and theta from the
// droplet's axes; the host forms them from the central moments.
#include <float.h>

#include "d3q19.h"
#include "lbfd_internal.h"

namespace lbfd {

constexpr int kDB = 256;

int64_t diag_blocks(int64_t N) {
    int64_t b = (N + kDB - 1) / kDB;
    return b < kMaxDiagBlocks ? b : kMaxDiagBlocks;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// kind: 0 = sum, 1 = min, 2 = max
__device__ __forceinline__ int red_kind(int k) { return k == 15 || k == 16 ? 1 : (k == 17 ? 2 : 0); }

__device__ void block_reduce_store(double (&acc)[kDiagVals], double* out) {
    __shared__ double sm[kDB / 64][kDiagVals];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) {
        const int kind = red_kind(k);
        double v = acc[k];
        v = kind == 0 ? wave_sum(v) : (kind == 1 ? wave_min(v) : wave_max(v));
        if (lane == 0) sm[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kDiagVals) {
        const int k = threadIdx.x;
        const int kind = red_kind(k);
        double v = sm[0][k];
        for (int w = 1; w < kDB / 64; ++w)
            v = kind == 0 ? v + sm[w][k] : (kind == 1 ? fmin(v, sm[w][k]) : fmax(v, sm[w][k]));
        out[k] = v;
    }
}

__global__ __launch_bounds__(kDB) void k_diag_stage1(DevParams p, const float* __restrict__ mom,
                                                     const float* __restrict__ uF,
                                                     const float* __restrict__ D,
                                                     double* __restrict__ part) {
    double acc[kDiagVals];
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) acc[k] = red_kind(k) == 1 ? DBL_MAX : (red_kind(k) == 2 ? 0.0 : 0.0);
    const int64_t N = p.N;
    const int64_t stride = (int64_t)gridDim.x * kDB;
    for (int64_t n = (int64_t)blockIdx.x * kDB + threadIdx.x; n < N; n += stride) {
        const int x = (int)(n % p.nx);
        const int64_t r = n / p.nx;
        const int y = (int)(r % p.ny);
        const int z = (int)(r / p.ny);
        const double rA = (double)p.rho0[0] + (double)mom[n];
        const double rB = p.nc == 2 ? (double)p.rho0[1] + (double)mom[N + n] : 0.0;
        const double rho = rA + rB;
        const double ux = uF[n], uy = uF[N + n], uz = uF[2 * N + n];
        acc[0] += rA;
        acc[1] += rB;
        acc[2] += rho * ux;
        acc[3] += rho * uy;
        acc[4] += rho * uz;
        const double phi = p.nc == 2 ? (rA - rB) / rho : 1.0;
        const double w = phi > 0.0 ? phi : 0.0;
        const double X = x, Y = y, Z = z;
        acc[5] += w;
        acc[6] += w * X;
        acc[7] += w * Y;
        acc[8] += w * Z;
        acc[9] += w * X * X;
        acc[10] += w * Y * Y;
        acc[11] += w * Z * Z;
        acc[12] += w * X * Y;
        acc[13] += w * X * Z;
        acc[14] += w * Y * Z;
        double c[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) c[k] = (double)D[k * N + n] + (k < 3 ? 1.0 : 0.0);
        acc[15] = fmin(acc[15], (double)p.L2 - (c[0] + c[1] + c[2]));
        const double m2 = c[0] * c[1] - c[3] * c[3];
        const double m3 = c[0] * (c[1] * c[2] - c[5] * c[5]) - c[3] * (c[3] * c[2] - c[5] * c[4]) +
                          c[4] * (c[3] * c[5] - c[1] * c[4]);
        acc[16] = fmin(acc[16], fmin(c[0], fmin(m2, m3)));
        acc[17] = fmax(acc[17], sqrt(ux * ux + uy * uy + uz * uz));
        double mp = 0.0;
        if (p.phase == 3) mp = 1.0;
        else if (p.phase == 1 || p.phase == 2) {
            const double t = tanh(phi * (double)p.inv_delta);
            mp = p.phase == 1 ? 0.5 * (1.0 + t) : 0.5 * (1.0 - t);
        }
        acc[18] += mp * (c[0] + c[1] + c[2] - 3.0);
        acc[19] += mp;
    }
    block_reduce_store(acc, part + (int64_t)blockIdx.x * kDiagVals);
}

__global__ __launch_bounds__(kDB) void k_diag_stage2(const double* __restrict__ part, int nblk,
                                                     double* __restrict__ out) {
    double acc[kDiagVals];
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) acc[k] = red_kind(k) == 1 ? DBL_MAX : 0.0;
    for (int b = threadIdx.x; b < nblk; b += kDB) {
#pragma unroll
        for (int k = 0; k < kDiagVals; ++k) {
            const double v = part[(int64_t)b * kDiagVals + k];
            const int kind = red_kind(k);
            acc[k] = kind == 0 ? acc[k] + v : (kind == 1 ? fmin(acc[k], v) : fmax(acc[k], v));
        }
    }
    block_reduce_store(acc, out);
}

hipError_t launch_diag_into(const DevParams& p, const Buffers& b, double* part, double* out, hipStream_t s) {
    // stage 1 writes every one of its nb records and stage 2 reads exactly those, so the
    // partials need no clearing between calls
    const int nb = (int)diag_blocks(p.N);
    hipLaunchKernelGGL(k_diag_stage1, dim3(nb), dim3(kDB), 0, s, p, b.mom, b.uF, b.D, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_stage2, dim3(1), dim3(kDB), 0, s, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_diag(const DevParams& p, const Buffers& b, hipStream_t s) {
    return launch_diag_into(p, b, b.red, b.red_out, s);
}

}  // namespace lbfd

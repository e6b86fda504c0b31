// k_fields.hip -- host <-> device field transfer kernels.
//
// k_init_box  : FP64 (rho_s, u, C) of a sub-box -> populations at the equilibrium of
//               Sec. 2 (no non-equilibrium part), stored as FP32 deviations
//               h = E_a(rho_s, u) - w_a rho0_s, and D = C - I.  The deviation is formed in
//               FP64 before rounding.
// k_fields_box: current side fields -> FP64 (rho_s, u with the half-force shift, C).
// Staging layout (FP64, B = box nodes): rho [nc][B], u [3][B], C [6][B].
#include "d3q19.h"
#include "lbfd_internal.h"

namespace lbfd {

constexpr int kFB = 256;

__global__ __launch_bounds__(kFB) void k_init_box(DevParams p, Box bx, const double* __restrict__ st,
                                                  float* __restrict__ h, float* __restrict__ D) {
    const int64_t B = (int64_t)bx.bx * bx.by * bx.bz;
    const int64_t i = (int64_t)blockIdx.x * kFB + threadIdx.x;
    if (i >= B) return;
    const int lx = (int)(i % bx.bx);
    const int64_t r = i / bx.bx;
    const int ly = (int)(r % bx.by);
    const int lz = (int)(r / bx.by);
    const int64_t n = ((int64_t)(bx.z0 + lz) * p.ny + (bx.y0 + ly)) * p.nx + (bx.x0 + lx);
    const int64_t N = p.N;
    const double* rho = st;
    const double* u = st + (int64_t)p.nc * B;
    const double* C = u + 3 * B;
    const double ux = u[i], uy = u[B + i], uz = u[2 * B + i];
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int s = 0; s < p.nc; ++s) {
        const double rs = rho[(int64_t)s * B + i];
        const double dr = rs - (double)p.rho0[s];
        float* hs = h + (int64_t)s * kQ * N;
#pragma unroll
        for (int a = 0; a < kQ; ++a) {
            const double cu = cx(a) * ux + cy(a) * uy + cz(a) * uz;
            const double w = a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
            hs[a * N + n] = (float)(w * (dr + rs * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)));
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) D[k * N + n] = (float)(C[k * B + i] - (k < 3 ? 1.0 : 0.0));
}

__global__ __launch_bounds__(kFB) void k_fields_box(DevParams p, Box bx, const float* __restrict__ mom,
                                                    const float* __restrict__ uF,
                                                    const float* __restrict__ D,
                                                    double* __restrict__ st) {
    const int64_t B = (int64_t)bx.bx * bx.by * bx.bz;
    const int64_t i = (int64_t)blockIdx.x * kFB + threadIdx.x;
    if (i >= B) return;
    const int lx = (int)(i % bx.bx);
    const int64_t r = i / bx.bx;
    const int ly = (int)(r % bx.by);
    const int lz = (int)(r / bx.by);
    const int64_t n = ((int64_t)(bx.z0 + lz) * p.ny + (bx.y0 + ly)) * p.nx + (bx.x0 + lx);
    const int64_t N = p.N;
    double* rho = st;
    double* u = st + (int64_t)p.nc * B;
    double* C = u + 3 * B;
    for (int s = 0; s < p.nc; ++s) rho[(int64_t)s * B + i] = (double)p.rho0[s] + (double)mom[s * N + n];
    for (int d = 0; d < 3; ++d) u[d * B + i] = (double)uF[d * N + n];
#pragma unroll
    for (int k = 0; k < 6; ++k) C[k * B + i] = (double)D[k * N + n] + (k < 3 ? 1.0 : 0.0);
}

hipError_t launch_init_box(const DevParams& p, const Buffers& b, const Box& box, hipStream_t s) {
    const int64_t B = (int64_t)box.bx * box.by * box.bz;
    hipLaunchKernelGGL(k_init_box, dim3((unsigned)((B + kFB - 1) / kFB)), dim3(kFB), 0, s, p, box,
                       b.stage, b.h, b.D);
    return hipGetLastError();
}

hipError_t launch_fields_box(const DevParams& p, const Buffers& b, const Box& box, hipStream_t s) {
    const int64_t B = (int64_t)box.bx * box.by * box.bz;
    hipLaunchKernelGGL(k_fields_box, dim3((unsigned)((B + kFB - 1) / kFB)), dim3(kFB), 0, s, p, box,
                       b.mom, b.uF, b.D, b.stage);
    return hipGetLastError();
}

}  // namespace lbfd

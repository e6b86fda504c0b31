// k_mlp.hip -- kernels of the small surrogate network 5 -> 128 -> 128 -> 3 (GELU) that maps
// droplet-sweep parameters to steady deformation, orientation and a warm-start amplitude.
//
// Training runs in FP32 with deterministic reductions (every sum has one thread and a fixed
// order; no atomics): layer forward with fused bias + GELU, MSE loss and its gradient,
// weight and input gradients, Adam.  Inference runs in BF16 with FP32 accumulation; the
// 128 x 128 hidden layer, the only real contraction, uses the CDNA matrix cores
// (v_mfma_f32_32x32x8bf16_1k).
//
// Parameter vector (FP32, this order): W1[128][5], b1[128], W2[128][128], b2[128],
// W3[3][128], b3[3].  Activations are row-major [sample][unit].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"

namespace lbfd {

namespace {

constexpr int kMB = 256;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z = X W^T + b, H = gelu(Z) (or H = Z): one thread per (sample, unit)
__global__ __launch_bounds__(kMB) void k_fwd(const float* __restrict__ X, int B, int K, const float* __restrict__ W,
                                             const float* __restrict__ bias, int M, float* __restrict__ Z,
                                             float* __restrict__ H, int act) {
    const int t = blockIdx.x * kMB + threadIdx.x;
    if (t >= B * M) return;
    const int b = t / M, m = t % M;
    float z = bias[m];
    for (int k = 0; k < K; ++k) z += W[m * K + k] * X[b * K + k];
    if (Z) Z[t] = z;
    H[t] = act ? gelu(z) : z;
}

// mean squared error over B x 3 outputs; dY = 2 (Y - T) / (3 B).  One block, fixed order.
__global__ __launch_bounds__(kMB) void k_loss(const float* __restrict__ Y, const float* __restrict__ T, int n,
                                              float* __restrict__ dY, float* __restrict__ loss) {
    __shared__ float sm[kMB];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += kMB) {
        const float d = Y[i] - T[i];
        dY[i] = 2.0f * d / (float)n;
        acc += d * d;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kMB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sm[0] / (float)n;
}

// dW[m][k] = sum_b dZ[b][m] X[b][k] (threads m*K + k), db[m] = sum_b dZ[b][m] (threads M*K + m)
__global__ __launch_bounds__(kMB) void k_wgrad(const float* __restrict__ dZ, int B, int M, const float* __restrict__ X,
                                               int K, float* __restrict__ dW, float* __restrict__ db) {
    const int t = blockIdx.x * kMB + threadIdx.x;
    if (t < M * K) {
        const int m = t / K, k = t % K;
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += dZ[b * M + m] * X[b * K + k];
        dW[t] = s;
    } else if (t < M * K + M) {
        const int m = t - M * K;
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += dZ[b * M + m];
        db[m] = s;
    }
}

// dZprev[b][k] = (sum_m dZ[b][m] W[m][k]) * gelu'(Zprev[b][k])
__global__ __launch_bounds__(kMB) void k_igrad(const float* __restrict__ dZ, int B, int M, const float* __restrict__ W,
                                               int K, const float* __restrict__ Zprev, float* __restrict__ dZprev) {
    const int t = blockIdx.x * kMB + threadIdx.x;
    if (t >= B * K) return;
    const int b = t / K, k = t % K;
    float s = 0.0f;
    for (int m = 0; m < M; ++m) s += dZ[b * M + m] * W[m * K + k];
    dZprev[t] = s * gelu_grad(Zprev[t]);
}

__global__ __launch_bounds__(kMB) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
    const int i = blockIdx.x * kMB + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// minibatch from the resident training set: rows idx[0..B) of X_all [n][5] and T_all [n][3]
__global__ __launch_bounds__(kMB) void k_gather(const float* __restrict__ Xa, const float* __restrict__ Ta,
                                                const int* __restrict__ idx, int B, float* __restrict__ X,
                                                float* __restrict__ T) {
    const int t = blockIdx.x * kMB + threadIdx.x;
    if (t >= B * 8) return;
    const int b = t / 8, c = t % 8;
    const int r = idx[b];
    if (c < 5)
        X[b * 5 + c] = Xa[r * 5 + c];
    else
        T[b * 3 + c - 5] = Ta[r * 3 + c - 5];
}

// FP32 -> BF16, round to nearest even (finite inputs)
__global__ __launch_bounds__(kMB) void k_to_bf16(const float* __restrict__ s, uint16_t* __restrict__ d, int n) {
    const int i = blockIdx.x * kMB + threadIdx.x;
    if (i >= n) return;
    const uint32_t u = __float_as_uint(s[i]);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    d[i] = (uint16_t)(r >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t x) { return __uint_as_float(((uint32_t)x) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// BF16 inference of 32 samples per workgroup (4 waves).  Layer 1 and 3 on the vector ALUs
// (K = 5 and N = 3 are too thin for the matrix cores); layer 2 as 4 wave tiles of
// 32 samples x 32 units, each 16 MFMA 32x32x8 steps over K = 128.
__global__ __launch_bounds__(256) void k_infer_bf16(const float* __restrict__ X, int B, const uint16_t* __restrict__ W1,
                                                    const float* __restrict__ b1, const uint16_t* __restrict__ W2,
                                                    const float* __restrict__ b2, const uint16_t* __restrict__ W3,
                                                    const float* __restrict__ b3, float* __restrict__ Y) {
    __shared__ uint16_t h1[32][128 + 8];  // bf16 activations, padded rows
    __shared__ float h2[32][128 + 4];
    const int s0 = blockIdx.x * 32;
    const int tid = threadIdx.x;
    // layer 1: 32 x 128 outputs, 16 per thread
    for (int o = tid; o < 32 * 128; o += 256) {
        const int m = o / 128, j = o % 128;
        const int s = s0 + m;
        float z = b1[j];
        if (s < B) {
#pragma unroll
            for (int k = 0; k < 5; ++k) z += bf2f(W1[j * 5 + k]) * bf2f(f2bf(X[s * 5 + k]));
        }
        h1[m][j] = f2bf(s < B ? gelu(z) : 0.0f);
    }
    __syncthreads();
    // layer 2 on the matrix cores
    const int wave = tid >> 6, lane = tid & 63;
    const int n = wave * 32 + (lane & 31);  // output unit of this lane (B operand column)
    const int kq = (lane >> 5) * 4;          // first of the 4 consecutive K values of this lane
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int k0 = 0; k0 < 128; k0 += 8) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = (short)h1[lane & 31][k0 + kq + i];
            b[i] = (short)W2[n * 128 + k0 + kq + i];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);  // sample row of accumulator r
        h2[m][n] = bf2f(f2bf(gelu(acc[r] + b2[n])));
    }
    __syncthreads();
    // layer 3: 32 x 3 outputs
    if (tid < 96) {
        const int m = tid / 3, o = tid % 3;
        const int s = s0 + m;
        float z = b3[o];
        for (int k = 0; k < 128; ++k) z += bf2f(W3[o * 128 + k]) * h2[m][k];
        if (s < B) Y[s * 3 + o] = z;
    }
}

inline dim3 g1(int64_t n) { return dim3((unsigned)((n + kMB - 1) / kMB)); }

}  // namespace

hipError_t mlp_forward(const MlpBuffers& m, const float* X, int B, float* Y, hipStream_t s) {
    hipLaunchKernelGGL(k_fwd, g1((int64_t)B * kHid), dim3(kMB), 0, s, X, B, kIn, m.W1, m.b1, kHid, m.Z1, m.H1, 1);
    hipLaunchKernelGGL(k_fwd, g1((int64_t)B * kHid), dim3(kMB), 0, s, m.H1, B, kHid, m.W2, m.b2, kHid, m.Z2, m.H2, 1);
    hipLaunchKernelGGL(k_fwd, g1((int64_t)B * kOut), dim3(kMB), 0, s, m.H2, B, kHid, m.W3, m.b3, kOut,
                       (float*)nullptr, Y, 0);
    return hipGetLastError();
}

hipError_t mlp_backward(const MlpBuffers& m, const float* X, const float* T, int B, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kMB), 0, s, m.Y, T, B * kOut, m.dY, m.loss);
    hipLaunchKernelGGL(k_wgrad, g1(kOut * kHid + kOut), dim3(kMB), 0, s, m.dY, B, kOut, m.H2, kHid, m.gW3, m.gb3);
    hipLaunchKernelGGL(k_igrad, g1((int64_t)B * kHid), dim3(kMB), 0, s, m.dY, B, kOut, m.W3, kHid, m.Z2, m.dZ2);
    hipLaunchKernelGGL(k_wgrad, g1(kHid * kHid + kHid), dim3(kMB), 0, s, m.dZ2, B, kHid, m.H1, kHid, m.gW2, m.gb2);
    hipLaunchKernelGGL(k_igrad, g1((int64_t)B * kHid), dim3(kMB), 0, s, m.dZ2, B, kHid, m.W2, kHid, m.Z1, m.dZ1);
    hipLaunchKernelGGL(k_wgrad, g1(kHid * kIn + kHid), dim3(kMB), 0, s, m.dZ1, B, kHid, X, kIn, m.gW1, m.gb1);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpBuffers& m, float lr, float b1, float b2, float eps, int64_t t, hipStream_t s) {
    const float bc1 = 1.0f - powf(b1, (float)t), bc2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, g1(kNParams), dim3(kMB), 0, s, m.P, m.G, m.mom1, m.mom2, kNParams, lr, b1, b2, eps, bc1,
                       bc2);
    return hipGetLastError();
}

hipError_t mlp_gather(const MlpBuffers& m, const int* idx, int B, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, g1((int64_t)B * 8), dim3(kMB), 0, s, m.Xall, m.Tall, idx, B, m.X, m.T);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const MlpBuffers& m, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, g1(kNParams), dim3(kMB), 0, s, m.P, m.Pb, kNParams);
    return hipGetLastError();
}

hipError_t mlp_infer_bf16(const MlpBuffers& m, const float* X, int B, float* Y, hipStream_t s) {
    const uint16_t* W1 = m.Pb + kOffW1;
    const uint16_t* W2 = m.Pb + kOffW2;
    const uint16_t* W3 = m.Pb + kOffW3;
    hipLaunchKernelGGL(k_infer_bf16, dim3((unsigned)((B + 31) / 32)), dim3(256), 0, s, X, B, W1, m.b1, W2, m.b2, W3,
                       m.b3, Y);
    return hipGetLastError();
}

}  // namespace lbfd

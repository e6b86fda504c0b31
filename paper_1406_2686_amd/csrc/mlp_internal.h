// mlp_internal.h -- sizes and device buffer views of the surrogate network (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfd {

constexpr int kIn = 5, kHid = 128, kOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kOut * kHid;
constexpr int kNParams = kOffB3 + kOut;  // 17667

struct MlpBuffers {
    float* P;        // parameters (FP32)
    float *W1, *b1, *W2, *b2, *W3, *b3;
    float* G;        // gradients, same layout
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
    float *mom1, *mom2;  // Adam moments
    uint16_t* Pb;    // BF16 copy of the parameters (inference)
    // activations for up to max_batch samples
    float *X, *T, *Z1, *H1, *Z2, *H2, *Y, *dY, *dZ2, *dZ1;
    float* loss;
    // resident training set and minibatch indices
    float *Xall, *Tall;
    int* idx;
    int max_batch, max_train;
};

hipError_t mlp_forward(const MlpBuffers& m, const float* X, int B, float* Y, hipStream_t s);
hipError_t mlp_backward(const MlpBuffers& m, const float* X, const float* T, int B, hipStream_t s);
hipError_t mlp_adam(const MlpBuffers& m, float lr, float b1, float b2, float eps, int64_t t, hipStream_t s);
hipError_t mlp_gather(const MlpBuffers& m, const int* idx, int B, hipStream_t s);
hipError_t mlp_to_bf16(const MlpBuffers& m, hipStream_t s);
hipError_t mlp_infer_bf16(const MlpBuffers& m, const float* X, int B, float* Y, hipStream_t s);

}  // namespace lbfd

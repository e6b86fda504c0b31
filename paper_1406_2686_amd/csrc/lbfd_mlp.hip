// lbfd_mlp.hip -- C ABI of the surrogate network (declared in include/lbfd.h): lifecycle,
// parameters, FP32 forward / loss+gradient / Adam, on-device training over a resident
// data set, and BF16 inference.  Kernels live in k_mlp.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "lbfd.h"
#include "mlp_internal.h"

using namespace lbfd;

struct lbfd_mlp {
    MlpBuffers m;
    hipStream_t stream;
    int device;
    int64_t adam_t;
    bool bf16_ok;
    std::string err;
};

namespace {

constexpr uint64_t kA = 256;
inline uint64_t a256(uint64_t v) { return (v + kA - 1) / kA * kA; }

struct MlpLayout {
    uint64_t P, G, m1, m2, Pb, X, T, Z1, H1, Z2, H2, Y, dY, dZ2, dZ1, loss, Xall, Tall, idx, total;
};

MlpLayout mlp_layout(int B, int NT) {
    MlpLayout L{};
    uint64_t off = 0;
    auto take = [&](uint64_t n) {
        uint64_t o = off;
        off = a256(off + n);
        return o;
    };
    L.P = take(4ull * kNParams);
    L.G = take(4ull * kNParams);
    L.m1 = take(4ull * kNParams);
    L.m2 = take(4ull * kNParams);
    L.Pb = take(2ull * kNParams);
    L.X = take(4ull * B * kIn);
    L.T = take(4ull * B * kOut);
    L.Z1 = take(4ull * B * kHid);
    L.H1 = take(4ull * B * kHid);
    L.Z2 = take(4ull * B * kHid);
    L.H2 = take(4ull * B * kHid);
    L.Y = take(4ull * B * kOut);
    L.dY = take(4ull * B * kOut);
    L.dZ2 = take(4ull * B * kHid);
    L.dZ1 = take(4ull * B * kHid);
    L.loss = take(4);
    L.Xall = take(4ull * std::max(NT, 1) * kIn);
    L.Tall = take(4ull * std::max(NT, 1) * kOut);
    L.idx = take(4ull * std::max(NT, 1));
    L.total = off;
    return L;
}

// splitmix64 (Steele, Lea & Flood 2014): counter-based, for the default initialisation
uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}
double unit(uint64_t seed, uint64_t i) { return (double)(splitmix64(seed * 0x100000001b3ull + i) >> 11) * (1.0 / 9007199254740992.0); }

lbfd_status mfail(lbfd_mlp* m, lbfd_status st, const std::string& msg) {
    if (m) m->err = msg;
    return st;
}

#define MCHK(mm, expr, where)                                                                    \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) return mfail(mm, LBFD_EDEVICE, std::string(where) + ": " + hipGetErrorString(_e)); \
    } while (0)

bool opts_ok(const lbfd_train_opts* o) {
    return o && o->epochs >= 1 && o->batch >= 1 && o->lr > 0.f && o->beta1 >= 0.f && o->beta1 < 1.f &&
           o->beta2 >= 0.f && o->beta2 < 1.f && o->eps > 0.f;
}

}  // namespace

extern "C" {

lbfd_status lbfd_mlp_state_bytes(int32_t max_batch, int32_t max_train, uint64_t* bytes) {
    if (max_batch < 1 || max_train < 0 || !bytes) return LBFD_EINVAL;
    *bytes = mlp_layout(max_batch, max_train).total;
    return LBFD_OK;
}

lbfd_status lbfd_mlp_create(int32_t max_batch, int32_t max_train, uint64_t seed, void* dev, uint64_t bytes,
                            void* hip_stream, lbfd_mlp** out) {
    if (!out) return LBFD_EINVAL;
    *out = nullptr;
    if (max_batch < 1 || max_train < 0 || !dev || ((uintptr_t)dev % kA)) return LBFD_EINVAL;
    const MlpLayout L = mlp_layout(max_batch, max_train);
    if (bytes < L.total) return LBFD_ENOMEM;
    lbfd_mlp* n = new (std::nothrow) lbfd_mlp();
    if (!n) return LBFD_ENOMEM;
    char* b = (char*)dev;
    MlpBuffers& m = n->m;
    m.P = (float*)(b + L.P);
    m.G = (float*)(b + L.G);
    m.mom1 = (float*)(b + L.m1);
    m.mom2 = (float*)(b + L.m2);
    m.Pb = (uint16_t*)(b + L.Pb);
    m.W1 = m.P + kOffW1; m.b1 = m.P + kOffB1; m.W2 = m.P + kOffW2; m.b2 = m.P + kOffB2; m.W3 = m.P + kOffW3; m.b3 = m.P + kOffB3;
    m.gW1 = m.G + kOffW1; m.gb1 = m.G + kOffB1; m.gW2 = m.G + kOffW2; m.gb2 = m.G + kOffB2; m.gW3 = m.G + kOffW3; m.gb3 = m.G + kOffB3;
    m.X = (float*)(b + L.X); m.T = (float*)(b + L.T); m.Z1 = (float*)(b + L.Z1); m.H1 = (float*)(b + L.H1);
    m.Z2 = (float*)(b + L.Z2); m.H2 = (float*)(b + L.H2); m.Y = (float*)(b + L.Y); m.dY = (float*)(b + L.dY);
    m.dZ2 = (float*)(b + L.dZ2); m.dZ1 = (float*)(b + L.dZ1); m.loss = (float*)(b + L.loss);
    m.Xall = (float*)(b + L.Xall); m.Tall = (float*)(b + L.Tall); m.idx = (int*)(b + L.idx);
    m.max_batch = max_batch;
    m.max_train = max_train;
    n->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&n->device);
    n->adam_t = 0;
    n->bf16_ok = false;
    // Glorot-uniform weights, zero biases
    std::vector<float> p(kNParams, 0.0f);
    auto fill = [&](int off, int fan_out, int fan_in) {
        const double a = sqrt(6.0 / (fan_in + fan_out));
        for (int i = 0; i < fan_out * fan_in; ++i) p[off + i] = (float)((2.0 * unit(seed, off + i) - 1.0) * a);
    };
    fill(kOffW1, kHid, kIn);
    fill(kOffW2, kHid, kHid);
    fill(kOffW3, kOut, kHid);
    lbfd_status st = lbfd_mlp_set_params(n, p.data());
    if (st != LBFD_OK) {
        delete n;
        return st;
    }
    *out = n;
    return LBFD_OK;
}

lbfd_status lbfd_mlp_set_params(lbfd_mlp* n, const float* params) {
    if (!n || !params) return LBFD_EINVAL;
    for (int i = 0; i < kNParams; ++i)
        if (!isfinite(params[i])) return mfail(n, LBFD_EINVAL, "non-finite parameter");
    (void)hipSetDevice(n->device);
    MCHK(n, hipMemcpyAsync(n->m.P, params, 4ull * kNParams, hipMemcpyHostToDevice, n->stream), "upload");
    MCHK(n, hipMemsetAsync(n->m.mom1, 0, 4ull * kNParams, n->stream), "adam reset");
    MCHK(n, hipMemsetAsync(n->m.mom2, 0, 4ull * kNParams, n->stream), "adam reset");
    MCHK(n, hipStreamSynchronize(n->stream), "sync");
    n->adam_t = 0;
    n->bf16_ok = false;
    return LBFD_OK;
}

lbfd_status lbfd_mlp_get_params(lbfd_mlp* n, float* params) {
    if (!n || !params) return LBFD_EINVAL;
    (void)hipSetDevice(n->device);
    MCHK(n, hipMemcpyAsync(params, n->m.P, 4ull * kNParams, hipMemcpyDeviceToHost, n->stream), "download");
    MCHK(n, hipStreamSynchronize(n->stream), "sync");
    return LBFD_OK;
}

lbfd_status lbfd_mlp_forward(lbfd_mlp* n, const float* X, int32_t count, float* Y) {
    if (!n || !X || !Y || count < 0) return LBFD_EINVAL;
    (void)hipSetDevice(n->device);
    for (int s0 = 0; s0 < count; s0 += n->m.max_batch) {
        const int B = std::min(n->m.max_batch, count - s0);
        MCHK(n, hipMemcpyAsync(n->m.X, X + (int64_t)s0 * kIn, 4ull * B * kIn, hipMemcpyHostToDevice, n->stream), "upload");
        MCHK(n, mlp_forward(n->m, n->m.X, B, n->m.Y, n->stream), "forward");
        MCHK(n, hipMemcpyAsync(Y + (int64_t)s0 * kOut, n->m.Y, 4ull * B * kOut, hipMemcpyDeviceToHost, n->stream), "download");
    }
    MCHK(n, hipStreamSynchronize(n->stream), "sync");
    return LBFD_OK;
}

lbfd_status lbfd_mlp_loss_grad(lbfd_mlp* n, const float* X, const float* T, int32_t count, float* loss, float* grad) {
    if (!n || !X || !T || count < 1 || count > n->m.max_batch) return LBFD_EINVAL;
    (void)hipSetDevice(n->device);
    MCHK(n, hipMemcpyAsync(n->m.X, X, 4ull * count * kIn, hipMemcpyHostToDevice, n->stream), "upload");
    MCHK(n, hipMemcpyAsync(n->m.T, T, 4ull * count * kOut, hipMemcpyHostToDevice, n->stream), "upload");
    MCHK(n, mlp_forward(n->m, n->m.X, count, n->m.Y, n->stream), "forward");
    MCHK(n, mlp_backward(n->m, n->m.X, n->m.T, count, n->stream), "backward");
    if (loss) MCHK(n, hipMemcpyAsync(loss, n->m.loss, 4, hipMemcpyDeviceToHost, n->stream), "download");
    if (grad) MCHK(n, hipMemcpyAsync(grad, n->m.G, 4ull * kNParams, hipMemcpyDeviceToHost, n->stream), "download");
    MCHK(n, hipStreamSynchronize(n->stream), "sync");
    return LBFD_OK;
}

lbfd_status lbfd_mlp_adam_step(lbfd_mlp* n, const lbfd_train_opts* o) {
    if (!n || !opts_ok(o)) return LBFD_EINVAL;
    (void)hipSetDevice(n->device);
    n->adam_t += 1;
    MCHK(n, mlp_adam(n->m, o->lr, o->beta1, o->beta2, o->eps, n->adam_t, n->stream), "adam");
    n->bf16_ok = false;
    MCHK(n, hipStreamSynchronize(n->stream), "sync");
    return LBFD_OK;
}

lbfd_status lbfd_mlp_train(lbfd_mlp* n, const float* X, const float* T, int32_t count, const lbfd_train_opts* o,
                           float* final_loss) {
    if (!n || !X || !T || count < 1 || !opts_ok(o)) return LBFD_EINVAL;
    if (count > n->m.max_train) return mfail(n, LBFD_EINVAL, "more samples than max_train");
    (void)hipSetDevice(n->device);
    MCHK(n, hipMemcpyAsync(n->m.Xall, X, 4ull * count * kIn, hipMemcpyHostToDevice, n->stream), "upload");
    MCHK(n, hipMemcpyAsync(n->m.Tall, T, 4ull * count * kOut, hipMemcpyHostToDevice, n->stream), "upload");
    const int B = std::min(std::min(o->batch, n->m.max_batch), count);
    std::vector<int> perm(count);
    float last = 0.0f;
    for (int ep = 0; ep < o->epochs; ++ep) {
        // seeded Fisher-Yates permutation per epoch; one upload per epoch, the minibatches
        // are gathered on the device
        std::iota(perm.begin(), perm.end(), 0);
        for (int i = count - 1; i > 0; --i) {
            const int j = (int)(unit(o->seed + 0x51ull * (uint64_t)(ep + 1), (uint64_t)i) * (i + 1));
            std::swap(perm[i], perm[std::min(j, i)]);
        }
        MCHK(n, hipMemcpyAsync(n->m.idx, perm.data(), 4ull * count, hipMemcpyHostToDevice, n->stream), "upload");
        for (int s0 = 0; s0 + B <= count; s0 += B) {
            MCHK(n, mlp_gather(n->m, n->m.idx + s0, B, n->stream), "gather");
            MCHK(n, mlp_forward(n->m, n->m.X, B, n->m.Y, n->stream), "forward");
            MCHK(n, mlp_backward(n->m, n->m.X, n->m.T, B, n->stream), "backward");
            n->adam_t += 1;
            MCHK(n, mlp_adam(n->m, o->lr, o->beta1, o->beta2, o->eps, n->adam_t, n->stream), "adam");
        }
        // the host copy (which waits for the stream) is the stream's only sync per epoch
        MCHK(n, hipMemcpyAsync(&last, n->m.loss, 4, hipMemcpyDeviceToHost, n->stream), "loss");
        MCHK(n, hipStreamSynchronize(n->stream), "sync");
    }
    n->bf16_ok = false;
    if (final_loss) *final_loss = last;
    return LBFD_OK;
}

lbfd_status lbfd_mlp_infer_bf16(lbfd_mlp* n, const float* X, int32_t count, float* Y) {
    if (!n || !X || !Y || count < 0) return LBFD_EINVAL;
    (void)hipSetDevice(n->device);
    if (!n->bf16_ok) {
        MCHK(n, mlp_to_bf16(n->m, n->stream), "bf16 weights");
        n->bf16_ok = true;
    }
    for (int s0 = 0; s0 < count; s0 += n->m.max_batch) {
        const int B = std::min(n->m.max_batch, count - s0);
        MCHK(n, hipMemcpyAsync(n->m.X, X + (int64_t)s0 * kIn, 4ull * B * kIn, hipMemcpyHostToDevice, n->stream), "upload");
        MCHK(n, mlp_infer_bf16(n->m, n->m.X, B, n->m.Y, n->stream), "infer");
        MCHK(n, hipMemcpyAsync(Y + (int64_t)s0 * kOut, n->m.Y, 4ull * B * kOut, hipMemcpyDeviceToHost, n->stream), "download");
    }
    MCHK(n, hipStreamSynchronize(n->stream), "sync");
    return LBFD_OK;
}

void lbfd_mlp_destroy(lbfd_mlp* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipStreamSynchronize(n->stream);
    delete n;
}

const char* lbfd_mlp_last_error(const lbfd_mlp* n) { return n ? n->err.c_str() : "null network"; }

}  // extern "C"

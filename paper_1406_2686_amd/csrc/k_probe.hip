// k_probe.hip -- streaming-bandwidth probe of the HBM of the GPU the library runs on: the
// read, write and copy rates a plain streaming kernel reaches, the ceiling the step kernels'
// traffic is judged against.  Every lane moves 16-byte vectors (one global_load/store_dwordx4),
// a wavefront 1 KiB of consecutive bytes per instruction; grid-stride loops over 8 waves
// per SIMD worth of workgroups.  Writes are plain or nontemporal (streaming) stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbfd.h"

namespace {

constexpr int kPB = 256;
typedef float v4f __attribute__((ext_vector_type(4)));  // one dwordx4 access per lane

__global__ __launch_bounds__(kPB) void k_probe_read(const v4f* __restrict__ src, int64_t n4,
                                                    float* __restrict__ sink) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int64_t stride = (int64_t)gridDim.x * kPB;
    for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n4; i += stride) {
        acc += src[i];
    }
    // one lane per block publishes (keeps the loads alive); the value itself is unused
    const float s = (acc.x + acc.y) + (acc.z + acc.w);
    if (s == 1234.5f) sink[blockIdx.x] = s;
}

template <bool NT>
__global__ __launch_bounds__(kPB) void k_probe_write(v4f* __restrict__ dst, int64_t n4, float v) {
    const int64_t stride = (int64_t)gridDim.x * kPB;
    const v4f q = {v, v, v, v};
    for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n4; i += stride) {
        if constexpr (NT) __builtin_nontemporal_store(q, dst + i);
        else dst[i] = q;
    }
}

template <bool NT>
__global__ __launch_bounds__(kPB) void k_probe_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                    int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kPB;
    for (int64_t i = (int64_t)blockIdx.x * kPB + threadIdx.x; i < n4; i += stride) {
        const v4f v = src[i];
        if constexpr (NT) __builtin_nontemporal_store(v, dst + i);
        else dst[i] = v;
    }
}

}  // namespace

extern "C" {

lbfd_status lbfd_stream_probe(int32_t kind, void* dev_src, void* dev_dst, uint64_t bytes, int32_t reps,
                              void* hip_stream, double* ms_per_launch) {
    if (kind < LBFD_PROBE_READ || kind > LBFD_PROBE_COPY_NT || reps < 1 || !ms_per_launch) return LBFD_EINVAL;
    if (bytes < 16 || bytes % 16 != 0) return LBFD_EINVAL;
    const bool needs_src = kind == LBFD_PROBE_READ || kind >= LBFD_PROBE_COPY;
    const bool needs_dst = kind != LBFD_PROBE_READ;
    if ((needs_src && (!dev_src || (uintptr_t)dev_src % 16)) || (needs_dst && (!dev_dst || (uintptr_t)dev_dst % 16)))
        return LBFD_EINVAL;
    // the read probe's sink: one float per workgroup at the start of dst when given, else of
    // src (grid <= bytes/4096, inside the buffer); a workgroup stores only when its sum is
    // exactly 1234.5, so in practice nothing is written
    float* sink = (float*)(dev_dst ? dev_dst : dev_src);
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return LBFD_EDEVICE;
    const int64_t n4 = (int64_t)(bytes / 16);
    const int64_t want = (int64_t)ncu * 32;  // 32 workgroups of 4 waves per CU: 8 waves per SIMD
    const unsigned grid = (unsigned)(want < (n4 + kPB - 1) / kPB ? want : (n4 + kPB - 1) / kPB);
    auto launch = [&]() {
        const v4f* src = (const v4f*)dev_src;
        v4f* dst = (v4f*)dev_dst;
        switch (kind) {
            case LBFD_PROBE_READ: hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(kPB), 0, s, src, n4, sink); break;
            case LBFD_PROBE_WRITE: hipLaunchKernelGGL(k_probe_write<false>, dim3(grid), dim3(kPB), 0, s, dst, n4, 1.0f); break;
            case LBFD_PROBE_WRITE_NT: hipLaunchKernelGGL(k_probe_write<true>, dim3(grid), dim3(kPB), 0, s, dst, n4, 1.0f); break;
            case LBFD_PROBE_COPY: hipLaunchKernelGGL(k_probe_copy<false>, dim3(grid), dim3(kPB), 0, s, src, dst, n4); break;
            default: hipLaunchKernelGGL(k_probe_copy<true>, dim3(grid), dim3(kPB), 0, s, src, dst, n4); break;
        }
    };
    launch();  // warm-up
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return LBFD_EDEVICE;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return LBFD_EDEVICE;
    }
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(b, s);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return LBFD_EDEVICE;
    *ms_per_launch = (double)ms / reps;
    return LBFD_OK;
}

}  // extern "C"

// lbfd_noalloc.hip -- lbfd_diagnostics_noalloc: the FP64 diagnostics of lbfd_diagnostics
// for callers that may not allocate device memory.  Its two-stage reduction keeps the
// stage-1 partial records and the final record in a file-scope device array (`scratch`)
// instead of the context's buffer; the kernels are those of lbfd_diagnostics, so both
// entry points return identical records.
//
// `scratch` exists once per GPU (each device that loads the library holds its own copy
// until the process ends).  In host code its name is only a stand-in for the symbol: the
// device address is taken once per device with hipGetSymbolAddress, with that device
// current, and only that address is handed to kernels and copies.  Every call on one GPU
// shares the array, so calls that overlap on one GPU (from different streams or threads)
// race; callers serialise them.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>

#include "lbfd.h"
#include "lbfd_ctx.h"
#include "lbfd_internal.h"

using namespace lbfd;

namespace {

// stage-1 partials (one record per workgroup, at most kMaxDiagBlocks) and the final record
constexpr int kScratchRecords = kMaxDiagBlocks + 1;
constexpr size_t kScratchDoubles = (size_t)kScratchRecords * kDiagVals;  // 164,000 bytes

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), taken on the first call
// for that device and kept for the rest of the process.
hipError_t scratch_on(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

lbfd_status na_fail(lbfd_ctx* c, lbfd_status st, const std::string& msg) {
    c->err = msg;
    return st;
}

#define NACHK(c, expr, where)                                                                      \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess) return na_fail(c, LBFD_EDEVICE, std::string(where) + ": " + hipGetErrorString(_e)); \
    } while (0)

}  // namespace

extern "C" {

lbfd_status lbfd_diagnostics_noalloc(lbfd_ctx* c, lbfd_diag* out) {
    if (!c || !out) return LBFD_EINVAL;
    if (!c->have_fields) return na_fail(c, LBFD_ESTATE, "diagnostics before set_fields");
    NACHK(c, hipSetDevice(c->device), "set device");
    const int64_t nb = diag_blocks(c->dp.N);
    if (nb < 1 || nb > kMaxDiagBlocks)
        return na_fail(c, LBFD_EINVAL, "the reduction needs " + std::to_string(nb) +
                                           " partial records; the static scratch holds " +
                                           std::to_string(kMaxDiagBlocks));
    double* s = nullptr;
    NACHK(c, scratch_on(c->device, &s), "scratch address");
    double* part = s;
    double* rec = s + (size_t)kMaxDiagBlocks * kDiagVals;
    NACHK(c, compute_side_fields(c), "side fields");
    NACHK(c, launch_diag_into(c->dp, c->buf, part, rec, c->stream), "diag kernel");
    double r[kDiagVals];
    NACHK(c, hipMemcpyAsync(r, rec, sizeof(r), hipMemcpyDeviceToHost, c->stream), "diag download");
    unsigned f = 0;
    NACHK(c, read_flags(c, &f), "read flags");  // synchronises the stream
    c->flags_seen |= f;
    fill_diag(c, r, out);
    return LBFD_OK;
}

}  // extern "C"

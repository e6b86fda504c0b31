// lbfd_ctx.h -- the lattice context shared by the single-lattice and batched host code
// of liblbfd.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "lbfd.h"
#include "lbfd_internal.h"

struct lbfd_ctx {
    lbfd_grid grid;
    lbfd_params params;
    double ub[3], ut[3];
    lbfd::DevParams dp;
    lbfd::Buffers buf;
    lbfd::Tuning tune;
    float* hbuf[2];
    float* Dbuf[2];
    float* mbuf[2];    // moments of two levels (the chained step reads one, writes the other)
    float* abuf[2];    // FENE-P rate history, abuf[cur] read and abuf[1 - cur] written by a step
    int cur;
    int mcur;          // mbuf[mcur] holds the moments of the current level when mom_valid
    bool mom_valid;
    bool ab_valid;     // buf.ab holds the FENE-P rate of the previous step (Cholesky AB2)
    hipStream_t stream;
    int device;
    char* dev;
    uint64_t bytes;
    int64_t steps;
    unsigned flags_seen;
    bool have_fields;
    std::string err;
};

namespace lbfd {
hipError_t compute_side_fields(lbfd_ctx* c);
hipError_t ensure_moments(lbfd_ctx* c);
int auto_zchunk(const lbfd_grid& g, int tile);
hipError_t enqueue_steps(lbfd_ctx* c, int64_t n);
// whether a launch path implements the lattice's collision and FENE-P options, and the
// path a step takes (the tuned one, or the split path when the tuned one lacks an option)
bool path_supports(const lbfd_ctx* c, int path);
int step_path(const lbfd_ctx* c);
hipError_t read_flags(lbfd_ctx* c, unsigned* out);
// the public record from the kDiagVals FP64 sums of the diagnostics kernels (D and theta
// from the x-y block of the central second moments)
void fill_diag(const lbfd_ctx* c, const double* r, lbfd_diag* out);
void bind_current(lbfd_ctx* c);
}  // namespace lbfd

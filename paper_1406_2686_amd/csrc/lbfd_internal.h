// lbfd_internal.h -- device-side parameter block, buffer set and kernel launchers
// shared by the host API translation units of liblbfd.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfd {

// Scalars every kernel needs, pre-converted to FP32 where the kernels compute in FP32.
struct DevParams {
    int nx, ny, nz, nc;
    int64_t N;         // nx*ny*nz
    float tauA, tauB;  // BGK times of the A-rich / B-rich phases
    float G;           // Shan-Chen coupling
    float inv_delta;   // 1/Delta of f+-(phi)
    float rho0[2];     // storage shift per component
    int phase;         // polymer phase (LBFD_POLYMER_*)
    float pstress;     // eta_p/tau_p (0 when there is no feedback)
    float inv_tau_p;   // 1/tau_p
    float L2;          // L^2
    float L2m3;        // L^2 - 3
    float ub[3], ut[3];
    int coupling;      // LBFD_COUPLING_* (0: body force, 1: stress in the equilibrium)
    int collision;     // LBFD_COLLISION_* (0: BGK, 1: MRT; the split path only)
    int fene;          // LBFD_FENE_* (0: upwind Euler, 1: Cholesky AB2; the split path only)
    int ab_hist;       // Cholesky AB2: the history buffer holds the previous rate
    float kappa;       // Cholesky AB2: artificial diffusivity
    int pad_;
};

// Views into the caller-owned device buffer.
struct Buffers {
    float* h;          // populations (f - w rho0) at time n: [nc][19][N]
    float* hn;         // populations at n+1
    float* D;          // C - I at time n: [6][N]
    float* Dn;         // C - I at n+1
    float* mom;        // side field: [nc+3][N] = delta rho_A, (delta rho_B), j_x, j_y, j_z (level n)
    float* mom_next;   // the same at level n+1, written by the chained step
    float* uF;         // side field: [3+3nc][N] = u (half-force), F_A, (F_B)
    float* ab;         // Cholesky AB2 history: [6][N] rate of (ln l11, l21, ln l22, l31, l32, ln l33) at n-1
    float* ab_next;    // the rate at n, written by the step (so a trial step leaves the state intact)
    double* stage;     // FP64 staging for host transfers: 11 x stage_nodes
    int64_t stage_nodes;
    double* red;       // reduction partials
    int64_t red_blocks;
    double* red_out;   // final reduction record
    unsigned* flags;   // fault bits (LBFD_FLAG_*), accumulated with atomicOr
};

// Sub-box of the lattice (global coordinates, x fastest in the flattened box).
struct Box {
    int x0, y0, z0, bx, by, bz;
};

// Launch shape of the fused step: tile 0 = 32x8, 1 = 32x16 (runs as 32x8), 2 = 16x16 (x by y
// nodes per workgroup); zchunk = planes per workgroup along z (0 = all).  path 0 = fused single
// pass, 1 = three-pass split (moments, forces, collide).
struct Tuning {
    int path;
    int tile;
    int zchunk;
};

constexpr int kDiagVals = 20;        // per-block FP64 reduction record length
constexpr int kMaxDiagBlocks = 1024;  // stage-1 workgroups of the diagnostics (grid-stride beyond)

// One lattice of a batch, as the batched step kernel sees it (device memory).
struct BatchInstance {
    DevParams p;
    float* h[2];       // the two population buffers
    float* D[2];       // the two C - I buffers
    float* mom[2];     // the two moments buffers (chained batch step; same parity as h and D)
    float* ab[2];      // the two FENE-P rate-history buffers (Cholesky integrator; same parity)
    unsigned* flags;   // this instance's fault bits
    int cur;           // buffer index holding time level n when the launch parity is 0
    int pad;
};

// One workgroup of a batched step: instance, tile origin, z range [z0, z1).
struct WorkItem {
    int inst, x0, y0, z0, z1, pad0, pad1, pad2;
};

// kernels of one time step (k_step.hip)
hipError_t launch_moments(const DevParams& p, const Buffers& b, hipStream_t s);
hipError_t launch_forces(const DevParams& p, const Buffers& b, hipStream_t s);
hipError_t launch_collide(const DevParams& p, const Buffers& b, hipStream_t s);
hipError_t launch_clear_flags(const Buffers& b, hipStream_t s);
// prescribed-velocity FENE-P step: D -> Dn (and the rate history ab -> abn) with the velocity
// field uF[0..2] held fixed; no lattice-Boltzmann part
hipError_t launch_fenep_kinematic(const DevParams& p, const float* uF, const float* D, float* Dn, const float* ab,
                                  float* abn, unsigned* flags, hipStream_t s);
hipError_t launch_set_flags(const Buffers& b, unsigned v, hipStream_t s);
// the fused single-pass step (k_fused.hip)
hipError_t launch_fused(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s);
// second pass of the two-pass step (after launch_moments over the same time level)
hipError_t launch_fused2(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s);
// chained two-pass step: launch_fused2's work plus the moments of level n+1 (b.mom -> b.mom_next)
hipError_t launch_fused3(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s);
hipError_t launch_fused_batch(const BatchInstance* inst, const WorkItem* work, int64_t nwork, int ncomp, int tile,
                              int parity, hipStream_t s);
// chained step over a work table of tx-wide tiles, tx 64 (64x8) or 32 (32x16) (moments of
// level n in mom[cur ^ parity]); fene, collision: the options every instance of the batch
// shares (DevParams::fene, ::collision)
hipError_t launch_fused3_batch(const BatchInstance* inst, const WorkItem* work, int64_t nwork, int ncomp, int fene,
                               int collision, int tx, int parity, hipStream_t s);
void chained_batch_tile_shape(int tile, int* tx, int* ty);
void fused_tile_shape(int ncomp, int tile, int* tx, int* ty);

// field transfer kernels (k_fields.hip)
hipError_t launch_init_box(const DevParams& p, const Buffers& b, const Box& box, hipStream_t s);
hipError_t launch_fields_box(const DevParams& p, const Buffers& b, const Box& box, hipStream_t s);

// diagnostics (k_diag.hip): writes kDiagVals doubles to b.red_out
hipError_t launch_diag(const DevParams& p, const Buffers& b, hipStream_t s);
// the same with the diag_blocks(N) stage-1 records in `part` and the final record in `out`
hipError_t launch_diag_into(const DevParams& p, const Buffers& b, double* part, double* out, hipStream_t s);
int64_t diag_blocks(int64_t N);

}  // namespace lbfd

/*
 * lbfd.h -- C ABI of the MI355X (gfx950) library for the hybrid lattice-Boltzmann /
 * finite-difference step of Gupta, Sbragaglia & Scagliarini, arXiv:1406.2686:
 * two Shan-Chen components on a D3Q19 lattice (interaction force, BGK collision with
 * forcing, streaming, moving-wall bounce-back) coupled to a finite-difference FENE-P
 * conformation tensor whose stress divergence is fed back as a body force.
 *
 * Conventions (all calls):
 *  - Every call returns lbfd_status; 0 is success.  No C++ exception crosses the ABI.
 *    lbfd_last_error() returns a context-owned, NUL-terminated description of the last
 *    failure (valid until the next call on that context).
 *  - Geometry: x and z periodic; y is wall-normal with half-way walls at y = -1/2 and
 *    y = ny - 1/2 (Sec. 3.1 and Sec. 4.1 set-ups: walls moving in x, periodic in x and z).
 *  - Host field layout: FP64 structure-of-arrays [field][z][y][x], x fastest.  Symmetric
 *    tensors are stored as 6 components (xx, yy, zz, xy, xz, yz).
 *  - Device memory is caller-owned: the caller allocates one device buffer of
 *    lbfd_state_bytes() bytes (256-byte aligned) and passes it to lbfd_create.  The
 *    library never allocates or frees device memory; it keeps populations, conformation
 *    tensor, side fields, staging and reduction scratch inside that buffer.
 *  - All device work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*, NULL = the null stream).  Calls that return host data synchronise it.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Device arithmetic is FP32 (populations stored as deviations f - w_a rho0_s, the
 *    conformation tensor as C - I); diagnostics reduce in FP64.
 */
#ifndef LBFD_H
#define LBFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbfd_status;
#define LBFD_OK 0
#define LBFD_EINVAL 1          /* invalid argument or parameter set                      */
#define LBFD_ENOMEM 2          /* device buffer too small                                */
#define LBFD_EDEVICE 3         /* HIP runtime error (message in lbfd_last_error)         */
#define LBFD_ENONFINITE 4      /* a population or C component became NaN/Inf             */
#define LBFD_EEXTENSIBILITY 5  /* tr C reached L^2 (FENE-P spring diverges)              */
#define LBFD_ENOTSPD 6         /* C lost positive definiteness (a leading minor <= 0)    */
#define LBFD_ESTATE 7          /* call out of order (e.g. step before set_fields)        */

/* fault bits reported in lbfd_diag.flags and folded into the step status */
#define LBFD_FLAG_NONFINITE 1u
#define LBFD_FLAG_EXTENSIBILITY 2u
#define LBFD_FLAG_NOT_SPD 4u

/* which phase carries the polymer feedback (modulation m(phi) of Sec. 2, Yue et al. form) */
#define LBFD_POLYMER_NONE 0 /* C evolves, no feedback into the fluid   */
#define LBFD_POLYMER_A 1    /* m = f+(phi) = (1 + tanh(phi/Delta))/2   */
#define LBFD_POLYMER_B 2    /* m = f-(phi) = (1 - tanh(phi/Delta))/2   */
#define LBFD_POLYMER_ALL 3  /* m = 1                                    */

/* how the polymer stress T = (eta_p/tau_p) m(phi) (f(r) C - I) acts on the fluid */
#define LBFD_COUPLING_FORCE 0  /* body force div T (central differences), split between the
                                  species by rho_s/rho (Sec. 2, eq. NS); the default        */
#define LBFD_COUPLING_STRESS 1 /* T_s = (rho_s/rho) T lowers the second moment of each
                                  species' equilibrium (Sec. 2, eq. MODEtransformation):
                                  E_a -= 4.5 w_a (c_a.T_s.c_a - tr T_s / 3); no body force  */

typedef struct lbfd_ctx lbfd_ctx;

typedef struct {
    int32_t nx, ny, nz; /* lattice nodes; ny >= 3 (wall-normal), nx, nz >= 1, and      */
                        /* nx*ny*nz < 2^30 (a field's byte offsets fit in 32 bits)     */
    int32_t ncomp;      /* 1 or 2 Shan-Chen components (A, B)                          */
} lbfd_grid;

typedef struct {
    double tau_A, tau_B;   /* BGK relaxation time in A-rich / B-rich regions (> 1/2);   */
                           /* local tau = tau_B + (tau_A - tau_B) f+(phi)              */
    double G;              /* Shan-Chen coupling (Sec. 2, eq. SCforce)                  */
    double delta;          /* smoothing width of f+-(phi) (Sec. 2, eq. smoothingvisco)  */
    double rho0[2];        /* storage shift per component (populations kept as f - w rho0) */
    int32_t polymer_phase; /* LBFD_POLYMER_*                                           */
    int32_t coupling;      /* LBFD_COUPLING_*; any other value is EINVAL               */
    double eta_p;          /* polymer viscosity (Sec. 2, eq. NS)                        */
    double tau_p;          /* polymer relaxation time in lattice steps (> 0)            */
    double L2;             /* FENE-P maximum extension squared (> 3)                    */
    int32_t collision;     /* LBFD_COLLISION_*; any other value is EINVAL              */
    int32_t fene_scheme;   /* LBFD_FENE_*; any other value is EINVAL                    */
    double fene_kappa;     /* artificial diffusivity of LBFD_FENE_CHOLESKY_AB2 (>= 0)    */
} lbfd_params;

/* FENE-P integrator.  UPWIND_EULER (default): C itself, first-order upwind advection,
 * forward Euler (reading of the paper's integrator).  CHOLESKY_AB2: the paper's integrator
 * (Sec. 2, paragraph on the FENE-P solver): sigma_P = f C = L L^t advanced through its
 * Cholesky factor with ln l_ii in place of l_ii, so that C stays symmetric positive
 * definite with tr C < L^2 by construction; second-order central differences in space,
 * the artificial diffusivity fene_kappa * lap C, second-order Adams-Bashforth in time
 * (forward Euler for the first step after set_fields).  Runs on the chained and split
 * paths (a lattice tuned to the fused or two-pass path steps on the split path, and
 * lbfd_get_tuning reports it).  Batches run it in the chained batch body; there an
 * instance's first step after its fields are set is a forward Euler step, as for a single
 * lattice. */
#define LBFD_FENE_UPWIND_EULER 0
#define LBFD_FENE_CHOLESKY_AB2 1

/* Collision operator.  BGK: one relaxation time, the local tau (reading of the paper's
 * collision at unit rates).  MRT: the multiple-relaxation-time collision of Sec. 2 in an
 * orthogonal D3Q19 moment basis: the bulk and shear modes relax with the local tau
 * (tau_s = tau_b), the species momenta with tau_M = 1, the other modes with rate 1, and
 * the source is weighted by I - Lambda/2 in moment space (eq. TRANSPORTCOEFF and the text
 * after it).  MRT runs on the chained and split paths (a lattice tuned to the fused or
 * two-pass path steps on the split path, and lbfd_get_tuning reports it).  Batches run it
 * in the chained batch body.  All instances of a batch share the collision and FENE-P
 * options (EINVAL otherwise, and with a non-default option on the fused batch path). */
#define LBFD_COLLISION_BGK 0
#define LBFD_COLLISION_MRT 1

/* FP64 diagnostics of the current state (droplet shape per Sec. 4.1: D = (a-b)/(a+b),
 * theta = angle of the major axis with the flow direction x, from the x-y block of the
 * second moments of w = max(phi, 0)). */
typedef struct {
    double mass[2];         /* sum of rho per component                               */
    double momentum[3];     /* sum of rho u (u with the half-force shift)             */
    double W;               /* sum of w                                               */
    double centroid[3];     /* sum(w x)/W                                             */
    double M[6];            /* second moments about the centroid / W (xx,yy,zz,xy,xz,yz) */
    double D;               /* deformation parameter                                  */
    double theta_deg;       /* orientation in degrees                                 */
    double min_L2_minus_trC;
    double min_minor;       /* smallest leading principal minor of C                  */
    double max_u;           /* max |u|                                                */
    uint32_t flags;         /* LBFD_FLAG_* seen since the last lbfd_set_fields         */
    uint32_t reserved;
    int64_t step;           /* steps taken since lbfd_set_fields                       */
    double poly_trace_excess; /* mean of tr C - 3 over the polymer phase, weighted by the
                               * feedback modulation m(phi); 0 without a polymer phase */
} lbfd_diag;

/* Device bytes needed for a grid (populations x2, C x2, side fields, staging, scratch).
 * EINVAL for an invalid grid. */
lbfd_status lbfd_state_bytes(const lbfd_grid* grid, uint64_t* bytes);

/* Create a context bound to a caller-owned device buffer `dev_state` of `bytes` bytes
 * on the current HIP device and to `hip_stream`.  Validates the grid and the
 * parameters (EINVAL) and the buffer size (ENOMEM).  *out is NULL on failure. */
lbfd_status lbfd_create(const lbfd_grid* grid, const lbfd_params* params, void* dev_state,
                        uint64_t bytes, void* hip_stream, lbfd_ctx** out);

/* Replace the parameter set (same validation as create).  Takes effect at the next step. */
lbfd_status lbfd_set_params(lbfd_ctx* ctx, const lbfd_params* params);

/* Wall velocities (bottom at y = -1/2, top at y = ny - 1/2).  Only tangential motion:
 * a non-zero y component is EINVAL (Sec. 3.1: walls slide in x). */
lbfd_status lbfd_set_walls(lbfd_ctx* ctx, const double u_bottom[3], const double u_top[3]);

/* Initialise populations to the equilibrium E(rho_s, u) (no non-equilibrium part) and
 * C as given, on the whole grid.  rho: ncomp x N, u: 3 x N, C: 6 x N host arrays.
 * Checks finiteness, positive definiteness and tr C < L^2 on the host (EINVAL).
 * Resets the step counter and the fault flags. */
lbfd_status lbfd_set_fields(lbfd_ctx* ctx, const double* rho, const double* u, const double* C);

/* Same on the sub-box [x0, x0+bx) x [y0, y0+by) x [z0, z0+bz); arrays are ncomp x B,
 * 3 x B, 6 x B with B = bx*by*bz in [z][y][x] order.  Does not reset the counters
 * (call lbfd_reset_counters after the last box). */
lbfd_status lbfd_set_fields_box(lbfd_ctx* ctx, int32_t x0, int32_t y0, int32_t z0, int32_t bx,
                                int32_t by, int32_t bz, const double* rho, const double* u,
                                const double* C);
lbfd_status lbfd_reset_counters(lbfd_ctx* ctx);

/* Advance nsteps >= 0 time steps.  Returns ENONFINITE / EEXTENSIBILITY / ENOTSPD (in
 * that priority) if the device fault flags were raised during this call; the state
 * then holds the result of all nsteps steps and is not repaired. */
lbfd_status lbfd_step(lbfd_ctx* ctx, int64_t nsteps);

/* Enqueue nsteps steps without synchronising or reading the fault flags (for timing
 * and graph capture).  Fault flags accumulate and are reported by the next
 * lbfd_step / lbfd_diagnostics / lbfd_get_flags. */
lbfd_status lbfd_step_async(lbfd_ctx* ctx, int64_t nsteps);
lbfd_status lbfd_get_flags(lbfd_ctx* ctx, uint32_t* flags);

/* Prescribed-velocity ("kinematic") FENE-P stepping for the homogeneous rheology benchmarks
 * of Sec. 3 (steady shear 3.1, uniaxial elongation 3.2, small-amplitude oscillatory shear
 * 3.3, inception and cessation 3.4), where the flow is imposed and the polymer does not act
 * back on it: the velocity is held at the host field u (3 x N, FP64, converted to FP32) and
 * only the FENE-P update of C (eq. FENE with the lattice's fene_scheme, fene_kappa, L2 and
 * tau_p; velocity gradients by central differences with wall ghosts 2 u_w - u from
 * lbfd_set_walls; C ghosts by linear extrapolation) runs nsteps >= 0 times.  The
 * lattice-Boltzmann populations are not advanced, the step counter does not move, and
 * fields read afterwards report the velocity of the populations, not u.  The Cholesky-log
 * integrator carries its Adams-Bashforth history across calls (forward Euler first after
 * set_fields).  Returns the first fault as lbfd_step; EINVAL for a non-finite u, ESTATE
 * before set_fields. */
lbfd_status lbfd_fenep_kinematic(lbfd_ctx* ctx, const double* u, int64_t nsteps);

/* Macroscopic fields of the current state: rho (ncomp x N), u (3 x N, including the
 * half-force shift of Sec. 2, eq. equilibrium:vel) and C (6 x N).  Any pointer may be
 * NULL.  Synchronises the stream. */
lbfd_status lbfd_get_fields(lbfd_ctx* ctx, double* rho, double* u, double* C);
lbfd_status lbfd_get_fields_box(lbfd_ctx* ctx, int32_t x0, int32_t y0, int32_t z0, int32_t bx,
                                int32_t by, int32_t bz, double* rho, double* u, double* C);

/* FP64 diagnostics record of the current state, on demand (there is no diagnostics cadence
 * in lbfd_params: a caller steps in chunks and calls this between them; the batch's steady
 * test carries its own cadence in lbfd_steady_crit).  Synchronises the stream. */
lbfd_status lbfd_diagnostics(lbfd_ctx* ctx, lbfd_diag* out);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * monitoring loops, harnesses that forbid hipMalloc): the record of lbfd_diagnostics,
 * computed by the same kernels in the same order (so the two records are identical), with
 * the reduction's partial records kept in a static per-device array of 164,000 bytes (at
 * most 1024 stage-1 records of 20 FP64 values plus the final record) instead of the
 * context's buffer.  Calls no allocating routine.  The array is shared by every call on
 * one GPU: calls that overlap on one GPU (different streams or threads) race and must be
 * serialised by the caller.  EINVAL if the reduction would need more partial records
 * than the array holds (not reachable for valid grids: the first stage is capped at 1024
 * workgroups), ESTATE before set_fields, EDEVICE on a HIP error.  Synchronises the stream. */
lbfd_status lbfd_diagnostics_noalloc(lbfd_ctx* ctx, lbfd_diag* out);

/* Raw checkpoint of the device state (FP32 populations, C - I and the moments delta rho, j
 * of the current level, step counter, flags): lbfd_checkpoint_bytes gives the size; get
 * copies device -> host, set host -> device.  A run restarted from a checkpoint continues
 * bitwise like the run that wrote it, on every path. */
lbfd_status lbfd_checkpoint_bytes(lbfd_ctx* ctx, uint64_t* bytes);
lbfd_status lbfd_get_state(lbfd_ctx* ctx, void* host, uint64_t bytes);
lbfd_status lbfd_set_state(lbfd_ctx* ctx, const void* host, uint64_t bytes);

/* Launch shape of the step.  path: LBFD_PATH_FUSED (one pass over HBM per step),
 * LBFD_PATH_TWOPASS (a streaming moments pass, then one pass that reads the moments and C
 * with their halos and only the tile's own populations), LBFD_PATH_CHAINED (the default:
 * the two-pass step whose second pass also forms the moments of the next level, so that a
 * run of steps needs one launch per step and the moments pass runs only when the moments
 * of the current level are not at hand: after set_fields, another path or a batch; 64x8
 * tiles whatever `tile` says) or LBFD_PATH_SPLIT (three passes: moments, forces, collide;
 * kept as a cross-check).  The paths compute the same step; their results agree to FP32
 * rounding.  A path that does not implement the lattice's collision or FENE-P option is
 * replaced by the split path for the steps (see LBFD_COLLISION_MRT, LBFD_FENE_CHOLESKY_AB2);
 * lbfd_get_tuning reports the path the steps take.  tile: LBFD_TILE_32x8 / 32x16 / 16x16 (x by y nodes per workgroup of the fused
 * and two-pass steps; 32x16 runs as 32x8).  zchunk: planes per workgroup along z, 0 =
 * automatic.  Within one path, results are identical for every tile and zchunk; only speed
 * changes. */
#define LBFD_PATH_FUSED 0
#define LBFD_PATH_SPLIT 1
#define LBFD_PATH_TWOPASS 2
#define LBFD_PATH_CHAINED 3
#define LBFD_TILE_32x8 0
#define LBFD_TILE_32x16 1
#define LBFD_TILE_16x16 2
#define LBFD_TILE_64x8 3   /* two-pass and chained steps only (one 64-lane row per wavefront);
                              the fused and split steps and fused batches run it as 32x8 */
typedef struct {
    int32_t path;
    int32_t tile;
    int32_t zchunk;
    int32_t reserved;
} lbfd_tuning;
lbfd_status lbfd_set_tuning(lbfd_ctx* ctx, const lbfd_tuning* t);
lbfd_status lbfd_get_tuning(lbfd_ctx* ctx, lbfd_tuning* t);

/* Launch-shape autotuner (single lattice): times the chained, two-pass and fused steps that
 * implement the lattice's options (the split step when none does) for every tile shape
 * they take and a range of z-chunks on the current state, `reps` launches each, and keeps
 * the fastest
 * (also returned in *best with its time in *ms_per_step; either may be NULL).  The trial
 * launches recompute the next time level from the current one without advancing, so the
 * lattice state, step counter and fault flags are unchanged.  ESTATE before set_fields. */
lbfd_status lbfd_autotune(lbfd_ctx* ctx, int32_t reps, lbfd_tuning* best, double* ms_per_step);

/* ---------------------------------------------------------------------------------
 * Batches: n independent lattices (same ncomp, any sizes) stepped together by one launch
 * per step over a shared work table, replayed from a captured two-step hipGraph when the
 * stream is not the null stream.  Used for parameter sweeps of droplets in shear.
 * Device memory is one caller-owned buffer of lbfd_batch_state_bytes() bytes.
 * --------------------------------------------------------------------------------- */
typedef struct lbfd_batch lbfd_batch;

/* Steady test: D (Sec. 4.1 deformation) is sampled every `every` steps (even); an instance
 * is steady when |D(t - j window) - D(t - (j + 1) window)| < tol for j = 0 .. windows - 1
 * (window a multiple of every; windows 0 counts as 1).  With one window the test is also
 * met where D(t) passes through a slow extremum or plateau of a transient; two consecutive
 * windows rule most of those out. */
typedef struct {
    int32_t every;
    int32_t window;
    double tol;
    int32_t windows;
    int32_t reserved;   /* 0 */
} lbfd_steady_crit;

/* Wall velocities of one batch instance (as lbfd_set_walls). */
typedef struct {
    double u_bottom[3];
    double u_top[3];
} lbfd_walls;

lbfd_status lbfd_batch_state_bytes(int32_t n, const lbfd_grid* grids, uint64_t* bytes);
/* params, walls: n entries each. */
lbfd_status lbfd_batch_create(int32_t n, const lbfd_grid* grids, const lbfd_params* params, const lbfd_walls* walls,
                              void* dev_state, uint64_t bytes, void* hip_stream, lbfd_batch** out);
/* Fields of instance i, as lbfd_set_fields. */
lbfd_status lbfd_batch_set_fields(lbfd_batch* b, int32_t i, const double* rho, const double* u, const double* C);
/* path LBFD_PATH_FUSED (the single-pass body; tile and zchunk as for a single lattice,
 * zchunk >= 4 in a batch) or LBFD_PATH_CHAINED (the chained body: each instance's moments
 * are carried from step to step; they are formed by the moments pass, or copied between
 * its two moments buffers, when an instance has none at its current level; tile
 * LBFD_TILE_32x16 runs 32x16 tiles, for lattices 32 or 96 nodes wide, every other tile
 * value 64x8).  A new batch runs the chained body, on 32x16 tiles when its instances would
 * leave 64x8 tiles emptier by a tenth of the lanes or more, else on 64x8.  Results of the two paths agree to FP32 rounding; within a path they do not
 * depend on the other instances or on tile and zchunk. */
lbfd_status lbfd_batch_set_tuning(lbfd_batch* b, const lbfd_tuning* t);
lbfd_status lbfd_batch_get_tuning(lbfd_batch* b, lbfd_tuning* t);
/* Instances with active[i] == 0 are skipped by lbfd_batch_step (n bytes). */
lbfd_status lbfd_batch_set_active(lbfd_batch* b, const uint8_t* active);
/* Advance every active instance by nsteps; fault status as lbfd_step (any instance). */
lbfd_status lbfd_batch_step(lbfd_batch* b, int64_t nsteps);
/* Diagnostics of all n instances (out: n records). */
lbfd_status lbfd_batch_diagnostics(lbfd_batch* b, lbfd_diag* out);
lbfd_status lbfd_batch_get_fields(lbfd_batch* b, int32_t i, double* rho, double* u, double* C);
/* Run all instances until each is steady (then retired from the launches) or max_steps.
 * out: final diagnostics per instance; steady_step[i]: step at which instance i met the
 * test, -1 if it did not, -2 if it raised a fault flag (it is then retired and its flags
 * are in out[i].flags).  Re-activates every instance before returning. */
lbfd_status lbfd_batch_run_to_steady(lbfd_batch* b, const lbfd_steady_crit* crit, int64_t max_steps,
                                     lbfd_diag* out, int64_t* steady_step);
/* Progress report of lbfd_batch_run_to_steady: after each chunk of `every` steps it calls
 * fn(steps taken, instances still stepping, user) on the calling thread (fn NULL: none).
 * fn must not call into the batch. */
typedef void (*lbfd_progress_fn)(int64_t step, int32_t active, void* user);
lbfd_status lbfd_batch_set_progress(lbfd_batch* b, lbfd_progress_fn fn, void* user);
/* Launch-shape autotuner for the batch: both paths, their tiles and a range of z-chunks
 * (state unchanged, as lbfd_autotune). */
lbfd_status lbfd_batch_autotune(lbfd_batch* b, int32_t reps, lbfd_tuning* best, double* ms_per_step);
/* The context of instance i (owned by the batch; valid until lbfd_batch_destroy). */
lbfd_ctx* lbfd_batch_instance(lbfd_batch* b, int32_t i);
void lbfd_batch_destroy(lbfd_batch* b);
const char* lbfd_batch_last_error(const lbfd_batch* b);

/* ---------------------------------------------------------------------------------
 * Surrogate network for droplet sweeps: an MLP 5 -> 128 -> 128 -> 3 with GELU
 * (GELU(z) = z (1 + erf(z / sqrt 2)) / 2) mapping (Ca, De, viscosity ratio, 2R/H, log L^2),
 * standardised by the caller, to standardised (D, theta, warm-start C amplitude).  Training
 * in FP32 on the device (mean-squared-error loss, Adam), inference in BF16 with FP32
 * accumulation on the matrix cores.  The lattice solver stays the reference: the network
 * only proposes warm starts and its error is judged against solver runs.
 * Parameter vector (FP32, LBFD_MLP_NPARAMS values in this order): W1[128][5], b1[128],
 * W2[128][128], b2[128], W3[3][128], b3[3]; row-major, y = W x + b.
 * All X / T / Y arrays here are host arrays, row-major [sample][feature].
 * --------------------------------------------------------------------------------- */
#define LBFD_MLP_IN 5
#define LBFD_MLP_HIDDEN 128
#define LBFD_MLP_OUT 3
#define LBFD_MLP_NPARAMS 17667

typedef struct lbfd_mlp lbfd_mlp;
typedef struct {
    int32_t epochs;  /* passes over the training set                        */
    int32_t batch;   /* minibatch size (<= max_batch)                        */
    float lr;        /* Adam step size                                       */
    float beta1, beta2, eps;
    uint64_t seed;   /* shuffling seed                                       */
} lbfd_train_opts;

/* Device bytes for a network with minibatches up to max_batch samples and a resident
 * training set of up to max_train samples. */
lbfd_status lbfd_mlp_state_bytes(int32_t max_batch, int32_t max_train, uint64_t* bytes);
/* Create in a caller-owned device buffer; weights Glorot-uniform from `seed`, biases 0. */
lbfd_status lbfd_mlp_create(int32_t max_batch, int32_t max_train, uint64_t seed, void* dev_state, uint64_t bytes,
                            void* hip_stream, lbfd_mlp** out);
/* Replace / read the LBFD_MLP_NPARAMS parameters (set also resets the Adam moments). */
lbfd_status lbfd_mlp_set_params(lbfd_mlp* m, const float* params);
lbfd_status lbfd_mlp_get_params(lbfd_mlp* m, float* params);
/* FP32 forward pass, n samples (chunked by max_batch). */
lbfd_status lbfd_mlp_forward(lbfd_mlp* m, const float* X, int32_t n, float* Y);
/* Mean-squared-error loss over n x 3 outputs (n <= max_batch) and its gradient with respect
 * to every parameter (grad: LBFD_MLP_NPARAMS floats, may be NULL; loss may be NULL). */
lbfd_status lbfd_mlp_loss_grad(lbfd_mlp* m, const float* X, const float* T, int32_t n, float* loss, float* grad);
/* One Adam update with the gradient of the last lbfd_mlp_loss_grad (bias-corrected). */
lbfd_status lbfd_mlp_adam_step(lbfd_mlp* m, const lbfd_train_opts* opts);
/* Minibatch Adam training on the device over n samples (n <= max_train); returns the loss
 * of the last minibatch. */
lbfd_status lbfd_mlp_train(lbfd_mlp* m, const float* X, const float* T, int32_t n, const lbfd_train_opts* opts,
                           float* final_loss);
/* BF16 inference (weights rounded to BF16 once after each update); the inference call of
 * the surrogate (named for its arithmetic, since lbfd_mlp_forward is the FP32 forward pass). */
lbfd_status lbfd_mlp_infer_bf16(lbfd_mlp* m, const float* X, int32_t n, float* Y);
void lbfd_mlp_destroy(lbfd_mlp* m);
const char* lbfd_mlp_last_error(const lbfd_mlp* m);

/* ---------------------------------------------------------------------------------
 * Streaming-bandwidth probe: the read, write and copy rates a plain streaming kernel reaches
 * on the current device, the ceiling against which the step's traffic is judged (every
 * lane moves 16-byte vectors; grid-stride loops at 8 waves per SIMD).  kind: one of the
 * LBFD_PROBE_*; src and dst are caller-owned device buffers of `bytes` bytes (a multiple
 * of 16, 16-byte aligned; src unused by the write kinds, dst by the read kind).  Runs one
 * warm-up launch, then times `reps` launches with HIP events on `hip_stream` and returns
 * the mean milliseconds per launch (bytes moved per launch: `bytes` for read and write,
 * 2 x `bytes` for copy).  EINVAL for a bad argument, EDEVICE on a HIP error.
 * Synchronises the stream.
 * --------------------------------------------------------------------------------- */
#define LBFD_PROBE_READ 0
#define LBFD_PROBE_WRITE 1     /* plain stores */
#define LBFD_PROBE_WRITE_NT 2  /* nontemporal (streaming) stores */
#define LBFD_PROBE_COPY 3
#define LBFD_PROBE_COPY_NT 4
lbfd_status lbfd_stream_probe(int32_t kind, void* dev_src, void* dev_dst, uint64_t bytes, int32_t reps,
                              void* hip_stream, double* ms_per_launch);

/* Library build/version string (static). */
const char* lbfd_version(void);

void lbfd_destroy(lbfd_ctx* ctx);
const char* lbfd_last_error(const lbfd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBFD_H */

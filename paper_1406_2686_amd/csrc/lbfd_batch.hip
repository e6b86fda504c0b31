// lbfd_batch.hip -- many independent lattices stepped by ONE launch per step, a captured
// two-step hipGraph replayed for long runs, a run-to-steady controller that retires
// converged instances, and the launch-shape autotuners (single lattice and batch).
//
// Each instance is an ordinary lbfd_ctx bound to its own slice of the batch's device
// buffer, so fields, diagnostics and checkpoints use the single-lattice code.  The batch
// adds a device instance table (parameters + buffer pointers + parity) and a work table
// with one entry per workgroup: (instance, tile origin, z range).  Workgroups of unequal
// instances share one launch, so small lattices do not leave the GPU idle.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbfd.h"
#include "lbfd_ctx.h"
#include "lbfd_internal.h"

using namespace lbfd;

struct lbfd_batch {
    int n;
    int ncomp;
    std::vector<lbfd_ctx*> inst;
    std::vector<uint8_t> active;
    std::vector<int> cur;  // buffer parity per instance (kept equal to inst[i]->cur)
    BatchInstance* d_inst;
    WorkItem* d_work;
    int64_t max_work;
    int64_t nwork;
    Tuning tune;
    hipStream_t stream;
    int device;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool graph_ok;
    bool tables_dirty;
    lbfd_progress_fn progress = nullptr;  // run_to_steady: called after each chunk of steps
    void* progress_user = nullptr;
    std::string err;
};

namespace {

constexpr uint64_t kAl = 256;
inline uint64_t al(uint64_t v) { return (v + kAl - 1) / kAl * kAl; }

lbfd_status bfail(lbfd_batch* b, lbfd_status st, const std::string& m) {
    if (b) b->err = m;
    return st;
}

#define BCHK(b, expr, where)                                                                  \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) return bfail(b, LBFD_EDEVICE, std::string(where) + ": " + hipGetErrorString(_e)); \
    } while (0)

int64_t work_bound(const lbfd_grid& g) {
    // smallest tile 16x8, z-chunks of at least 4 planes
    return (int64_t)((g.nx + 15) / 16) * ((g.ny + 7) / 8) * ((g.nz + 3) / 4);
}

void release_graph(lbfd_batch* b) {
    if (b->graph_ok) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->graph_ok = false;
    }
}

// Tile extent of the batch's current tuning.
void batch_tile(const lbfd_batch* b, int ncomp, int* tx, int* ty) {
    if (b->tune.path == LBFD_PATH_CHAINED)
        chained_batch_tile_shape(b->tune.tile, tx, ty);
    else
        fused_tile_shape(ncomp, b->tune.tile, tx, ty);
}

// Automatic z-chunk of a batch: the longest of 64, 32, 16 planes that still gives every
// instance together at least six workgroups per CU (short chunks re-read and re-collide
// their boundary planes: on the 255-lattice halved-grid sweep 8 planes take 4.70 ms per
// step, 32 planes 4.09), else 8.
int batch_auto_zchunk(const lbfd_batch* b) {
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
    for (int zc : {64, 32, 16}) {
        int64_t items = 0;
        for (int i = 0; i < b->n; ++i) {
            if (!b->active[i]) continue;
            const lbfd_grid& g = b->inst[i]->grid;
            int tx = 64, ty = 8;
            batch_tile(b, g.ncomp, &tx, &ty);
            items += (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty) * ((g.nz + zc - 1) / zc);
        }
        if (items >= 6 * (int64_t)ncu) return zc;
    }
    return 8;
}

int batch_zchunk(const lbfd_batch* b, const lbfd_grid& g, int auto_zc) {
    return std::max(4, std::min(b->tune.zchunk > 0 ? b->tune.zchunk : auto_zc, g.nz));
}

// Build and upload the instance and work tables for the active instances.
hipError_t upload_tables(lbfd_batch* b) {
    std::vector<BatchInstance> it(b->n);
    for (int i = 0; i < b->n; ++i) {
        lbfd_ctx* c = b->inst[i];
        it[i].p = c->dp;
        it[i].h[0] = c->hbuf[0];
        it[i].h[1] = c->hbuf[1];
        it[i].D[0] = c->Dbuf[0];
        it[i].D[1] = c->Dbuf[1];
        it[i].mom[0] = c->mbuf[0];
        it[i].mom[1] = c->mbuf[1];
        it[i].ab[0] = c->abuf[0];
        it[i].ab[1] = c->abuf[1];
        it[i].p.ab_hist = c->ab_valid ? 1 : 0;
        it[i].flags = c->buf.flags;
        it[i].cur = b->cur[i];
        it[i].pad = 0;
    }
    std::vector<WorkItem> w;
    const int auto_zc = b->tune.zchunk > 0 ? 0 : batch_auto_zchunk(b);
    for (int i = 0; i < b->n; ++i) {
        if (!b->active[i]) continue;
        const lbfd_grid& g = b->inst[i]->grid;
        int tx = 64, ty = 8;
        batch_tile(b, g.ncomp, &tx, &ty);
        const int zc = batch_zchunk(b, g, auto_zc);
        for (int z0 = 0; z0 < g.nz; z0 += zc)
            for (int y0 = 0; y0 < g.ny; y0 += ty)
                for (int x0 = 0; x0 < g.nx; x0 += tx) w.push_back(WorkItem{i, x0, y0, z0, std::min(z0 + zc, g.nz), 0, 0, 0});
    }
    if ((int64_t)w.size() > b->max_work) return hipErrorInvalidValue;
    b->nwork = (int64_t)w.size();
    hipError_t e = hipMemcpyAsync(b->d_inst, it.data(), sizeof(BatchInstance) * it.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !w.empty())
        e = hipMemcpyAsync(b->d_work, w.data(), sizeof(WorkItem) * w.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    b->tables_dirty = false;
    return e;
}

// The collision and FENE-P options of the batch: every instance must share them (one
// kernel instantiation runs them all).  Returns false if they differ.
bool batch_options(const lbfd_batch* b, int* fene, int* collision) {
    *fene = b->inst[0]->dp.fene;
    *collision = b->inst[0]->dp.collision;
    for (int i = 1; i < b->n; ++i)
        if (b->inst[i]->dp.fene != *fene || b->inst[i]->dp.collision != *collision) return false;
    return true;
}

hipError_t launch_batch(lbfd_batch* b, int parity) {
    int fene = 0, coll = 0;
    (void)batch_options(b, &fene, &coll);
    if (b->tune.path == LBFD_PATH_CHAINED) {
        int tx = 64, ty = 8;
        chained_batch_tile_shape(b->tune.tile, &tx, &ty);
        return launch_fused3_batch(b->d_inst, b->d_work, b->nwork, b->ncomp, fene, coll, tx, parity, b->stream);
    }
    return launch_fused_batch(b->d_inst, b->d_work, b->nwork, b->ncomp, b->tune.tile, parity, b->stream);
}

// The chained batch step reads each active instance's moments of the current level from
// mbuf[cur]: carried moments in the other buffer are copied over, missing ones formed by
// the moments pass.
hipError_t align_moments(lbfd_batch* b) {
    if (b->tune.path != LBFD_PATH_CHAINED) return hipSuccess;
    for (int i = 0; i < b->n; ++i) {
        if (!b->active[i]) continue;
        lbfd_ctx* c = b->inst[i];
        if (c->mom_valid && c->mcur == c->cur) continue;
        hipError_t e = hipSuccess;
        if (c->mom_valid) {
            e = hipMemcpyAsync(c->mbuf[c->cur], c->mbuf[c->mcur], (size_t)(c->grid.ncomp + 3) * c->dp.N * 4,
                               hipMemcpyDeviceToDevice, b->stream);
            c->mcur = c->cur;
            bind_current(c);
        } else {
            c->mcur = c->cur;
            bind_current(c);
            e = launch_moments(c->dp, c->buf, b->stream);
            c->mom_valid = true;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Capture [step parity 0, step parity 1] into a graph (non-null streams only).
hipError_t capture(lbfd_batch* b) {
    release_graph(b);
    if (b->stream == nullptr || b->nwork == 0) return hipSuccess;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e1 = launch_batch(b, 0);
    hipError_t e2 = launch_batch(b, 1);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (e1 != hipSuccess) return e1;
    if (e2 != hipSuccess) return e2;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    b->graph = g;
    b->graph_ok = true;
    return hipSuccess;
}

hipError_t ensure_ready(lbfd_batch* b) {
    if (b->tables_dirty) {
        hipError_t e = upload_tables(b);
        if (e != hipSuccess) return e;
        e = capture(b);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// advance the bookkeeping of the active instances by n steps
void advance(lbfd_batch* b, int64_t n) {
    for (int i = 0; i < b->n; ++i) {
        if (!b->active[i]) continue;
        lbfd_ctx* c = b->inst[i];
        c->steps += n;
        if (n & 1) {
            b->cur[i] ^= 1;
            c->cur = b->cur[i];
        }
        if (b->tune.path == LBFD_PATH_CHAINED && n > 0) {
            c->mcur = c->cur;  // the chained step carried the moments along with h and D
            c->mom_valid = true;
        } else if (n > 0) {
            c->mom_valid = false;  // the fused batch step does not carry moments
        }
        if (n > 0) c->ab_valid = c->dp.fene == LBFD_FENE_CHOLESKY_AB2;  // this step's rate was written
        bind_current(c);
    }
}

lbfd_status flags_to_status(unsigned f) {
    if (f & LBFD_FLAG_NONFINITE) return LBFD_ENONFINITE;
    if (f & LBFD_FLAG_EXTENSIBILITY) return LBFD_EEXTENSIBILITY;
    if (f & LBFD_FLAG_NOT_SPD) return LBFD_ENOTSPD;
    return LBFD_OK;
}

}  // namespace

extern "C" {

lbfd_status lbfd_batch_state_bytes(int32_t n, const lbfd_grid* grids, uint64_t* bytes) {
    if (n < 1 || !grids || !bytes) return LBFD_EINVAL;
    uint64_t tot = 0;
    int64_t wb = 0;
    for (int i = 0; i < n; ++i) {
        uint64_t b = 0;
        if (lbfd_state_bytes(&grids[i], &b) != LBFD_OK) return LBFD_EINVAL;
        if (grids[i].ncomp != grids[0].ncomp) return LBFD_EINVAL;
        tot += al(b);
        wb += work_bound(grids[i]);
    }
    tot += al(sizeof(BatchInstance) * (uint64_t)n);
    tot += al(sizeof(WorkItem) * (uint64_t)wb);
    *bytes = tot;
    return LBFD_OK;
}

lbfd_status lbfd_batch_create(int32_t n, const lbfd_grid* grids, const lbfd_params* params, const lbfd_walls* walls,
                              void* dev_state, uint64_t bytes, void* hip_stream, lbfd_batch** out) {
    if (!out) return LBFD_EINVAL;
    *out = nullptr;
    uint64_t need = 0;
    lbfd_status st = lbfd_batch_state_bytes(n, grids, &need);
    if (st != LBFD_OK) return st;
    if (!params || !walls || !dev_state || ((uintptr_t)dev_state % kAl) != 0) return LBFD_EINVAL;
    if (bytes < need) return LBFD_ENOMEM;
    lbfd_batch* b = new (std::nothrow) lbfd_batch();
    if (!b) return LBFD_ENOMEM;
    b->n = n;
    b->ncomp = grids[0].ncomp;
    b->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&b->device);
    // the chained body (4.88 ms per step on the 255-lattice droplet sweep against 5.50 for
    // the fused single-pass body on 32x8 tiles), on 32x16 tiles when the instances leave
    // 64x8 tiles emptier by a tenth of the lanes or more (4.70 against 5.13 ms per step on
    // the same sweep, whose lattices are 32, 64 or 96 nodes wide)
    int64_t lanes64 = 0, lanes32 = 0;
    for (int i = 0; i < n; ++i) {
        const lbfd_grid& g = grids[i];
        lanes64 += (int64_t)((g.nx + 63) / 64 * 64) * ((g.ny + 7) / 8 * 8) * g.nz;
        lanes32 += (int64_t)((g.nx + 31) / 32 * 32) * ((g.ny + 15) / 16 * 16) * g.nz;
    }
    b->tune = Tuning{LBFD_PATH_CHAINED, lanes32 * 11 <= lanes64 * 10 ? LBFD_TILE_32x16 : LBFD_TILE_64x8, 0};
    b->graph_ok = false;
    b->tables_dirty = true;
    char* p = (char*)dev_state;
    int64_t wb = 0;
    for (int i = 0; i < n; ++i) {
        uint64_t sb = 0;
        lbfd_state_bytes(&grids[i], &sb);
        lbfd_ctx* c = nullptr;
        st = lbfd_create(&grids[i], &params[i], p, sb, hip_stream, &c);
        if (st == LBFD_OK) st = lbfd_set_walls(c, walls[i].u_bottom, walls[i].u_top);
        if (st != LBFD_OK) {
            if (c) lbfd_destroy(c);
            for (lbfd_ctx* q : b->inst) lbfd_destroy(q);
            delete b;
            return st;
        }
        b->inst.push_back(c);
        b->active.push_back(1);
        b->cur.push_back(0);
        p += al(sb);
        wb += work_bound(grids[i]);
    }
    b->d_inst = (BatchInstance*)p;
    p += al(sizeof(BatchInstance) * (uint64_t)n);
    b->d_work = (WorkItem*)p;
    b->max_work = wb;
    b->nwork = 0;
    *out = b;
    return LBFD_OK;
}

lbfd_status lbfd_batch_set_fields(lbfd_batch* b, int32_t i, const double* rho, const double* u, const double* C) {
    if (!b || i < 0 || i >= b->n) return LBFD_EINVAL;
    lbfd_status st = lbfd_set_fields(b->inst[i], rho, u, C);
    if (st != LBFD_OK) return bfail(b, st, lbfd_last_error(b->inst[i]));
    b->cur[i] = b->inst[i]->cur;
    b->tables_dirty = true;
    return LBFD_OK;
}

lbfd_status lbfd_batch_set_tuning(lbfd_batch* b, const lbfd_tuning* t) {
    if (!b || !t) return LBFD_EINVAL;
    if (t->path != LBFD_PATH_FUSED && t->path != LBFD_PATH_CHAINED)
        return bfail(b, LBFD_EINVAL, "the batch runs the fused or the chained path");
    if (t->tile < LBFD_TILE_32x8 || t->tile > LBFD_TILE_64x8 || t->zchunk < 0) return bfail(b, LBFD_EINVAL, "bad tuning");
    b->tune = Tuning{t->path, t->tile, t->zchunk};
    b->tables_dirty = true;
    return LBFD_OK;
}

lbfd_status lbfd_batch_get_tuning(lbfd_batch* b, lbfd_tuning* t) {
    if (!b || !t) return LBFD_EINVAL;
    t->path = b->tune.path;
    t->tile = b->tune.tile;
    t->zchunk = b->tune.zchunk;
    t->reserved = 0;
    return LBFD_OK;
}

lbfd_status lbfd_batch_set_active(lbfd_batch* b, const uint8_t* active) {
    if (!b || !active) return LBFD_EINVAL;
    for (int i = 0; i < b->n; ++i) b->active[i] = active[i] ? 1 : 0;
    b->tables_dirty = true;
    return LBFD_OK;
}

lbfd_status lbfd_batch_step(lbfd_batch* b, int64_t nsteps) {
    if (!b || nsteps < 0) return LBFD_EINVAL;
    for (int i = 0; i < b->n; ++i)
        if (b->active[i] && !b->inst[i]->have_fields) return bfail(b, LBFD_ESTATE, "instance without fields");
    int fene = 0, coll = 0;
    if (!batch_options(b, &fene, &coll))
        return bfail(b, LBFD_EINVAL, "the instances of a batch must share the collision and FENE-P options");
    if ((fene != LBFD_FENE_UPWIND_EULER || coll != LBFD_COLLISION_BGK) && b->tune.path != LBFD_PATH_CHAINED)
        return bfail(b, LBFD_EINVAL, "the MRT collision and the Cholesky integrator run in the chained batch body");
    (void)hipSetDevice(b->device);
    BCHK(b, ensure_ready(b), "batch tables");
    BCHK(b, align_moments(b), "batch moments");
    int64_t done = 0;
    if (nsteps > 0 && fene == LBFD_FENE_CHOLESKY_AB2) {
        // an instance without a rate history takes its first step as forward Euler: one
        // eager step with the history flags of the instance table as they stand, then the
        // table with every flag set for the graph replays
        bool need = false;
        for (int i = 0; i < b->n; ++i) need |= b->active[i] && !b->inst[i]->ab_valid;
        if (need) {
            BCHK(b, upload_tables(b), "batch tables");
            BCHK(b, launch_batch(b, 0), "batch launch");
            advance(b, 1);
            BCHK(b, upload_tables(b), "batch tables");
            done = 1;
        }
    }
    const int64_t first = done;
    if (b->graph_ok)
        for (; done + 2 <= nsteps; done += 2) BCHK(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
    // remaining steps (or all, without a graph): alternate the parity eagerly
    for (int par = 0; done < nsteps; ++done, par ^= 1) BCHK(b, launch_batch(b, par), "batch launch");
    advance(b, nsteps - first);
    if ((nsteps - first) & 1) BCHK(b, upload_tables(b), "batch tables");  // new parity per instance
    unsigned all = 0;
    for (int i = 0; i < b->n; ++i) {
        if (!b->active[i]) continue;
        unsigned f = 0;
        BCHK(b, read_flags(b->inst[i], &f), "read flags");
        b->inst[i]->flags_seen |= f;
        all |= f;
    }
    lbfd_status st = flags_to_status(all);
    if (st != LBFD_OK) return bfail(b, st, "fault flagged in a batch instance");
    return LBFD_OK;
}

lbfd_status lbfd_batch_diagnostics(lbfd_batch* b, lbfd_diag* out) {
    if (!b || !out) return LBFD_EINVAL;
    for (int i = 0; i < b->n; ++i) {
        lbfd_status st = lbfd_diagnostics(b->inst[i], &out[i]);
        if (st != LBFD_OK) return bfail(b, st, lbfd_last_error(b->inst[i]));
    }
    return LBFD_OK;
}

lbfd_status lbfd_batch_get_fields(lbfd_batch* b, int32_t i, double* rho, double* u, double* C) {
    if (!b || i < 0 || i >= b->n) return LBFD_EINVAL;
    lbfd_status st = lbfd_get_fields(b->inst[i], rho, u, C);
    if (st != LBFD_OK) return bfail(b, st, lbfd_last_error(b->inst[i]));
    return LBFD_OK;
}

lbfd_status lbfd_batch_run_to_steady(lbfd_batch* b, const lbfd_steady_crit* crit, int64_t max_steps, lbfd_diag* out,
                                     int64_t* steady_step) {
    if (!b || !crit || !out || !steady_step || crit->every < 2 || crit->window < crit->every || !(crit->tol > 0))
        return LBFD_EINVAL;
    if ((crit->every & 1) || crit->window % crit->every) return bfail(b, LBFD_EINVAL, "every must be even, window a multiple of every");
    if (crit->windows < 0 || crit->windows > 64) return bfail(b, LBFD_EINVAL, "windows must be in 0..64");
    const int lag = crit->window / crit->every;
    const int nwin = crit->windows > 0 ? crit->windows : 1;
    std::vector<std::vector<double>> hist(b->n);
    for (int i = 0; i < b->n; ++i) steady_step[i] = -1;
    int64_t t = 0;
    std::vector<uint8_t> act = b->active;
    while (t < max_steps) {
        bool any = false;
        for (int i = 0; i < b->n; ++i) any |= act[i] != 0;
        if (!any) break;
        lbfd_status st = lbfd_batch_set_active(b, act.data());
        if (st != LBFD_OK) return st;
        const int64_t n = std::min<int64_t>(crit->every, max_steps - t);
        st = lbfd_batch_step(b, n);
        if (st != LBFD_OK && st != LBFD_ENONFINITE && st != LBFD_EEXTENSIBILITY && st != LBFD_ENOTSPD) return st;
        t += n;
        int32_t left = 0;
        for (int i = 0; i < b->n; ++i) {
            if (!act[i]) continue;
            if (b->inst[i]->flags_seen) {  // a faulting instance is retired, not repaired
                act[i] = 0;
                steady_step[i] = -2;
                continue;
            }
            st = lbfd_diagnostics(b->inst[i], &out[i]);
            if (st != LBFD_OK) return bfail(b, st, lbfd_last_error(b->inst[i]));
            hist[i].push_back(out[i].D);
            const size_t k = hist[i].size();
            bool steady = (int64_t)k > (int64_t)nwin * lag;
            for (int j = 0; steady && j < nwin; ++j)
                steady = fabs(hist[i][k - 1 - (size_t)j * lag] - hist[i][k - 1 - (size_t)(j + 1) * lag]) < crit->tol;
            if (steady) {
                act[i] = 0;
                steady_step[i] = t;
            }
            left += act[i] ? 1 : 0;
        }
        if (b->progress) b->progress(t, left, b->progress_user);
    }
    for (int i = 0; i < b->n; ++i) {
        lbfd_status st = lbfd_diagnostics(b->inst[i], &out[i]);
        if (st != LBFD_OK) return bfail(b, st, lbfd_last_error(b->inst[i]));
    }
    std::vector<uint8_t> all(b->n, 1);
    return lbfd_batch_set_active(b, all.data());
}

lbfd_status lbfd_batch_set_progress(lbfd_batch* b, lbfd_progress_fn fn, void* user) {
    if (!b) return LBFD_EINVAL;
    b->progress = fn;
    b->progress_user = user;
    return LBFD_OK;
}

lbfd_status lbfd_batch_autotune(lbfd_batch* b, int32_t reps, lbfd_tuning* best, double* ms_per_step) {
    if (!b || reps < 1) return LBFD_EINVAL;
    (void)hipSetDevice(b->device);
    hipEvent_t e0, e1;
    BCHK(b, hipEventCreate(&e0), "event");
    BCHK(b, hipEventCreate(&e1), "event");
    // (path, tile) choices: the fused body on 32x8 and 16x16 tiles, the chained body on 64x8
    // and 32x16
    const int shapes[4][2] = {{LBFD_PATH_FUSED, LBFD_TILE_32x8}, {LBFD_PATH_FUSED, LBFD_TILE_16x16},
                              {LBFD_PATH_CHAINED, LBFD_TILE_64x8}, {LBFD_PATH_CHAINED, LBFD_TILE_32x16}};
    const int zcs[5] = {16, 32, 64, 128, 256};
    Tuning keep = b->tune, win = b->tune;
    float best_ms = 1e30f;
    int fene = 0, coll = 0;
    if (!batch_options(b, &fene, &coll))
        return bfail(b, LBFD_EINVAL, "the instances of a batch must share the collision and FENE-P options");
    const bool options = fene != LBFD_FENE_UPWIND_EULER || coll != LBFD_COLLISION_BGK;
    for (const auto& sh : shapes) {
        if (options && sh[0] != LBFD_PATH_CHAINED) continue;  // only the chained body has them
        for (int zc : zcs) {
            b->tune = Tuning{sh[0], sh[1], zc};
            BCHK(b, upload_tables(b), "batch tables");
            BCHK(b, align_moments(b), "batch moments");
            // trial launches read time level n and rewrite level n+1 without advancing, so the
            // state is unchanged by the sweep
            BCHK(b, launch_batch(b, 0), "trial");
            BCHK(b, hipEventRecord(e0, b->stream), "event");
            for (int r = 0; r < reps; ++r) BCHK(b, launch_batch(b, 0), "trial");
            BCHK(b, hipEventRecord(e1, b->stream), "event");
            BCHK(b, hipEventSynchronize(e1), "event");
            float ms = 0.f;
            BCHK(b, hipEventElapsedTime(&ms, e0, e1), "event");
            ms /= reps;
            if (ms < best_ms) {
                best_ms = ms;
                win = b->tune;
            }
        }
    }
    (void)keep;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tune = win;
    b->tables_dirty = true;
    if (best) {
        best->path = win.path;
        best->tile = win.tile;
        best->zchunk = win.zchunk;
        best->reserved = 0;
    }
    if (ms_per_step) *ms_per_step = best_ms;
    return LBFD_OK;
}

void lbfd_batch_destroy(lbfd_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    release_graph(b);
    for (lbfd_ctx* c : b->inst) lbfd_destroy(c);
    delete b;
}

const char* lbfd_batch_last_error(const lbfd_batch* b) { return b ? b->err.c_str() : "null batch"; }

lbfd_ctx* lbfd_batch_instance(lbfd_batch* b, int32_t i) { return (b && i >= 0 && i < b->n) ? b->inst[i] : nullptr; }

// Single-lattice autotuner: times each launch path that implements the lattice's options,
// for each tile shape and z-chunk, on the current state (trial launches do not advance it)
// and keeps the fastest.  A lattice whose options only the split path implements gets the
// split path.
lbfd_status lbfd_autotune(lbfd_ctx* c, int32_t reps, lbfd_tuning* best, double* ms_per_step) {
    if (!c || reps < 1) return LBFD_EINVAL;
    if (!c->have_fields) return LBFD_ESTATE;
    (void)hipSetDevice(c->device);
    unsigned saved = 0;
    if (read_flags(c, &saved) != hipSuccess) return LBFD_EDEVICE;
    c->flags_seen |= saved;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBFD_EDEVICE;
    const int zcs[6] = {8, 16, 32, 64, 128, 256};
    Tuning win{LBFD_PATH_SPLIT, c->tune.tile, c->tune.zchunk};
    float best_ms = 1e30f;
    // a trial step writes the other buffers (populations, C and moments of the next level)
    // but does not swap, so the state is unchanged; the two-pass and split trials form their
    // moments in the next level's moments buffer, so that moments carried by the chained
    // step stay, and the FENE-P rate history goes to the next level's buffer as in a step
    c->dp.ab_hist = c->ab_valid ? 1 : 0;
    auto trial = [&](const Tuning& t) -> hipError_t {
        if (t.path == LBFD_PATH_SPLIT) {
            Buffers tb = c->buf;
            tb.mom = c->buf.mom_next;
            hipError_t e = launch_moments(c->dp, tb, c->stream);
            if (e == hipSuccess) e = launch_forces(c->dp, tb, c->stream);
            return e != hipSuccess ? e : launch_collide(c->dp, tb, c->stream);
        }
        if (t.path == LBFD_PATH_TWOPASS) {
            Buffers tb = c->buf;
            tb.mom = c->buf.mom_next;
            hipError_t e = launch_moments(c->dp, tb, c->stream);
            return e != hipSuccess ? e : launch_fused2(c->dp, tb, t, c->stream);
        }
        if (t.path == LBFD_PATH_CHAINED) {
            hipError_t e = ensure_moments(c);
            return e != hipSuccess ? e : launch_fused3(c->dp, c->buf, t, c->stream);
        }
        return launch_fused(c->dp, c->buf, t, c->stream);
    };
    auto time_it = [&](const Tuning& t) -> bool {
        if (trial(t) != hipSuccess) return false;
        (void)hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps; ++r)
            if (trial(t) != hipSuccess) return false;
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_ms) {
            best_ms = ms;
            win = t;
        }
        return true;
    };
    bool any = false;
    for (int path : {LBFD_PATH_CHAINED, LBFD_PATH_TWOPASS, LBFD_PATH_FUSED}) {
        if (!path_supports(c, path)) continue;
        for (int ti : {LBFD_TILE_32x8, LBFD_TILE_16x16, LBFD_TILE_64x8}) {
            if (ti == LBFD_TILE_64x8 && path == LBFD_PATH_FUSED) continue;
            if (ti != LBFD_TILE_64x8 && path == LBFD_PATH_CHAINED) continue;
            for (int zc : zcs) {
                if (zc > c->grid.nz && zc != 8) continue;
                if (!time_it(Tuning{path, ti, std::min(zc, c->grid.nz)})) return LBFD_EDEVICE;
                any = true;
            }
        }
    }
    if (!any && !time_it(win)) return LBFD_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the trials may have raised the same flags the next real step would; restore
    if (launch_clear_flags(c->buf, c->stream) != hipSuccess) return LBFD_EDEVICE;
    if (saved && launch_set_flags(c->buf, saved, c->stream) != hipSuccess) return LBFD_EDEVICE;
    c->tune = win;
    if (best) {
        best->path = win.path;
        best->tile = win.tile;
        best->zchunk = win.zchunk;
        best->reserved = 0;
    }
    if (ms_per_step) *ms_per_step = best_ms;
    return LBFD_OK;
}

}  // extern "C"

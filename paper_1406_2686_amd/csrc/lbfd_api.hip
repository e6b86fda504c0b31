// lbfd_api.hip -- C ABI of liblbfd (declared in include/lbfd.h): context lifecycle,
// parameter validation, layout of the caller-owned device buffer, stepping, field
// transfer, diagnostics and checkpoints.  All device work runs in the kernels of
// k_step.hip, k_fields.hip and k_diag.hip on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbfd.h"
#include "lbfd_ctx.h"
#include "lbfd_internal.h"

using namespace lbfd;

namespace {

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    uint64_t h0, h1, D0, D1, mom, mom2, uF, ab0, ab1, stage, red, red_out, flags, total;
    int64_t stage_nodes, red_blocks;
};

bool grid_ok(const lbfd_grid* g) {
    if (!g) return false;
    if (g->nx < 1 || g->ny < 3 || g->nz < 1) return false;
    if (g->ncomp != 1 && g->ncomp != 2) return false;
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    // kernels address one field with 32-bit byte offsets
    return N < ((int64_t)1 << 30);
}

Layout layout(const lbfd_grid* g) {
    Layout L{};
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    const int nc = g->ncomp;
    const int64_t plane = (int64_t)g->nx * g->ny;
    L.stage_nodes = std::min<int64_t>(N, std::max<int64_t>(plane, (int64_t)1 << 22));
    L.red_blocks = diag_blocks(N);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.h0 = take((uint64_t)nc * 19 * N * 4);
    L.h1 = take((uint64_t)nc * 19 * N * 4);
    L.D0 = take((uint64_t)6 * N * 4);
    L.D1 = take((uint64_t)6 * N * 4);
    L.mom = take((uint64_t)(nc + 3) * N * 4);
    L.mom2 = take((uint64_t)(nc + 3) * N * 4);
    L.uF = take((uint64_t)(3 + 3 * nc) * N * 4);
    L.ab0 = take((uint64_t)6 * N * 4);
    L.ab1 = take((uint64_t)6 * N * 4);
    L.stage = take((uint64_t)11 * L.stage_nodes * 8);
    L.red = take((uint64_t)L.red_blocks * kDiagVals * 8);
    L.red_out = take((uint64_t)kDiagVals * 8);
    L.flags = take(64);
    L.total = off;
    return L;
}

bool is_fin(double v) { return isfinite(v) != 0; }

const char* params_problem(const lbfd_params* p) {
    if (!p) return "params is NULL";
    const double v[] = {p->tau_A, p->tau_B, p->G, p->delta, p->rho0[0], p->rho0[1], p->eta_p, p->tau_p, p->L2};
    for (double x : v)
        if (!is_fin(x)) return "non-finite parameter";
    if (!(p->tau_A > 0.5 && p->tau_B > 0.5)) return "tau_A and tau_B must exceed 1/2";
    if (!(p->delta > 0.0)) return "delta must be positive";
    if (!(p->tau_p > 0.0)) return "tau_p must be positive";
    if (!(p->L2 > 3.0)) return "L2 must exceed 3";
    if (p->eta_p < 0.0) return "eta_p must be non-negative";
    if (p->polymer_phase < LBFD_POLYMER_NONE || p->polymer_phase > LBFD_POLYMER_ALL) return "bad polymer_phase";
    if (p->coupling != LBFD_COUPLING_FORCE && p->coupling != LBFD_COUPLING_STRESS) return "bad coupling";
    if (p->collision != LBFD_COLLISION_BGK && p->collision != LBFD_COLLISION_MRT) return "bad collision";
    if (p->fene_scheme != LBFD_FENE_UPWIND_EULER && p->fene_scheme != LBFD_FENE_CHOLESKY_AB2) return "bad fene_scheme";
    if (!is_fin(p->fene_kappa) || p->fene_kappa < 0.0) return "fene_kappa must be finite and >= 0";
    return nullptr;
}

void fill_devparams(lbfd_ctx* c) {
    DevParams& d = c->dp;
    const lbfd_params& p = c->params;
    d.nx = c->grid.nx;
    d.ny = c->grid.ny;
    d.nz = c->grid.nz;
    d.nc = c->grid.ncomp;
    d.N = (int64_t)d.nx * d.ny * d.nz;
    d.tauA = (float)p.tau_A;
    d.tauB = (float)p.tau_B;
    d.G = (float)p.G;
    d.inv_delta = (float)(1.0 / p.delta);
    d.rho0[0] = (float)p.rho0[0];
    d.rho0[1] = (float)p.rho0[1];
    d.phase = p.polymer_phase;
    d.pstress = p.polymer_phase == LBFD_POLYMER_NONE ? 0.0f : (float)(p.eta_p / p.tau_p);
    d.inv_tau_p = (float)(1.0 / p.tau_p);
    d.L2 = (float)p.L2;
    d.L2m3 = (float)(p.L2 - 3.0);
    d.coupling = p.coupling;
    d.collision = p.collision;
    d.fene = p.fene_scheme;
    d.kappa = (float)p.fene_kappa;
    d.ab_hist = 0;
    d.pad_ = 0;
    for (int k = 0; k < 3; ++k) {
        d.ub[k] = (float)c->ub[k];
        d.ut[k] = (float)c->ut[k];
    }
}


lbfd_status fail(lbfd_ctx* c, lbfd_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

lbfd_status hip_fail(lbfd_ctx* c, hipError_t e, const char* where) {
    return fail(c, LBFD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr, where)                      \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return hip_fail(c, _e, where); \
    } while (0)

lbfd_status flags_status(unsigned f) {
    if (f & LBFD_FLAG_NONFINITE) return LBFD_ENONFINITE;
    if (f & LBFD_FLAG_EXTENSIBILITY) return LBFD_EEXTENSIBILITY;
    if (f & LBFD_FLAG_NOT_SPD) return LBFD_ENOTSPD;
    return LBFD_OK;
}

bool box_ok(const lbfd_ctx* c, int x0, int y0, int z0, int bx, int by, int bz) {
    return x0 >= 0 && y0 >= 0 && z0 >= 0 && bx >= 1 && by >= 1 && bz >= 1 && x0 + bx <= c->grid.nx &&
           y0 + by <= c->grid.ny && z0 + bz <= c->grid.nz;
}

}  // namespace

namespace lbfd {

void bind_current(lbfd_ctx* c) {
    c->buf.h = c->hbuf[c->cur];
    c->buf.hn = c->hbuf[1 - c->cur];
    c->buf.D = c->Dbuf[c->cur];
    c->buf.Dn = c->Dbuf[1 - c->cur];
    c->buf.mom = c->mbuf[c->mcur];
    c->buf.mom_next = c->mbuf[1 - c->mcur];
    c->buf.ab = c->abuf[c->cur];
    c->buf.ab_next = c->abuf[1 - c->cur];
}

// moments of the current state in buf.mom: kept when they are already there (the chained
// step carries them from step to step, and recomputing them here would round them
// differently), else formed by the moments pass
hipError_t ensure_moments(lbfd_ctx* c) {
    if (c->mom_valid) return hipSuccess;
    hipError_t e = launch_moments(c->dp, c->buf, c->stream);
    if (e == hipSuccess) c->mom_valid = true;
    return e;
}

// derived side fields (moments, forces, half-force velocity) of the current state
hipError_t compute_side_fields(lbfd_ctx* c) {
    hipError_t e = ensure_moments(c);
    if (e != hipSuccess) return e;
    return launch_forces(c->dp, c->buf, c->stream);
}

// planes per workgroup of the fused pass: enough workgroups to fill 256 CUs several
// times over, at least 8 planes so the 4-plane pipeline fill stays small, and at most 64
// (measured best on the 1024x256x1024 droplet grid: 49.4 ms at 64 vs 50.9 at 256 and
// 53.5 at 16 planes per workgroup)
int auto_zchunk(const lbfd_grid& g, int tile) {
    const int tx = tile == 2 ? 16 : (tile == 3 ? 64 : 32);
    const int ty = tile == 2 ? 16 : 8;
    const int64_t tiles = (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
    int64_t zc = ((int64_t)g.nz * tiles + 2047) / 2048;
    zc = std::min<int64_t>(std::max<int64_t>(zc, 8), 64);
    return (int)std::min<int64_t>(zc, g.nz);
}

bool path_supports(const lbfd_ctx* c, int path) {
    if (path == LBFD_PATH_SPLIT) return true;
    // the MRT collision and the Cholesky integrator are in the chained tile body only (MRT
    // collides each node from all 19 of its populations, halo nodes included)
    if (c->dp.collision == LBFD_COLLISION_MRT || c->dp.fene == LBFD_FENE_CHOLESKY_AB2)
        return path == LBFD_PATH_CHAINED;
    return true;
}

int step_path(const lbfd_ctx* c) { return path_supports(c, c->tune.path) ? c->tune.path : LBFD_PATH_SPLIT; }

hipError_t enqueue_steps(lbfd_ctx* c, int64_t n) {
    const int path = step_path(c);
    for (int64_t t = 0; t < n; ++t) {
        hipError_t e;
        c->dp.ab_hist = c->ab_valid ? 1 : 0;
        if (path == LBFD_PATH_SPLIT) {
            e = launch_moments(c->dp, c->buf, c->stream);
            if (e == hipSuccess) e = launch_forces(c->dp, c->buf, c->stream);
            if (e == hipSuccess) e = launch_collide(c->dp, c->buf, c->stream);
        } else if (path == LBFD_PATH_TWOPASS) {
            Tuning tt = c->tune;
            if (tt.zchunk <= 0) tt.zchunk = auto_zchunk(c->grid, tt.tile);
            e = launch_moments(c->dp, c->buf, c->stream);
            if (e == hipSuccess) e = launch_fused2(c->dp, c->buf, tt, c->stream);
        } else if (path == LBFD_PATH_CHAINED) {
            Tuning tt = c->tune;
            tt.tile = LBFD_TILE_64x8;
            if (tt.zchunk <= 0) tt.zchunk = auto_zchunk(c->grid, tt.tile);
            e = ensure_moments(c);
            if (e == hipSuccess) e = launch_fused3(c->dp, c->buf, tt, c->stream);
        } else {
            Tuning tt = c->tune;
            if (tt.zchunk <= 0) tt.zchunk = auto_zchunk(c->grid, tt.tile);
            e = launch_fused(c->dp, c->buf, tt, c->stream);
        }
        if (e != hipSuccess) return e;
        c->cur = 1 - c->cur;
        c->ab_valid = c->dp.fene == LBFD_FENE_CHOLESKY_AB2;  // the step wrote this step's rate
        if (path == LBFD_PATH_CHAINED) {
            c->mcur = 1 - c->mcur;  // the step wrote the moments of the new level
            c->mom_valid = true;
        } else {
            c->mom_valid = false;
        }
        bind_current(c);
        c->steps++;
    }
    return hipSuccess;
}

void fill_diag(const lbfd_ctx* c, const double* r, lbfd_diag* out) {
    memset(out, 0, sizeof(*out));
    out->mass[0] = r[0];
    out->mass[1] = r[1];
    for (int d = 0; d < 3; ++d) out->momentum[d] = r[2 + d];
    const double W = r[5];
    out->W = W;
    if (W > 0.0) {
        const double xc = r[6] / W, yc = r[7] / W, zc = r[8] / W;
        out->centroid[0] = xc;
        out->centroid[1] = yc;
        out->centroid[2] = zc;
        const double cen[3] = {xc, yc, zc};
        const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
        for (int k = 0; k < 6; ++k) out->M[k] = r[9 + k] / W - cen[ii[k]] * cen[jj[k]];
        // principal axes of the x-y block (Sec. 4.1: axes a, b in the shear plane)
        const double tr = out->M[0] + out->M[1], df = out->M[0] - out->M[1];
        const double rad = sqrt(0.25 * df * df + out->M[3] * out->M[3]);
        const double l1 = 0.5 * tr + rad;
        double l2 = 0.5 * tr - rad;
        if (l2 < 0.0) l2 = 0.0;
        const double a = sqrt(l1), b = sqrt(l2);
        out->D = (a + b) > 0.0 ? (a - b) / (a + b) : 0.0;
        out->theta_deg = rad > 0.0 ? 0.5 * atan2(2.0 * out->M[3], df) * (180.0 / M_PI) : 0.0;
    }
    out->min_L2_minus_trC = r[15];
    out->min_minor = r[16];
    out->max_u = r[17];
    out->flags = c->flags_seen;
    out->step = c->steps;
    out->poly_trace_excess = r[19] > 0.0 ? r[18] / r[19] : 0.0;
}

hipError_t read_flags(lbfd_ctx* c, unsigned* out) {
    unsigned f = 0;
    hipError_t e = hipMemcpyAsync(&f, c->buf.flags, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    *out = f;
    return e;
}

}  // namespace lbfd

namespace {

// Checks of one box of host fields before upload (finite, positive densities, C SPD with tr C < L^2).
const char* fields_problem(const lbfd_ctx* c, int64_t B, const double* rho, const double* u, const double* C) {
    const int nc = c->grid.ncomp;
    for (int64_t i = 0; i < B; ++i) {
        double tot = 0.0;
        for (int s = 0; s < nc; ++s) {
            const double r = rho[(int64_t)s * B + i];
            if (!is_fin(r) || !(r > 0.0)) return "densities must be finite and positive";
            tot += r;
        }
        (void)tot;
        for (int d = 0; d < 3; ++d)
            if (!is_fin(u[d * B + i])) return "non-finite velocity";
        double cc[6];
        for (int k = 0; k < 6; ++k) {
            cc[k] = C[k * B + i];
            if (!is_fin(cc[k])) return "non-finite conformation tensor";
        }
        if (!(cc[0] + cc[1] + cc[2] < c->params.L2)) return "tr C must be below L2";
        const double m2 = cc[0] * cc[1] - cc[3] * cc[3];
        const double m3 = cc[0] * (cc[1] * cc[2] - cc[5] * cc[5]) - cc[3] * (cc[3] * cc[2] - cc[5] * cc[4]) +
                          cc[4] * (cc[3] * cc[5] - cc[1] * cc[4]);
        if (!(cc[0] > 0.0 && m2 > 0.0 && m3 > 0.0)) return "C must be symmetric positive definite";
    }
    return nullptr;
}

}  // namespace

extern "C" {

const char* lbfd_version(void) { return "lbfd 0.1 (gfx950, FP32 populations/C, FP64 diagnostics)"; }

lbfd_status lbfd_state_bytes(const lbfd_grid* grid, uint64_t* bytes) {
    if (!grid_ok(grid) || !bytes) return LBFD_EINVAL;
    *bytes = layout(grid).total;
    return LBFD_OK;
}

lbfd_status lbfd_create(const lbfd_grid* grid, const lbfd_params* params, void* dev_state, uint64_t bytes,
                        void* hip_stream, lbfd_ctx** out) {
    if (!out) return LBFD_EINVAL;
    *out = nullptr;
    if (!grid_ok(grid)) return LBFD_EINVAL;
    if (params_problem(params)) return LBFD_EINVAL;
    if (!dev_state || ((uintptr_t)dev_state % kAlign) != 0) return LBFD_EINVAL;
    const Layout L = layout(grid);
    if (bytes < L.total) return LBFD_ENOMEM;
    lbfd_ctx* c = new (std::nothrow) lbfd_ctx();
    if (!c) return LBFD_ENOMEM;
    c->grid = *grid;
    c->params = *params;
    for (int k = 0; k < 3; ++k) c->ub[k] = c->ut[k] = 0.0;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LBFD_EDEVICE;
    }
    c->dev = (char*)dev_state;
    c->bytes = bytes;
    c->hbuf[0] = (float*)(c->dev + L.h0);
    c->hbuf[1] = (float*)(c->dev + L.h1);
    c->Dbuf[0] = (float*)(c->dev + L.D0);
    c->Dbuf[1] = (float*)(c->dev + L.D1);
    c->cur = 0;
    c->mbuf[0] = (float*)(c->dev + L.mom);
    c->mbuf[1] = (float*)(c->dev + L.mom2);
    c->mcur = 0;
    c->mom_valid = false;
    c->buf.uF = (float*)(c->dev + L.uF);
    c->abuf[0] = (float*)(c->dev + L.ab0);
    c->abuf[1] = (float*)(c->dev + L.ab1);
    c->ab_valid = false;
    c->buf.stage = (double*)(c->dev + L.stage);
    c->buf.stage_nodes = L.stage_nodes;
    c->buf.red = (double*)(c->dev + L.red);
    c->buf.red_blocks = L.red_blocks;
    c->buf.red_out = (double*)(c->dev + L.red_out);
    c->buf.flags = (unsigned*)(c->dev + L.flags);
    bind_current(c);
    fill_devparams(c);
    // the chained step is the fastest shape on large lattices (25.5 ms per step on the
    // 1024x256x1024 droplet, against 30.0 for the two-pass step on the same 64x8 tiles and
    // 47.2 for the fused single pass); lbfd_autotune compares the shapes for a given lattice
    c->tune = Tuning{LBFD_PATH_CHAINED, LBFD_TILE_64x8, 0};
    c->steps = 0;
    c->flags_seen = 0;
    c->have_fields = false;
    (void)hipSetDevice(c->device);
    hipError_t e = launch_clear_flags(c->buf, c->stream);
    if (e != hipSuccess) {
        delete c;
        return LBFD_EDEVICE;
    }
    *out = c;
    return LBFD_OK;
}

lbfd_status lbfd_set_params(lbfd_ctx* c, const lbfd_params* params) {
    if (!c) return LBFD_EINVAL;
    if (const char* why = params_problem(params)) return fail(c, LBFD_EINVAL, why);
    if (params->fene_scheme != c->params.fene_scheme) c->ab_valid = false;
    c->params = *params;
    fill_devparams(c);
    return LBFD_OK;
}

lbfd_status lbfd_set_walls(lbfd_ctx* c, const double u_bottom[3], const double u_top[3]) {
    if (!c || !u_bottom || !u_top) return LBFD_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!is_fin(u_bottom[k]) || !is_fin(u_top[k])) return fail(c, LBFD_EINVAL, "non-finite wall velocity");
    if (u_bottom[1] != 0.0 || u_top[1] != 0.0) return fail(c, LBFD_EINVAL, "walls move tangentially only (u_y = 0)");
    for (int k = 0; k < 3; ++k) {
        c->ub[k] = u_bottom[k];
        c->ut[k] = u_top[k];
    }
    fill_devparams(c);
    return LBFD_OK;
}

lbfd_status lbfd_set_fields_box(lbfd_ctx* c, int32_t x0, int32_t y0, int32_t z0, int32_t bx, int32_t by,
                                int32_t bz, const double* rho, const double* u, const double* C) {
    if (!c || !rho || !u || !C) return LBFD_EINVAL;
    if (!box_ok(c, x0, y0, z0, bx, by, bz)) return fail(c, LBFD_EINVAL, "box outside the lattice");
    (void)hipSetDevice(c->device);
    const int nc = c->grid.ncomp;
    const int64_t plane = (int64_t)bx * by;
    const int64_t B = plane * bz;
    if (const char* why = fields_problem(c, B, rho, u, C)) return fail(c, LBFD_EINVAL, why);
    // slab chunks in z so that each fits in the staging area
    const int64_t zchunk = std::max<int64_t>(1, c->buf.stage_nodes / plane);
    std::vector<double> tmp;
    for (int64_t zs = 0; zs < bz; zs += zchunk) {
        const int nz_ = (int)std::min<int64_t>(zchunk, bz - zs);
        const int64_t Bc = plane * nz_;
        tmp.resize((size_t)(nc + 9) * Bc);
        for (int s = 0; s < nc; ++s) memcpy(&tmp[(size_t)s * Bc], rho + (int64_t)s * B + zs * plane, Bc * 8);
        for (int d = 0; d < 3; ++d) memcpy(&tmp[(size_t)(nc + d) * Bc], u + (int64_t)d * B + zs * plane, Bc * 8);
        for (int k = 0; k < 6; ++k) memcpy(&tmp[(size_t)(nc + 3 + k) * Bc], C + (int64_t)k * B + zs * plane, Bc * 8);
        HIPCHK(c, hipMemcpyAsync(c->buf.stage, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice, c->stream),
               "set_fields upload");
        Box box{x0, y0, (int)(z0 + zs), bx, by, nz_};
        HIPCHK(c, launch_init_box(c->dp, c->buf, box, c->stream), "init kernel");
        // the staging area is reused by the next chunk: wait for this one
        HIPCHK(c, hipStreamSynchronize(c->stream), "set_fields sync");
    }
    c->have_fields = true;
    c->mom_valid = false;
    c->ab_valid = false;
    return LBFD_OK;
}

lbfd_status lbfd_reset_counters(lbfd_ctx* c) {
    if (!c) return LBFD_EINVAL;
    (void)hipSetDevice(c->device);
    c->steps = 0;
    c->flags_seen = 0;
    HIPCHK(c, launch_clear_flags(c->buf, c->stream), "clear flags");
    return LBFD_OK;
}

lbfd_status lbfd_set_fields(lbfd_ctx* c, const double* rho, const double* u, const double* C) {
    if (!c) return LBFD_EINVAL;
    lbfd_status st = lbfd_set_fields_box(c, 0, 0, 0, c->grid.nx, c->grid.ny, c->grid.nz, rho, u, C);
    if (st != LBFD_OK) return st;
    return lbfd_reset_counters(c);
}

lbfd_status lbfd_step_async(lbfd_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return LBFD_EINVAL;
    if (!c->have_fields) return fail(c, LBFD_ESTATE, "step before set_fields");
    (void)hipSetDevice(c->device);
    HIPCHK(c, enqueue_steps(c, nsteps), "step launch");
    return LBFD_OK;
}

lbfd_status lbfd_step(lbfd_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return LBFD_EINVAL;
    if (!c->have_fields) return fail(c, LBFD_ESTATE, "step before set_fields");
    (void)hipSetDevice(c->device);
    unsigned before = 0;
    HIPCHK(c, read_flags(c, &before), "read flags");
    c->flags_seen |= before;
    HIPCHK(c, launch_clear_flags(c->buf, c->stream), "clear flags");
    HIPCHK(c, enqueue_steps(c, nsteps), "step launch");
    unsigned f = 0;
    HIPCHK(c, read_flags(c, &f), "read flags");
    c->flags_seen |= f;
    lbfd_status st = flags_status(f);
    if (st != LBFD_OK) return fail(c, st, "fault flagged during step");
    return LBFD_OK;
}

lbfd_status lbfd_fenep_kinematic(lbfd_ctx* c, const double* u, int64_t nsteps) {
    if (!c || !u || nsteps < 0) return LBFD_EINVAL;
    if (!c->have_fields) return fail(c, LBFD_ESTATE, "kinematic steps before set_fields");
    (void)hipSetDevice(c->device);
    const int64_t N = c->dp.N;
    std::vector<float> uf((size_t)3 * N);
    for (int64_t i = 0; i < 3 * N; ++i) {
        if (!is_fin(u[i])) return fail(c, LBFD_EINVAL, "non-finite velocity");
        uf[(size_t)i] = (float)u[i];
    }
    // the prescribed velocity takes the place of the half-force velocity of the side fields
    HIPCHK(c, hipMemcpyAsync(c->buf.uF, uf.data(), uf.size() * 4, hipMemcpyHostToDevice, c->stream),
           "velocity upload");
    unsigned before = 0;
    HIPCHK(c, read_flags(c, &before), "read flags");  // synchronises: the upload has left uf
    c->flags_seen |= before;
    HIPCHK(c, launch_clear_flags(c->buf, c->stream), "clear flags");
    // C - I and the rate history alternate between their two buffers; the populations and
    // the buffer index of the lattice state are left as they are
    float* Din = c->Dbuf[c->cur];
    float* Dout = c->Dbuf[1 - c->cur];
    float* ain = c->abuf[c->cur];
    float* aout = c->abuf[1 - c->cur];
    for (int64_t t = 0; t < nsteps; ++t) {
        c->dp.ab_hist = c->ab_valid ? 1 : 0;
        HIPCHK(c, launch_fenep_kinematic(c->dp, c->buf.uF, Din, Dout, ain, aout, c->buf.flags, c->stream),
               "kinematic step launch");
        std::swap(Din, Dout);
        std::swap(ain, aout);
        c->ab_valid = c->dp.fene == LBFD_FENE_CHOLESKY_AB2;
    }
    if (Din != c->Dbuf[c->cur]) {
        HIPCHK(c, hipMemcpyAsync(c->Dbuf[c->cur], Din, (size_t)6 * N * 4, hipMemcpyDeviceToDevice, c->stream),
               "C copy");
        if (c->ab_valid)
            HIPCHK(c, hipMemcpyAsync(c->abuf[c->cur], ain, (size_t)6 * N * 4, hipMemcpyDeviceToDevice, c->stream),
                   "history copy");
    }
    unsigned f = 0;
    HIPCHK(c, read_flags(c, &f), "read flags");
    c->flags_seen |= f;
    lbfd_status st = flags_status(f);
    if (st != LBFD_OK) return fail(c, st, "fault flagged during kinematic steps");
    return LBFD_OK;
}

lbfd_status lbfd_get_flags(lbfd_ctx* c, uint32_t* flags) {
    if (!c || !flags) return LBFD_EINVAL;
    (void)hipSetDevice(c->device);
    unsigned f = 0;
    HIPCHK(c, read_flags(c, &f), "read flags");
    c->flags_seen |= f;
    *flags = c->flags_seen;
    return LBFD_OK;
}

lbfd_status lbfd_get_fields_box(lbfd_ctx* c, int32_t x0, int32_t y0, int32_t z0, int32_t bx, int32_t by,
                                int32_t bz, double* rho, double* u, double* C) {
    if (!c) return LBFD_EINVAL;
    if (!c->have_fields) return fail(c, LBFD_ESTATE, "get_fields before set_fields");
    if (!box_ok(c, x0, y0, z0, bx, by, bz)) return fail(c, LBFD_EINVAL, "box outside the lattice");
    (void)hipSetDevice(c->device);
    const int nc = c->grid.ncomp;
    HIPCHK(c, compute_side_fields(c), "side fields");
    const int64_t plane = (int64_t)bx * by;
    const int64_t B = plane * bz;
    const int64_t zchunk = std::max<int64_t>(1, c->buf.stage_nodes / plane);
    std::vector<double> tmp;
    for (int64_t zs = 0; zs < bz; zs += zchunk) {
        const int nz_ = (int)std::min<int64_t>(zchunk, bz - zs);
        const int64_t Bc = plane * nz_;
        Box box{x0, y0, (int)(z0 + zs), bx, by, nz_};
        HIPCHK(c, launch_fields_box(c->dp, c->buf, box, c->stream), "fields kernel");
        tmp.resize((size_t)(nc + 9) * Bc);
        HIPCHK(c, hipMemcpyAsync(tmp.data(), c->buf.stage, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream),
               "get_fields download");
        HIPCHK(c, hipStreamSynchronize(c->stream), "get_fields sync");
        if (rho)
            for (int s = 0; s < nc; ++s) memcpy(rho + (int64_t)s * B + zs * plane, &tmp[(size_t)s * Bc], Bc * 8);
        if (u)
            for (int d = 0; d < 3; ++d) memcpy(u + (int64_t)d * B + zs * plane, &tmp[(size_t)(nc + d) * Bc], Bc * 8);
        if (C)
            for (int k = 0; k < 6; ++k)
                memcpy(C + (int64_t)k * B + zs * plane, &tmp[(size_t)(nc + 3 + k) * Bc], Bc * 8);
    }
    return LBFD_OK;
}

lbfd_status lbfd_get_fields(lbfd_ctx* c, double* rho, double* u, double* C) {
    if (!c) return LBFD_EINVAL;
    return lbfd_get_fields_box(c, 0, 0, 0, c->grid.nx, c->grid.ny, c->grid.nz, rho, u, C);
}

lbfd_status lbfd_diagnostics(lbfd_ctx* c, lbfd_diag* out) {
    if (!c || !out) return LBFD_EINVAL;
    if (!c->have_fields) return fail(c, LBFD_ESTATE, "diagnostics before set_fields");
    (void)hipSetDevice(c->device);
    HIPCHK(c, compute_side_fields(c), "side fields");
    HIPCHK(c, launch_diag(c->dp, c->buf, c->stream), "diag kernel");
    double r[kDiagVals];
    HIPCHK(c, hipMemcpyAsync(r, c->buf.red_out, sizeof(r), hipMemcpyDeviceToHost, c->stream), "diag download");
    unsigned f = 0;
    HIPCHK(c, read_flags(c, &f), "read flags");
    c->flags_seen |= f;
    fill_diag(c, r, out);
    return LBFD_OK;
}

lbfd_status lbfd_checkpoint_bytes(lbfd_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return LBFD_EINVAL;
    const int64_t N = c->dp.N;
    *bytes = 64 + (uint64_t)(c->grid.ncomp * 19 + 6 + c->grid.ncomp + 3 + 6) * N * 4;
    return LBFD_OK;
}

lbfd_status lbfd_get_state(lbfd_ctx* c, void* host, uint64_t bytes) {
    uint64_t need = 0;
    if (!c || !host || lbfd_checkpoint_bytes(c, &need) != LBFD_OK || bytes < need) return LBFD_EINVAL;
    if (!c->have_fields) return fail(c, LBFD_ESTATE, "get_state before set_fields");
    (void)hipSetDevice(c->device);
    unsigned f = 0;
    HIPCHK(c, read_flags(c, &f), "read flags");
    c->flags_seen |= f;
    const int64_t N = c->dp.N;
    char* p = (char*)host;
    int64_t hdr[8] = {0x4c424644, (int64_t)c->grid.nx, (int64_t)c->grid.ny, (int64_t)c->grid.nz,
                      (int64_t)c->grid.ncomp, c->steps, (int64_t)c->flags_seen, c->ab_valid ? 1 : 0};
    memcpy(p, hdr, 64);
    HIPCHK(c, hipMemcpyAsync(p + 64, c->buf.h, (size_t)c->grid.ncomp * 19 * N * 4, hipMemcpyDeviceToHost, c->stream),
           "state download");
    HIPCHK(c, hipMemcpyAsync(p + 64 + (size_t)c->grid.ncomp * 19 * N * 4, c->buf.D, (size_t)6 * N * 4,
                             hipMemcpyDeviceToHost, c->stream),
           "state download");
    // the moments of this level, so that a restart continues bitwise like the run it came from
    HIPCHK(c, ensure_moments(c), "moments");
    HIPCHK(c, hipMemcpyAsync(p + 64 + (size_t)(c->grid.ncomp * 19 + 6) * N * 4, c->buf.mom,
                             (size_t)(c->grid.ncomp + 3) * N * 4, hipMemcpyDeviceToHost, c->stream),
           "state download");
    // the FENE-P integrator's history (second-order Adams-Bashforth)
    HIPCHK(c, hipMemcpyAsync(p + 64 + (size_t)(c->grid.ncomp * 19 + 6 + c->grid.ncomp + 3) * N * 4, c->buf.ab,
                             (size_t)6 * N * 4, hipMemcpyDeviceToHost, c->stream),
           "state download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "state sync");
    return LBFD_OK;
}

lbfd_status lbfd_set_state(lbfd_ctx* c, const void* host, uint64_t bytes) {
    uint64_t need = 0;
    if (!c || !host || lbfd_checkpoint_bytes(c, &need) != LBFD_OK || bytes < need) return LBFD_EINVAL;
    int64_t hdr[8];
    memcpy(hdr, host, 64);
    if (hdr[0] != 0x4c424644 || hdr[1] != c->grid.nx || hdr[2] != c->grid.ny || hdr[3] != c->grid.nz ||
        hdr[4] != c->grid.ncomp)
        return fail(c, LBFD_EINVAL, "checkpoint does not match this lattice");
    (void)hipSetDevice(c->device);
    const int64_t N = c->dp.N;
    const char* p = (const char*)host;
    HIPCHK(c, hipMemcpyAsync(c->buf.h, p + 64, (size_t)c->grid.ncomp * 19 * N * 4, hipMemcpyHostToDevice, c->stream),
           "state upload");
    HIPCHK(c, hipMemcpyAsync(c->buf.D, p + 64 + (size_t)c->grid.ncomp * 19 * N * 4, (size_t)6 * N * 4,
                             hipMemcpyHostToDevice, c->stream),
           "state upload");
    HIPCHK(c, hipMemcpyAsync(c->buf.mom, p + 64 + (size_t)(c->grid.ncomp * 19 + 6) * N * 4,
                             (size_t)(c->grid.ncomp + 3) * N * 4, hipMemcpyHostToDevice, c->stream),
           "state upload");
    HIPCHK(c, hipMemcpyAsync(c->buf.ab, p + 64 + (size_t)(c->grid.ncomp * 19 + 6 + c->grid.ncomp + 3) * N * 4,
                             (size_t)6 * N * 4, hipMemcpyHostToDevice, c->stream),
           "state upload");
    c->mom_valid = true;
    c->ab_valid = hdr[7] != 0;
    HIPCHK(c, launch_clear_flags(c->buf, c->stream), "clear flags");
    HIPCHK(c, hipStreamSynchronize(c->stream), "state sync");
    c->steps = hdr[5];
    c->flags_seen = (unsigned)hdr[6];
    c->have_fields = true;
    return LBFD_OK;
}

lbfd_status lbfd_set_tuning(lbfd_ctx* c, const lbfd_tuning* t) {
    if (!c || !t) return LBFD_EINVAL;
    if (t->path != LBFD_PATH_FUSED && t->path != LBFD_PATH_SPLIT && t->path != LBFD_PATH_TWOPASS &&
        t->path != LBFD_PATH_CHAINED)
        return fail(c, LBFD_EINVAL, "bad path");
    if (t->tile < LBFD_TILE_32x8 || t->tile > LBFD_TILE_64x8) return fail(c, LBFD_EINVAL, "bad tile");
    if (t->zchunk < 0) return fail(c, LBFD_EINVAL, "zchunk must be >= 0");
    c->tune = Tuning{t->path, t->tile, t->zchunk};
    return LBFD_OK;
}

lbfd_status lbfd_get_tuning(lbfd_ctx* c, lbfd_tuning* t) {
    if (!c || !t) return LBFD_EINVAL;
    t->path = step_path(c);
    t->tile = t->path == LBFD_PATH_CHAINED ? LBFD_TILE_64x8 : c->tune.tile;
    t->zchunk = c->tune.zchunk > 0 ? c->tune.zchunk : auto_zchunk(c->grid, t->tile);
    t->reserved = 0;
    return LBFD_OK;
}

void lbfd_destroy(lbfd_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

const char* lbfd_last_error(const lbfd_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// k_step.hip -- one time step of the hybrid LB/FD method on gfx950, three passes:
//
//   k_moments : populations -> delta rho_s, j                       (Sec. 2, moments)
//   k_forces  : Shan-Chen force (Sec. 2, eq. SCforce), polymer-stress divergence of
//               T = (eta_p/tau_p) m(phi) (f(r) C - I) (FENE-P feedback, modulated by
//               f+-(phi)), species split F_s = g_s + (rho_s/rho) F_p (weight of eq.
//               MODEtransformation), half-force velocity u (eq. equilibrium:vel)
//   k_collide : BGK collision with the forcing source (eq. LB, Lambda = I/tau(phi)),
//               push streaming with half-way moving-wall bounce-back, and the explicit
//               FENE-P step C += -(u.grad)_upwind C + G^T C + C G - (f C - I)/tau_p with
//               G_ij = d_i u_j (eq. FENE), all reading time level n only.
//
// Every pass is a one-thread-per-node map over [z][y][x] with x fastest, so each
// wavefront reads and writes 64 consecutive FP32 words per population plane.  Blocks
// are remapped so that each XCD (8 per MI355X) owns one contiguous range of the
// lattice; neighbour reads in y and z then hit the same XCD's L2.
#include "d3q19.h"
#include "fene_chol.h"
#include "lbfd_internal.h"

namespace lbfd {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int64_t node_id() {
    return xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
}

// delta rho and momentum of the populations of one component at node n.  Opposite
// pairs are differenced first (c_{a+1} = -c_a), which keeps j free of the rho0 shift.
__device__ __forceinline__ void pop_moments(const float* __restrict__ h, int64_t N, int64_t n,
                                            float& dr, float& jx, float& jy, float& jz) {
    float f[kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a) f[a] = h[a * N + n];
    float s = f[0];
#pragma unroll
    for (int a = 1; a < kQ; a += 2) s += f[a] + f[a + 1];
    dr = s;
#pragma unroll
    for (int a = 1; a < kQ; a += 2) {
        const float d = f[a] - f[a + 1];
        jx += cx(a) * d;
        jy += cy(a) * d;
        jz += cz(a) * d;
    }
}

__global__ __launch_bounds__(kBlock) void k_moments(DevParams p, const float* __restrict__ h,
                                                    float* __restrict__ mom) {
    const int64_t n = node_id();
    if (n >= p.N) return;
    const int64_t N = p.N;
    float jx = 0.f, jy = 0.f, jz = 0.f;
    for (int s = 0; s < p.nc; ++s) {
        float dr;
        pop_moments(h + (int64_t)s * kQ * N, N, n, dr, jx, jy, jz);
        mom[s * N + n] = dr;
    }
    mom[(p.nc + 0) * N + n] = jx;
    mom[(p.nc + 1) * N + n] = jy;
    mom[(p.nc + 2) * N + n] = jz;
}

// order parameter and feedback modulation
__device__ __forceinline__ float phase_phi(const DevParams& p, float rA, float rB) {
    return p.nc == 2 ? (rA - rB) / (rA + rB) : 1.0f;
}
__device__ __forceinline__ float modulation(const DevParams& p, float phi) {
    if (p.phase == 3) return 1.0f;
    if (p.phase == 0) return 0.0f;
    const float t = tanhf(phi * p.inv_delta);
    return p.phase == 1 ? 0.5f * (1.0f + t) : 0.5f * (1.0f - t);
}

// Polymer stress of one (possibly ghost) node from D = C - I and phi:
// T = (eta_p/tau_p) m (f D + (f - 1) I), f = (L^2 - 3)/(L^2 - 3 - tr D).
__device__ __forceinline__ void stress(const DevParams& p, const float d[6], float phi, float T[6],
                                       unsigned& bad) {
    const float trd = d[0] + d[1] + d[2];
    const float den = p.L2m3 - trd;
    if (!(den > 0.0f)) bad |= 2u;
    const float inv = 1.0f / den;
    const float f = p.L2m3 * inv;
    const float fm1 = trd * inv;
    const float pre = p.pstress * modulation(p, phi);
#pragma unroll
    for (int k = 0; k < 6; ++k) T[k] = pre * (f * d[k] + (k < 3 ? fm1 : 0.0f));
}

__global__ __launch_bounds__(kBlock) void k_forces(DevParams p, const float* __restrict__ mom,
                                                   const float* __restrict__ D,
                                                   float* __restrict__ uF,
                                                   unsigned* __restrict__ flags) {
    const int64_t n = node_id();
    if (n >= p.N) return;
    const int64_t N = p.N;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int x = (int)(n % nx);
    const int64_t r = n / nx;
    const int y = (int)(r % ny);
    const int z = (int)(r / ny);

    const float dA = mom[n];
    const float dB = p.nc == 2 ? mom[N + n] : 0.0f;
    const float rA = p.rho0[0] + dA;
    const float rB = p.nc == 2 ? p.rho0[1] + dB : 0.0f;
    const float rho = rA + rB;
    float j[3] = {mom[(p.nc + 0) * N + n], mom[(p.nc + 1) * N + n], mom[(p.nc + 2) * N + n]};

    float gA[3] = {0.f, 0.f, 0.f}, gB[3] = {0.f, 0.f, 0.f};
    if (p.nc == 2 && p.G != 0.0f) {
        // s_s = sum_a w_a rho_s(x + c_a) c_a, summed over opposite pairs as differences
        float sA[3] = {0.f, 0.f, 0.f}, sB[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 1; a < kQ; a += 2) {
            const int xp = wrap1(x + cx(a), nx), yp = clampy(y + cy(a), ny), zp = wrap1(z + cz(a), nz);
            const int xm = wrap1(x - cx(a), nx), ym = clampy(y - cy(a), ny), zm = wrap1(z - cz(a), nz);
            const int64_t np_ = ((int64_t)zp * ny + yp) * nx + xp;
            const int64_t nm_ = ((int64_t)zm * ny + ym) * nx + xm;
            const float da = wgt(a) * (mom[np_] - mom[nm_]);
            const float db = wgt(a) * (mom[N + np_] - mom[N + nm_]);
            sA[0] += cx(a) * da; sA[1] += cy(a) * da; sA[2] += cz(a) * da;
            sB[0] += cx(a) * db; sB[1] += cy(a) * db; sB[2] += cz(a) * db;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            gA[d] = -p.G * rA * sB[d];
            gB[d] = -p.G * rB * sA[d];
        }
    }

    float Fp[3] = {0.f, 0.f, 0.f};
    unsigned bad = 0u;
    if (p.pstress != 0.0f && p.phase != 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float Tp[6], Tm[6];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int sg = side == 0 ? 1 : -1;
                int xn = x, yn = y, zn = z;
                if (i == 0) xn = wrap1(x + sg, nx);
                if (i == 1) yn = y + sg;
                if (i == 2) zn = wrap1(z + sg, nz);
                float dv[6];
                float phi;
                if (yn >= 0 && yn < ny) {
                    const int64_t m = ((int64_t)zn * ny + yn) * nx + xn;
#pragma unroll
                    for (int k = 0; k < 6; ++k) dv[k] = D[k * N + m];
                    const float a_ = p.rho0[0] + mom[m];
                    const float b_ = p.nc == 2 ? p.rho0[1] + mom[N + m] : 0.0f;
                    phi = phase_phi(p, a_, b_);
                } else {
                    // linear extrapolation of C across the wall; phi copies the wall layer
                    const int y0 = yn < 0 ? 0 : ny - 1;
                    const int y1 = yn < 0 ? 1 : ny - 2;
                    const int64_t m0 = ((int64_t)zn * ny + y0) * nx + xn;
                    const int64_t m1 = ((int64_t)zn * ny + y1) * nx + xn;
#pragma unroll
                    for (int k = 0; k < 6; ++k) dv[k] = 2.0f * D[k * N + m0] - D[k * N + m1];
                    const float a_ = p.rho0[0] + mom[m0];
                    const float b_ = p.nc == 2 ? p.rho0[1] + mom[N + m0] : 0.0f;
                    phi = phase_phi(p, a_, b_);
                }
                if (side == 0) stress(p, dv, phi, Tp, bad);
                else stress(p, dv, phi, Tm, bad);
            }
#pragma unroll
            for (int jd = 0; jd < 3; ++jd) Fp[jd] += 0.5f * (Tp[sidx(i, jd)] - Tm[sidx(i, jd)]);
        }
    }

    // with the stress coupling the polymer acts through the equilibrium, not as a force (the
    // stresses above are still evaluated for the fault checks)
    if (p.coupling != 0) Fp[0] = Fp[1] = Fp[2] = 0.0f;
    const float inv_rho = 1.0f / rho;
    const float shA = rA * inv_rho, shB = rB * inv_rho;
    float FA[3], FB[3], u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        FA[d] = gA[d] + shA * Fp[d];
        FB[d] = gB[d] + shB * Fp[d];
        u[d] = (j[d] + 0.5f * (FA[d] + FB[d])) * inv_rho;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        uF[d * N + n] = u[d];
        uF[(3 + d) * N + n] = FA[d];
        if (p.nc == 2) uF[(6 + d) * N + n] = FB[d];
    }
    if (bad) atomicOr(flags, bad);
}

// FENE-P update of C = I + D at node n (Sec. 2, eq. FENE): velocity gradient G_ij = d_i u_j by
// central differences of the velocity field uF[0..2] (wall ghosts 2 u_w - u), first-order
// upwind advection and forward Euler (FENE = 0), or the paper's integrator (FENE = 1:
// central advection, artificial diffusivity, the rate taken through the Cholesky factor of
// f C with Adams-Bashforth 2; history in ab / abn).  Ghost C across a wall by linear
// extrapolation.  Writes the new D to dnew (and the rate history to abn) and returns the
// fault bits raised on the way (2: tr C reached L^2, 4: the Cholesky factor failed).
template <int FENE>
__device__ __forceinline__ unsigned fenep_node(const DevParams& p, int64_t n, int x, int y, int z, int xp, int xm,
                                               int zp, int zm, const float u[3], const float* __restrict__ uF,
                                               const float* __restrict__ D, const float* __restrict__ ab,
                                               float* __restrict__ abn, float dnew[6]) {
    const int64_t N = p.N;
    const int nx = p.nx, ny = p.ny;
    float d0[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) d0[k] = D[k * N + n];
    float Gm[3][3];
    float adv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // neighbours along axis i
        int64_t mp, mm;
        float up[3], um[3];
        if (i == 0) {
            mp = ((int64_t)z * ny + y) * nx + xp;
            mm = ((int64_t)z * ny + y) * nx + xm;
        } else if (i == 2) {
            mp = ((int64_t)zp * ny + y) * nx + x;
            mm = ((int64_t)zm * ny + y) * nx + x;
        } else {
            // at a wall the ghost replaces the neighbour; keep the index in bounds anyway
            mp = y == ny - 1 ? n : n + nx;
            mm = y == 0 ? n : n - nx;
        }
        const bool top = (i == 1) && (y == ny - 1);
        const bool bot = (i == 1) && (y == 0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            up[d] = top ? 2.0f * p.ut[d] - u[d] : uF[d * N + mp];
            um[d] = bot ? 2.0f * p.ub[d] - u[d] : uF[d * N + mm];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) Gm[i][d] = 0.5f * (up[d] - um[d]);
        if constexpr (FENE == 1) {
            // second-order central difference and the artificial diffusivity (ghosts at
            // the walls by linear extrapolation)
            float dpl[6], dmi[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                dpl[k] = top ? 2.0f * d0[k] - D[k * N + n - nx] : D[k * N + mp];
                dmi[k] = bot ? 2.0f * d0[k] - D[k * N + n + nx] : D[k * N + mm];
                adv[k] += u[i] * (0.5f * (dpl[k] - dmi[k])) - p.kappa * (dpl[k] - 2.0f * d0[k] + dmi[k]);
            }
            continue;
        }
        // first-order upwind difference of D along i
        float dn[6];
        if (u[i] >= 0.0f) {
            if (bot) {
#pragma unroll
                for (int k = 0; k < 6; ++k) dn[k] = 2.0f * d0[k] - D[k * N + n + nx];
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) dn[k] = D[k * N + mm];
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) adv[k] += u[i] * (d0[k] - dn[k]);
        } else {
            if (top) {
#pragma unroll
                for (int k = 0; k < 6; ++k) dn[k] = 2.0f * d0[k] - D[k * N + n - nx];
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) dn[k] = D[k * N + mp];
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) adv[k] += u[i] * (dn[k] - d0[k]);
        }
    }
    unsigned bad = 0u;
    const float trd = d0[0] + d0[1] + d0[2];
    const float den = p.L2m3 - trd;
    if (!(den > 0.0f)) bad |= 2u;
    const float inv = 1.0f / den;
    const float f = p.L2m3 * inv;
    const float fm1 = trd * inv;
    float rate[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = a; b < 3; ++b) {
            const int kk = sidx(a, b);
            // (G^T C + C G)_ab with C = I + D
            float st = Gm[b][a] + Gm[a][b];
#pragma unroll
            for (int k = 0; k < 3; ++k) st += Gm[k][a] * d0[sidx(k, b)] + d0[sidx(a, k)] * Gm[k][b];
            const float relax = (f * d0[kk] + (a == b ? fm1 : 0.0f)) * p.inv_tau_p;
            rate[kk] = -adv[kk] + st - relax;
            dnew[kk] = d0[kk] + rate[kk];
        }
    }
    if (FENE == 1 && !(bad & 2u)) {
        // the paper's integrator: the same rate, taken through the Cholesky factor of f C
        float yp[6], dn6[6], yd[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) yp[k] = p.ab_hist ? ab[k * N + n] : 0.0f;
        if (cholesky_ab2_step(p.L2, p.L2m3, d0, rate, yp, p.ab_hist != 0, dn6, yd)) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                dnew[k] = dn6[k];
                abn[k * N + n] = yd[k];
            }
        } else {
            bad |= 4u;
        }
    }
    return bad;
}

// Fault bits of a node's new state (S11): 1 non-finite (`check` sums every new value of the
// node), 2 tr C >= L^2, 4 a leading principal minor of C = I + dnew not positive.
__device__ __forceinline__ unsigned new_state_faults(const DevParams& p, const float dnew[6], float check) {
    unsigned bad = 0u;
    if (!isfinite(check)) bad |= 1u;
    const float c0 = 1.0f + dnew[0], c1 = 1.0f + dnew[1], c2 = 1.0f + dnew[2];
    if (!(c0 + c1 + c2 < p.L2)) bad |= 2u;
    const float m2 = c0 * c1 - dnew[3] * dnew[3];
    const float m3 = c0 * (c1 * c2 - dnew[5] * dnew[5]) - dnew[3] * (dnew[3] * c2 - dnew[5] * dnew[4]) +
                     dnew[4] * (dnew[3] * dnew[5] - c1 * dnew[4]);
    if (!(c0 > 0.0f && m2 > 0.0f && m3 > 0.0f)) bad |= 4u;
    return bad;
}

// COLL: 0 BGK, 1 MRT; FENE: 0 upwind/Euler, 1 the Cholesky-log AB2 integrator.  Each option
// pair is its own instantiation, so the default BGK body keeps the register budget of the
// plain scheme.  Two workgroups per CU at least (the MRT body keeps E + S/2 of the 19
// directions between its two loops and must stay within 256 registers).
template <int COLL, int FENE>
__global__ __launch_bounds__(kBlock, 2) void k_collide(DevParams p, const float* __restrict__ h,
                                                    float* __restrict__ hn,
                                                    const float* __restrict__ D,
                                                    float* __restrict__ Dn,
                                                    const float* __restrict__ uF,
                                                    const float* __restrict__ ab,
                                                    float* __restrict__ abn,
                                                    unsigned* __restrict__ flags) {
    const int64_t n = node_id();
    if (n >= p.N) return;
    const int64_t N = p.N;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int x = (int)(n % nx);
    const int64_t r = n / nx;
    const int y = (int)(r % ny);
    const int z = (int)(r / ny);

    const float u[3] = {uF[n], uF[N + n], uF[2 * N + n]};
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    // densities of both components first (needed for phi and the local tau)
    float dr[2] = {0.f, 0.f};
    {
        float jx = 0.f, jy = 0.f, jz = 0.f;
        for (int s = 0; s < p.nc; ++s) pop_moments(h + (int64_t)s * kQ * N, N, n, dr[s], jx, jy, jz);
    }
    const float rA = p.rho0[0] + dr[0];
    const float rB = p.nc == 2 ? p.rho0[1] + dr[1] : 0.0f;
    float tau = p.tauA;
    if (p.nc == 2) {
        const float phi = (rA - rB) / (rA + rB);
        const float fp = 0.5f * (1.0f + tanhf(phi * p.inv_delta));
        tau = p.tauB + (p.tauA - p.tauB) * fp;
    }
    const float om = 1.0f / tau;
    const float cf = 1.0f - 0.5f * om;
    // stress coupling (eq. MODEtransformation): T at this node, shared by rho_s/rho below
    float T[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const bool stress_eq = p.coupling == 1 && p.pstress != 0.0f;
    if (stress_eq) {
        float dv[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) dv[k] = D[k * N + n];
        unsigned bad_own = 0u;
        stress(p, dv, phase_phi(p, rA, rB), T, bad_own);
    }

    // destination row offsets (push streaming); -1 marks a link that leaves through a wall
    const int xp = wrap1(x + 1, nx), xm = wrap1(x - 1, nx);
    const int zp = wrap1(z + 1, nz), zm = wrap1(z - 1, nz);
    float check = 0.0f;

    for (int s = 0; s < p.nc; ++s) {
        const float* hs = h + (int64_t)s * kQ * N;
        float* hns = hn + (int64_t)s * kQ * N;
        const float rs = s == 0 ? rA : rB;
        const float drs = dr[s];
        const float F[3] = {uF[(3 + 3 * s) * N + n], uF[(4 + 3 * s) * N + n], uF[(5 + 3 * s) * N + n]};
        const float uFd = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        const float share = rs / (rA + rB);
        float Ts[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) Ts[k] = share * T[k];
        const float trs3 = (Ts[0] + Ts[1] + Ts[2]) * (1.0f / 3.0f);
        // push streaming of one post-collision population, bounce-back at the walls
        auto emit = [&](int a, float post) {
            const int yd = y + cy(a);
            if (yd >= 0 && yd < ny) {
                const int xd = cx(a) == 0 ? x : (cx(a) > 0 ? xp : xm);
                const int zd = cz(a) == 0 ? z : (cz(a) > 0 ? zp : zm);
                hns[a * N + ((int64_t)zd * ny + yd) * nx + xd] = post;
            } else {
                const float* uw = yd < 0 ? p.ub : p.ut;
                hns[opp(a) * N + n] = post - 6.0f * wgt(a) * rs * wall_cu(a, uw);
            }
        };
        // equilibrium (with the stress term of eq. MODEtransformation) and source of direction
        // a, and E + S/2 with S/2 joined to the even part before its one rounding (a small
        // term added to a part already rounded is dropped when below half an ulp of it)
        auto eq_src = [&](int a, float& heq, float& src, float& base) {
            const float cu = cx(a) * u[0] + cy(a) * u[1] + cz(a) * u[2];
            const float cF = cx(a) * F[0] + cy(a) * F[1] + cz(a) * F[2];
            const Wt w = wsplit(a);
            // even part, then the odd part 3 w rho (c.u) with rho (c.u) carried exactly
            // (rc + rce) and rounded once, as in the tile body
            const float rc = rs * cu;
            const float rce = fmaf(rs, cu, -rc);
            // the even part with the stress term of eq. MODEtransformation, rounded once
            float st = 0.0f;
            if (stress_eq) {
                const float cTc = float(cx(a) * cx(a)) * Ts[0] + float(cy(a) * cy(a)) * Ts[1] +
                                  float(cz(a) * cz(a)) * Ts[2] +
                                  2.0f * (float(cx(a) * cy(a)) * Ts[3] + float(cx(a) * cz(a)) * Ts[4] +
                                          float(cy(a) * cz(a)) * Ts[5]);
                st = -4.5f * wgt(a) * (cTc - trs3);
            }
            const float xe = drs + rs * (4.5f * cu * cu - 1.5f * uu);
            const float eo = fmaf(w.w3, rc, fmaf(w.w3, rce, w.w3l * rc));
            heq = fmaf(w.w, xe, fmaf(w.wl, xe, st)) + eo;
            src = wmul(w.w, w.wl, 3.0f * (cF - uFd) + 9.0f * cu * cF);
            base = fmaf(w.w, xe, fmaf(w.wl, xe, fmaf(0.5f, src, st))) + eo;
        };
        if constexpr (COLL == 1) {
            // MRT (Sec. 2): with every rate 1 except the bulk and shear modes (rate om), the
            // collision f - T^-1 Lambda T (f - E) + T^-1 (I - Lambda/2) T S reduces to
            //   f* = E + S/2 + (1 - om) P2 (f - E + S/2),
            // P2 the orthogonal projection on the modes e, 3p_xx, p_ww, p_xy, p_yz, p_xz of
            // the D3Q19 basis (rows 19c^2 - 30, 3c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_y c_z,
            // c_x c_z; squared norms 2394, 36, 12, 4, 4, 4)
            // E + S/2 as `base`, the mode sum added to it once
            float base[kQ];
            float pe = 0.f, pxx = 0.f, pww = 0.f, pxy = 0.f, pyz = 0.f, pxz = 0.f;
#pragma unroll
            for (int a = 0; a < kQ; ++a) {
                float heq, src;
                eq_src(a, heq, src, base[a]);
                const float ha = hs[a * N + n];
                const float g = (ha - base[a]) + src;  // f - E + S/2
                const int c2 = cx(a) * cx(a) + cy(a) * cy(a) + cz(a) * cz(a);
                pe += float(19 * c2 - 30) * g;
                if (3 * cx(a) * cx(a) - c2 != 0) pxx += float(3 * cx(a) * cx(a) - c2) * g;
                if (cy(a) * cy(a) - cz(a) * cz(a) != 0) pww += float(cy(a) * cy(a) - cz(a) * cz(a)) * g;
                if (cx(a) * cy(a) != 0) pxy += float(cx(a) * cy(a)) * g;
                if (cy(a) * cz(a) != 0) pyz += float(cy(a) * cz(a)) * g;
                if (cx(a) * cz(a) != 0) pxz += float(cx(a) * cz(a)) * g;
            }
            const float k2 = 1.0f - om;
            pe *= k2 * (1.0f / 2394.0f);
            pxx *= k2 * (1.0f / 36.0f);
            pww *= k2 * (1.0f / 12.0f);
            pxy *= k2 * 0.25f;
            pyz *= k2 * 0.25f;
            pxz *= k2 * 0.25f;
#pragma unroll
            for (int a = 0; a < kQ; ++a) {
                const int c2 = cx(a) * cx(a) + cy(a) * cy(a) + cz(a) * cz(a);
                float r = float(19 * c2 - 30) * pe;
                if (3 * cx(a) * cx(a) - c2 != 0) r += float(3 * cx(a) * cx(a) - c2) * pxx;
                if (cy(a) * cy(a) - cz(a) * cz(a) != 0) r += float(cy(a) * cy(a) - cz(a) * cz(a)) * pww;
                if (cx(a) * cy(a) != 0) r += float(cx(a) * cy(a)) * pxy;
                if (cy(a) * cz(a) != 0) r += float(cy(a) * cz(a)) * pyz;
                if (cx(a) * cz(a) != 0) r += float(cx(a) * cz(a)) * pxz;
                const float post = base[a] + r;
                check += post;
                emit(a, post);
            }
        } else {
            // all 19 loads are issued before the first store (interleaving them per
            // direction leaves few loads in flight)
            float hv[kQ];
#pragma unroll
            for (int a = 0; a < kQ; ++a) hv[a] = hs[a * N + n];
#pragma unroll
            for (int a = 0; a < kQ; ++a) {
                const float ha = hv[a];
                float heq, src, base;
                eq_src(a, heq, src, base);
                // the increment first, added to h once: a small term added to a value already
                // rounded at the scale of h is dropped when below half an ulp of it
                const float post = ha + fmaf(cf, src, -om * (ha - heq));
                check += post;
                emit(a, post);
            }
        }
    }

    // ---- FENE-P step on C = I + D ----
    float dnew[6];
    unsigned bad = fenep_node<FENE>(p, n, x, y, z, xp, xm, zp, zm, u, uF, D, ab, abn, dnew);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        Dn[k * N + n] = dnew[k];
        check += dnew[k];
    }
    bad |= new_state_faults(p, dnew, check);
    if (bad) atomicOr(flags, bad);
}

// Prescribed-velocity ("kinematic") FENE-P step: the lattice-Boltzmann part is not run; the
// velocity field uF[0..2] is given and held fixed, and only the FENE-P update above advances
// C (the homogeneous benchmarks of Sec. 3 prescribe the flow and switch the feedback off).
template <int FENE>
__global__ __launch_bounds__(kBlock) void k_fenep_kinematic(DevParams p, const float* __restrict__ uF,
                                                            const float* __restrict__ D,
                                                            float* __restrict__ Dn,
                                                            const float* __restrict__ ab,
                                                            float* __restrict__ abn,
                                                            unsigned* __restrict__ flags) {
    const int64_t n = node_id();
    if (n >= p.N) return;
    const int64_t N = p.N;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int x = (int)(n % nx);
    const int64_t r = n / nx;
    const int y = (int)(r % ny);
    const int z = (int)(r / ny);
    const float u[3] = {uF[n], uF[N + n], uF[2 * N + n]};
    const int xp = wrap1(x + 1, nx), xm = wrap1(x - 1, nx);
    const int zp = wrap1(z + 1, nz), zm = wrap1(z - 1, nz);
    float dnew[6];
    unsigned bad = fenep_node<FENE>(p, n, x, y, z, xp, xm, zp, zm, u, uF, D, ab, abn, dnew);
    float check = 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        Dn[k * N + n] = dnew[k];
        check += dnew[k];
    }
    bad |= new_state_faults(p, dnew, check);
    if (bad) atomicOr(flags, bad);
}

__global__ void k_clear_flags(unsigned* flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) flags[0] = 0u;
}

__global__ void k_set_flags(unsigned* flags, unsigned v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) flags[0] = v;
}

static inline dim3 grid_for(int64_t N) { return dim3((unsigned)((N + kBlock - 1) / kBlock)); }

hipError_t launch_moments(const DevParams& p, const Buffers& b, hipStream_t s) {
    hipLaunchKernelGGL(k_moments, grid_for(p.N), dim3(kBlock), 0, s, p, b.h, b.mom);
    return hipGetLastError();
}
hipError_t launch_forces(const DevParams& p, const Buffers& b, hipStream_t s) {
    hipLaunchKernelGGL(k_forces, grid_for(p.N), dim3(kBlock), 0, s, p, b.mom, b.D, b.uF, b.flags);
    return hipGetLastError();
}
hipError_t launch_collide(const DevParams& p, const Buffers& b, hipStream_t s) {
    const auto k = p.collision == 1 ? (p.fene == 1 ? k_collide<1, 1> : k_collide<1, 0>)
                                    : (p.fene == 1 ? k_collide<0, 1> : k_collide<0, 0>);
    hipLaunchKernelGGL(k, grid_for(p.N), dim3(kBlock), 0, s, p, b.h, b.hn, b.D, b.Dn, b.uF, b.ab, b.ab_next,
                       b.flags);
    return hipGetLastError();
}
hipError_t launch_fenep_kinematic(const DevParams& p, const float* uF, const float* D, float* Dn, const float* ab,
                                  float* abn, unsigned* flags, hipStream_t s) {
    const auto k = p.fene == 1 ? k_fenep_kinematic<1> : k_fenep_kinematic<0>;
    hipLaunchKernelGGL(k, grid_for(p.N), dim3(kBlock), 0, s, p, uF, D, Dn, ab, abn, flags);
    return hipGetLastError();
}
hipError_t launch_set_flags(const Buffers& b, unsigned v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, s, b.flags, v);
    return hipGetLastError();
}
hipError_t launch_clear_flags(const Buffers& b, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, b.flags);
    return hipGetLastError();
}

}  // namespace lbfd

// k_fused.hip -- the whole hybrid LB/FD time step in ONE pass over HBM (gfx950).
//
// Each workgroup owns a TX x TY column of the (x, y) plane and marches along z through a
// chunk of planes.  Per plane q entering the tile it
//   A  reads the populations and C of plane q on the tile plus a 2-node halo, forms
//      delta rho_s, j (Sec. 2, moments), the order parameter and the polymer-stress
//      coefficients s = (eta_p/tau_p) m(phi) f(r), s1 = (eta_p/tau_p) m(phi) (f(r) - 1), so
//      T = s (C - I) + s1 I (FENE-P feedback modulated by f+-(phi)), into LDS rings;
//   B  computes, for plane q-1 on the tile plus a 1-node halo, the Shan-Chen force
//      (eq. SCforce), the central divergence of T, the species split F_s = g_s +
//      (rho_s/rho) F_p and the half-force velocity u (eq. equilibrium:vel);
//   C  collides plane q-1 (BGK with the forcing source, eq. LB with Lambda = I/tau(phi);
//      in the chained body, the multiple-relaxation-time collision of Sec. 2 as an option)
//      and pushes the post-collision populations to their neighbours, bouncing links that
//      leave through a wall back with the moving-wall correction;
//   D  advances C on plane q-2 with the explicit FENE-P update (eq. FENE): first-order
//      upwind advection, G^T C + C G with central G_ij = d_i u_j, Peterlin relaxation (in
//      the chained body, the Cholesky-log Adams-Bashforth-2 integrator of Sec. 2 with
//      central differences and artificial diffusivity as an option).
// Every stage reads time level n only, so HBM sees each population and C component read
// once and written once per step: 2 x ncomp x 19 x 4 + 2 x 6 x 4 bytes per node.  The halo
// re-reads of neighbouring tiles are meant to hit a cache: blocks are mapped so that the
// tiles running together on one XCD form a compact group and the groups running together
// on the chip form a band (tile_of_block).
//
// Ghost rules at the y walls (same as the host-visible definition of the method):
// densities copy the wall layer, C is extrapolated linearly, u is reflected through the
// wall velocity; x and z are periodic.
#include "d3q19.h"
#include "fene_chol.h"
#include "lbfd_internal.h"

namespace lbfd {

namespace {

__device__ __forceinline__ int64_t xcd_remap_f(int64_t b, int64_t nb) {
    const int64_t per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// Block -> (x tile, y tile, z chunk).  The hardware hands block b to XCD b % 8 and each
// XCD starts its blocks in order, 32 at a time (one per CU at this kernel's occupancy).
// Generation g of 256 blocks (32 per XCD) gets 256 consecutive logical indices, XCD k the
// k-th run of 32; logical indices walk groups of gxw x gyh tiles (x fastest inside a
// group, groups x-fastest, then group rows, then z chunks).  A tile's halo lines are then
// the own lines of tiles that run at the same time on the same XCD (L2) or on a
// neighbouring one (memory-side cache) instead of lines last touched a generation ago.
// Blocks beyond the last whole generation keep their index.  The map is a bijection.
__device__ __forceinline__ void tile_of_block(int64_t b, int64_t nb, int ntx, int nty, int gxw, int gyh, int& tx,
                                              int& ty, int& zc) {
    int64_t L = b;
    const int64_t full = nb - nb % 256;
    if (b < full) {
        const int64_t slot = b >> 3;
        L = (slot >> 5) * 256 + (b & 7) * 32 + (slot & 31);
    }
    const int64_t per = (int64_t)ntx * nty;
    zc = (int)(L / per);
    int64_t r = L - (int64_t)zc * per;
    const int64_t rowsz = (int64_t)ntx * gyh;
    const int gyi = (int)(r / rowsz);
    r -= (int64_t)gyi * rowsz;
    const int h = min(gyh, nty - gyi * gyh);
    const int gxi = (int)(r / ((int64_t)gxw * h));
    r -= (int64_t)gxi * gxw * h;
    const int w = min(gxw, ntx - gxi * gxw);
    tx = gxi * gxw + (int)(r % w);
    ty = gyi * gyh + (int)(r / w);
}

__device__ __forceinline__ int wrapn(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Workgroup barrier for LDS only.  __syncthreads() also waits for every outstanding
// global access (vmcnt(0)), which would drain the prefetch of the next plane; this kernel
// never reads global data written by another thread of the same launch, so completing the
// LDS operations (lgkmcnt(0)) before s_barrier is all the ordering it needs.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// R2 halo position k (0 <= k < 4*TX + 4*TY + 16) -> local (lx, ly) in [-2, TX+2) x [-2, TY+2)
template <int TX, int TY>
__device__ __forceinline__ void halo2_pos(int k, int& lx, int& ly) {
    constexpr int W2 = TX + 4;
    if (k < 2 * W2) {
        ly = k / W2 - 2;
        lx = k % W2 - 2;
    } else if (k < 4 * W2) {
        k -= 2 * W2;
        ly = TY + k / W2;
        lx = k % W2 - 2;
    } else {
        k -= 4 * W2;
        ly = k >> 2;
        const int c = k & 3;
        lx = c < 2 ? c - 2 : TX + c - 2;
    }
}

// R1 halo position k (0 <= k < 2*TX + 2*TY + 4) -> local (lx, ly) in [-1, TX+1) x [-1, TY+1)
template <int TX, int TY>
__device__ __forceinline__ void halo1_pos(int k, int& lx, int& ly) {
    constexpr int W1 = TX + 2;
    if (k < W1) {
        ly = -1;
        lx = k - 1;
    } else if (k < 2 * W1) {
        ly = TY;
        lx = k - W1 - 1;
    } else {
        k -= 2 * W1;
        ly = k >> 1;
        lx = (k & 1) ? TX : -1;
    }
}

}  // namespace

// LDS of one workgroup.  TP (two-pass step): the moments come from a preceding pass, so
// the per-component momenta and the ring of own populations are not needed (size 1).
// MO (chained two-pass step): the tile also forms the moments of the next time level; the
// partial moments that cross from one row of the tile to the next pass through X, which
// shares its storage with the species forces (they are dead between phase C and phase B).
template <int NC, int TX, int TY, bool TP, bool MO = false>
struct FusedTile {
    static constexpr int NT = TX * TY;    // nodes per tile
    static constexpr int NTH = NC * NT;   // threads: one per (node, component)
    static constexpr int W2 = TX + 4, H2 = TY + 4, A2 = W2 * H2;
    static constexpr int W1 = TX + 2, H1 = TY + 2, A1 = W1 * H1;
    static constexpr int NH2 = A2 - NT;  // R2 halo nodes
    static constexpr int NH1 = A1 - NT;  // R1 halo nodes
    static constexpr int NFO = NC * 3 * A1;                     // species forces
    static constexpr int NXR = NC * 8 * NT;                     // row exchange: 8 values per (node, comp)
    static constexpr int NXJ = NFO + 3 * NT;                    // forces + the momentum of one component
    static constexpr int NX = !MO ? 1 : (NXR > NXJ ? NXR : NXJ);
    float rho[3][NC][A2];       // delta rho per component (ring over planes)
    float cs[3][8][A2];         // D = C - I (6), s, s1 (ring over planes)
    float u[3][3][A1];          // total j (after A2), u (after B) (ring over planes)
    union {
        float Fo[NC][3][A1];    // species forces on the tile + 1-node halo, phase B -> C
        float X[NX];            // MO: row exchange after phase C; momentum of one component in A2 -> B
    };
    float fpl[2][A1];           // f+(phi) on the tile + 1-node halo, planes q and q-1
    float jc[TP ? 1 : NC][3][TP ? 1 : A1];                  // momentum per component
    float pop[TP ? 1 : 2][TP ? 1 : NC][kQ][TP ? 1 : NT];     // own populations, planes q, q-1
};

// Populations of one component and (optionally) D of one node, as loaded.
struct NodeLoad {
    float f[kQ];
    float d[6];
};

// A field is addressed as a wave-uniform base plus a 32-bit byte offset (grids hold fewer
// than 2^30 nodes), which keeps addresses out of 64-bit vector arithmetic.
__device__ __forceinline__ float ld_off(const float* __restrict__ base, uint32_t boff) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + boff);
}
__device__ __forceinline__ void st_off(float* __restrict__ base, uint32_t boff, float v) {
    // streaming store: the next step reads it, this launch does not
    __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + boff));
}

__device__ __forceinline__ void issue_load(const float* __restrict__ hs, const float* __restrict__ D, uint32_t N,
                                           uint32_t n, bool with_d, NodeLoad& v) {
    const uint32_t bo = n * 4u;
#pragma unroll
    for (int a = 0; a < kQ; ++a) v.f[a] = ld_off(hs + (size_t)a * N, bo);
    if (with_d) {
#pragma unroll
        for (int k = 0; k < 6; ++k) v.d[k] = ld_off(D + (size_t)k * N, bo);
    }
}

// Phase A1 for one (node, component) of plane q: delta rho and momentum of this component,
// D when with_d, and for an own node the populations themselves (collided one plane
// later).  Positions beyond a wall hold the wall layer's values (densities copy the wall
// layer; C and the stress are replaced in phase A2).
template <int NC, int TX, int TY, bool OWN>
__device__ __forceinline__ void phase_a1(FusedTile<NC, TX, TY, false>& L, int sq, int s2, int c, int nid, int lx, int ly,
                                         bool with_d, const NodeLoad& v) {
    using T = FusedTile<NC, TX, TY, false>;
    float sum = v.f[0];
#pragma unroll
    for (int a = 1; a < kQ; a += 2) sum += v.f[a] + v.f[a + 1];
    float jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int a = 1; a < kQ; a += 2) {
        const float d = v.f[a] - v.f[a + 1];
        jx += cx(a) * d;
        jy += cy(a) * d;
        jz += cz(a) * d;
    }
    const int i2 = (ly + 2) * T::W2 + lx + 2;
    L.rho[sq][c][i2] = sum;
    if (with_d) {
#pragma unroll
        for (int k = 0; k < 6; ++k) L.cs[sq][k][i2] = v.d[k];
    }
    if (lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) {
        const int i1 = (ly + 1) * T::W1 + lx + 1;
        L.jc[c][0][i1] = jx;
        L.jc[c][1][i1] = jy;
        L.jc[c][2][i1] = jz;
    }
    if (OWN) {
#pragma unroll
        for (int a = 0; a < kQ; ++a) L.pop[s2][c][a][nid] = v.f[a];
    }
}

// Phase A2 for one R2 position of plane q: wall ghosts of C (linear extrapolation from the
// two wall-adjacent layers, Sec. 2 boundary condition of C), f+(phi), the stress
// coefficients s = (eta_p/tau_p) m(phi) f(r), s1 = (eta_p/tau_p) m(phi) (f(r) - 1), and the
// total momentum.
template <int NC, int TX, int TY, bool TP, class TL>
__device__ __forceinline__ void phase_a2(const DevParams& p, TL& L, int sq, int s2, int y0, int k,
                                         unsigned& bad) {
    using T = FusedTile<NC, TX, TY, TP>;
    const int lx = k % T::W2 - 2, ly = k / T::W2 - 2;
    const int gy = y0 + ly;
    const int i2 = k;
    float dv[6];
    if (gy == -1 || gy == p.ny) {
        const int lyw = gy < 0 ? ly + 1 : ly - 1;  // wall layer
        const int lyi = gy < 0 ? ly + 2 : ly - 2;  // next layer inwards
        const int iw = (lyw + 2) * T::W2 + lx + 2, ii = (lyi + 2) * T::W2 + lx + 2;
#pragma unroll
        for (int c = 0; c < 6; ++c) dv[c] = 2.0f * L.cs[sq][c][iw] - L.cs[sq][c][ii];
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) dv[c] = L.cs[sq][c][i2];
    }
    float phi = 1.0f;
    if (NC == 2) {
        const float ra = p.rho0[0] + L.rho[sq][0][i2];
        const float rb = p.rho0[1] + L.rho[sq][NC - 1][i2];
        phi = (ra - rb) / (ra + rb);
    }
    // f+-(phi) = (1 +- tanh(phi/Delta))/2 (Sec. 2, smoothing of the viscosity and of the
    // polymer feedback)
    const float th = (NC == 2 || p.phase == 1 || p.phase == 2) ? tanhf(phi * p.inv_delta) : 0.0f;
    float m = 0.0f;
    if (p.phase == 3) m = 1.0f;
    else if (p.phase == 1) m = 0.5f * (1.0f + th);
    else if (p.phase == 2) m = 0.5f * (1.0f - th);
    const float trd = dv[0] + dv[1] + dv[2];
    const float den = p.L2m3 - trd;
    if (!(den > 0.0f) && gy >= -1 && gy <= p.ny) bad |= 2u;
    const float inv = 1.0f / den;
    const float pm = p.pstress * m;
    // ghost rows are written only by this thread and read after the next barrier
    if (gy == -1 || gy == p.ny) {
#pragma unroll
        for (int c = 0; c < 6; ++c) L.cs[sq][c][i2] = dv[c];
    }
    L.cs[sq][6][i2] = pm * p.L2m3 * inv;
    L.cs[sq][7][i2] = pm * trd * inv;
    if (NC == 2 && lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) L.fpl[s2][(ly + 1) * T::W1 + lx + 1] = 0.5f * (1.0f + th);
    if (!TP && lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) {
        const int i1 = (ly + 1) * T::W1 + lx + 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) L.u[sq][d][i1] = NC == 2 ? L.jc[0][d][i1] + L.jc[NC - 1][d][i1] : L.jc[0][d][i1];
    }
}

// Phase B for one in-domain node of plane q-1 at local (lx, ly): Shan-Chen force, polymer
// stress divergence, species forces and velocity; u replaces j in LDS slot sr.
template <int NC, int TX, int TY, bool TP, class TL>
__device__ __forceinline__ void phase_b(const DevParams& p, TL& L, int sp, int sr,
                                        int sn, int lx, int ly, float (&Fs)[2][3]) {
    using T = FusedTile<NC, TX, TY, TP>;
    const int i2 = (ly + 2) * T::W2 + lx + 2;
    const int i1 = (ly + 1) * T::W1 + lx + 1;
    float rs[2];
    rs[0] = p.rho0[0] + L.rho[sr][0][i2];
    rs[1] = NC == 2 ? p.rho0[1] + L.rho[sr][NC - 1][i2] : 0.0f;
    const float rho = rs[0] + rs[1];
    float g[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    if (NC == 2 && p.G != 0.0f) {
        float sA[3] = {0.f, 0.f, 0.f}, sB[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 1; a < kQ; a += 2) {
            const int slp = cz(a) > 0 ? sn : (cz(a) < 0 ? sp : sr);
            const int slm = cz(a) > 0 ? sp : (cz(a) < 0 ? sn : sr);
            const int ip = i2 + cy(a) * T::W2 + cx(a);
            const int im = i2 - cy(a) * T::W2 - cx(a);
            const float da = wgt(a) * (L.rho[slp][0][ip] - L.rho[slm][0][im]);
            const float db = wgt(a) * (L.rho[slp][NC - 1][ip] - L.rho[slm][NC - 1][im]);
            sA[0] += cx(a) * da;
            sA[1] += cy(a) * da;
            sA[2] += cz(a) * da;
            sB[0] += cx(a) * db;
            sB[1] += cy(a) * db;
            sB[2] += cz(a) * db;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g[0][d] = -p.G * rs[0] * sB[d];
            g[1][d] = -p.G * rs[1] * sA[d];
        }
    }
    float Fp[3] = {0.f, 0.f, 0.f};
    if (p.pstress != 0.0f && p.coupling == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int slp = i == 2 ? sn : sr;
            const int slm = i == 2 ? sp : sr;
            const int off = i == 0 ? 1 : (i == 1 ? T::W2 : 0);
            const int ip = i2 + off, im = i2 - off;
            const float spp = L.cs[slp][6][ip], s1p = L.cs[slp][7][ip];
            const float smm = L.cs[slm][6][im], s1m = L.cs[slm][7][im];
#pragma unroll
            for (int jd = 0; jd < 3; ++jd) {
                const int k = sidx(i, jd);
                const float tp = spp * L.cs[slp][k][ip] + (k < 3 ? s1p : 0.0f);
                const float tm = smm * L.cs[slm][k][im] + (k < 3 ? s1m : 0.0f);
                Fp[jd] += 0.5f * (tp - tm);
            }
        }
    }
    const float inv_rho = 1.0f / rho;
    const float sh0 = rs[0] * inv_rho, sh1 = rs[1] * inv_rho;
    float u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Fs[0][d] = g[0][d] + sh0 * Fp[d];
        Fs[1][d] = g[1][d] + sh1 * Fp[d];
        u[d] = (L.u[sr][d][i1] + 0.5f * (Fs[0][d] + Fs[1][d])) * inv_rho;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) L.u[sr][d][i1] = u[d];
}

// Moments and D of one position of the tile + 2-node halo, as loaded (two-pass step).
template <int NC>
struct MomLoad {
    float r[NC];
    float j[3];
    float d[6];
};

// Node quantities the collision needs, read from LDS: velocity, species force, density,
// relaxation, and (stress coupling, eq. MODEtransformation) the species' share T_s of the
// polymer stress.
struct CollideIn {
    float u[3], F[3];
    float drs, rs, om, cfac, uF, b, trs3;
    float Ts[6];
    bool stress;
};

template <int NC, int TX, int TY, bool TP, class TL>
__device__ __forceinline__ CollideIn collide_in(const DevParams& p, TL& L, int sr, int p2,
                                                int comp, int i1, int i2) {
    // no FMA contraction in the collision helpers: the same node is collided by its own
    // lane in one launch shape and by a tile-edge lane of a neighbouring tile in another,
    // and contraction would depend on which results the caller uses
#pragma clang fp contract(off)
    CollideIn c;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c.u[d] = L.u[sr][d][i1];
        c.F[d] = L.Fo[comp][d][i1];
    }
    c.drs = L.rho[sr][comp][i2];
    c.rs = (comp == 0 ? p.rho0[0] : p.rho0[1]) + c.drs;
    const float uu = fmaf(c.u[2], c.u[2], fmaf(c.u[1], c.u[1], c.u[0] * c.u[0]));
    const float tau = NC == 2 ? fmaf(p.tauA - p.tauB, L.fpl[p2][i1], p.tauB) : p.tauA;
    c.om = 1.0f / tau;
    c.cfac = fmaf(-0.5f, c.om, 1.0f);
    c.uF = fmaf(c.u[2], c.F[2], fmaf(c.u[1], c.F[1], c.u[0] * c.F[0]));
    c.b = -1.5f * uu;
    c.stress = p.coupling == 1 && p.pstress != 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) c.Ts[k] = 0.0f;
    if (c.stress) {
        const float rtot = p.rho0[0] + L.rho[sr][0][i2] + (NC == 2 ? p.rho0[1] + L.rho[sr][NC - 1][i2] : 0.0f);
        const float share = c.rs / rtot;
        const float sv = share * L.cs[sr][6][i2], s1v = share * L.cs[sr][7][i2];
#pragma unroll
        for (int k = 0; k < 6; ++k) c.Ts[k] = k < 3 ? fmaf(sv, L.cs[sr][k][i2], s1v) : sv * L.cs[sr][k][i2];
    }
    c.trs3 = (c.Ts[0] + c.Ts[1] + c.Ts[2]) * (1.0f / 3.0f);
    return c;
}

// rest population: h + [(1 - 1/(2 tau)) S - (h - h_eq)/tau]
__device__ __forceinline__ float collide_rest(const CollideIn& c, float ha) {
#pragma clang fp contract(off)
    constexpr Wt w = wsplit(0);
    const float x0 = fmaf(c.rs, c.b, c.drs);
    const float heq0 = fmaf(w.w, x0, fmaf(w.wl, x0, c.stress ? 1.5f * c.trs3 : 0.0f));
    // the rest source is w_0 (-3 u.F) = -u.F exactly
    return ha + fmaf(c.cfac, -c.uF, -c.om * (ha - heq0));
}

// The odd part of the equilibrium of one direction, 3 w rho (c.u), rounded once: rho (c.u) is
// carried as the exact pair rc + rce (the product's rounding error recovered with an fma).  A
// steady node rounds this product the same way at every step, and the rounding of rho (c.u)
// alone acted as a fixed, node-by-node momentum source; the channel's slowest flow mode
// integrated it into a relative velocity error that grew to 1e-5 within a thousand steps of the
// 128 x 64 x 128 droplet.
// `extra` is a small term of the same parity that joins it before that rounding.
__device__ __forceinline__ float odd_equilibrium(const Wt& w, float rs, float cu, float extra = 0.0f) {
#pragma clang fp contract(off)
    const float rc = rs * cu;
    const float rce = fmaf(rs, cu, -rc);
    return fmaf(w.w3, rc, fmaf(w.w3, rce, fmaf(w.w3l, rc, extra)));
}

// The even part of the equilibrium of one direction, w (delta rho + rho (4.5 (c.u)^2 - 1.5
// u^2)), with the stress term of eq. MODEtransformation when that coupling is on, and a small
// even term `extra`, rounded once.
__device__ __forceinline__ float even_equilibrium(const CollideIn& c, float ex, float ey, float ez, const Wt& w,
                                                  float cu, float extra = 0.0f) {
#pragma clang fp contract(off)
    const float xe = fmaf(c.rs, fmaf(4.5f * cu, cu, c.b), c.drs);
    float lo = fmaf(w.wl, xe, extra);
    if (c.stress) {
        const float cTc = fmaf(ex * ex, c.Ts[0], fmaf(ey * ey, c.Ts[1], ez * ez * c.Ts[2])) +
                          2.0f * fmaf(ex * ey, c.Ts[3], fmaf(ex * ez, c.Ts[4], ey * ez * c.Ts[5]));
        lo = fmaf(-4.5f * w.w, cTc - c.trs3, lo);  // 4.5 w rounds to 1/4, 1/8 or 3/2 exactly
    }
    return fmaf(w.w, xe, lo);
}

// Opposite pair (a, a+1), c_{a+1} = -c_a, given c_a = (ex, ey, ez) and its weight w: the
// equilibrium and the source split into parts even and odd in c, formed once.  Each
// population is relaxed as h + [(1 - 1/(2 tau)) S - (h - h_eq)/tau]: the increment is formed
// first and added to h once.  In the form fma(1 - 1/(2 tau), S, h - (h - h_eq)/tau) the
// source was added to a value already rounded at the scale of h, and a source below half an
// ulp of h was dropped; it was dropped the same way at every step and in every plane of a
// sheared flow, so the lost force acted coherently and the channel's slowest mode integrated
// it.  Fixed fma pattern, contraction off: the result is the same whether c_a is a
// compile-time constant (own nodes) or a run-time value (the tile-edge lanes that collide a
// halo node's inbound directions).
__device__ __forceinline__ void collide_pair_c(const CollideIn& c, float ex, float ey, float ez, const Wt& w,
                                               float ha, float hb, float& pa, float& pb) {
#pragma clang fp contract(off)
    const float cu = fmaf(ez, c.u[2], fmaf(ey, c.u[1], ex * c.u[0]));
    const float cF = fmaf(ez, c.F[2], fmaf(ey, c.F[1], ex * c.F[0]));
    const float ee = even_equilibrium(c, ex, ey, ez, w, cu);             // equilibrium, even part
    const float eo = odd_equilibrium(w, c.rs, cu);                       // equilibrium, odd part
    const float se = wmul(w.w, w.wl, fmaf(9.0f * cu, cF, -3.0f * c.uF));  // source, even part
    const float so = wmul(w.w3, w.w3l, cF);                             // source, odd part
    pa = ha + fmaf(c.cfac, se + so, -c.om * (ha - (ee + eo)));
    pb = hb + fmaf(c.cfac, se - so, -c.om * (hb - (ee - eo)));
}

__device__ __forceinline__ void collide_pair(const CollideIn& c, int a, float ha, float hb, float& pa, float& pb) {
    collide_pair_c(c, float(cx(a)), float(cy(a)), float(cz(a)), wsplit(a), ha, hb, pa, pb);
}

// MRT collision (Sec. 2) with every rate 1 except the bulk and shear modes (rate 1/tau):
//   f* = E + S/2 + (1 - 1/tau) P2 (f - E + S/2),
// P2 the orthogonal projection on the modes e, 3p_xx, p_ww, p_xy, p_yz, p_xz of the D3Q19
// basis (rows 19c^2 - 30, 3c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_y c_z, c_x c_z; squared
// norms 2394, 36, 12, 4, 4, 4).  Mrt holds (1 - 1/tau) times the six projection
// coefficients of a node; every node is collided from all 19 of its populations, whichever
// tile does it, with the same fixed fma pattern (contraction off), so the values a halo
// collide forms are those of the node's own tile, bit for bit.
struct Mrt {
    float e, xx, ww, xy, yz, xz;
};

// the projection coefficients of a node from its 19 populations h.  The coefficients are
// moments of g = f - E + S/2 of order two and below, and the lattice's fourth-order
// isotropy gives those of E and S in closed form:
//   sum E = delta rho_s, sum E c_i c_j = delta rho_s / 3 d_ij + rho_s u_i u_j - T_s,ij,
//   sum S = 0,           sum S c_i c_j = u_i F_j + u_j F_i,
// so only the populations' own moments are summed.
__device__ __forceinline__ Mrt mrt_coef(const CollideIn& c, const float (&h)[kQ]) {
#pragma clang fp contract(off)
    float s0 = 0.f, sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, syz = 0.f, sxz = 0.f;
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        s0 += h[a];
        if (cx(a) != 0) sxx += h[a];
        if (cy(a) != 0) syy += h[a];
        if (cz(a) != 0) szz += h[a];
        if (cx(a) * cy(a) > 0) sxy += h[a];
        if (cx(a) * cy(a) < 0) sxy -= h[a];
        if (cy(a) * cz(a) > 0) syz += h[a];
        if (cy(a) * cz(a) < 0) syz -= h[a];
        if (cx(a) * cz(a) > 0) sxz += h[a];
        if (cx(a) * cz(a) < 0) sxz -= h[a];
    }
    constexpr Wt third = wsplit(0);  // 1/3 as a split weight
    const float d3 = wmul(third.w, third.wl, c.drs);
    const float* u = c.u;
    const float* F = c.F;
    const float gxx = (sxx - (fmaf(c.rs * u[0], u[0], d3) - c.Ts[0])) + u[0] * F[0];
    const float gyy = (syy - (fmaf(c.rs * u[1], u[1], d3) - c.Ts[1])) + u[1] * F[1];
    const float gzz = (szz - (fmaf(c.rs * u[2], u[2], d3) - c.Ts[2])) + u[2] * F[2];
    const float gxy = (sxy - (c.rs * u[0] * u[1] - c.Ts[3])) + 0.5f * fmaf(u[0], F[1], u[1] * F[0]);
    const float gxz = (sxz - (c.rs * u[0] * u[2] - c.Ts[4])) + 0.5f * fmaf(u[0], F[2], u[2] * F[0]);
    const float gyz = (syz - (c.rs * u[1] * u[2] - c.Ts[5])) + 0.5f * fmaf(u[1], F[2], u[2] * F[1]);
    const float g0 = s0 - c.drs;
    const float tr = (gxx + gyy) + gzz;
    const float k2 = 1.0f - c.om;
    return Mrt{fmaf(19.0f, tr, -30.0f * g0) * (k2 * (1.0f / 2394.0f)), fmaf(2.0f, gxx, -(gyy + gzz)) * (k2 * (1.0f / 36.0f)),
               (gyy - gzz) * (k2 * (1.0f / 12.0f)), gxy * (k2 * 0.25f), gyz * (k2 * 0.25f), gxz * (k2 * 0.25f)};
}

// Post-collision populations of the opposite pair c_a = (ex, ey, ez), c_b = -c_a (a run-time
// or compile-time direction: the rows are exact small integers either way).  The
// equilibrium and the source split into parts even and odd in c, and the mode sum
// (1 - 1/tau) P2 g is even in c, so the pair shares everything but the odd parts.  The small
// terms (the source and the mode sum) join each part before its one rounding: added to a
// part already rounded, a term below half an ulp of it would be dropped, the same way at
// every step.
__device__ __forceinline__ void mrt_pair_c(const CollideIn& c, const Mrt& m, float ex, float ey, float ez,
                                           const Wt& w, float& pa, float& pb) {
#pragma clang fp contract(off)
    const float cu = fmaf(ez, c.u[2], fmaf(ey, c.u[1], ex * c.u[0]));
    const float cF = fmaf(ez, c.F[2], fmaf(ey, c.F[1], ex * c.F[0]));
    const float se = wmul(w.w, w.wl, fmaf(9.0f * cu, cF, -3.0f * c.uF));  // source, even part
    const float so = wmul(w.w3, w.w3l, cF);                             // source, odd part
    const float c2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
    float r = fmaf(19.0f, c2, -30.0f) * m.e;
    r = fmaf(fmaf(3.0f * ex, ex, -c2), m.xx, r);
    r = fmaf(fmaf(ey, ey, -(ez * ez)), m.ww, r);
    r = fmaf(ex * ey, m.xy, r);
    r = fmaf(ey * ez, m.yz, r);
    r = fmaf(ex * ez, m.xz, r);
    const float ev = even_equilibrium(c, ex, ey, ez, w, cu, fmaf(0.5f, se, r));  // E + S/2 + r, even part
    const float od = odd_equilibrium(w, c.rs, cu, 0.5f * so);                  // E + S/2, odd part
    pa = ev + od;
    pb = ev - od;
}
__device__ __forceinline__ void mrt_pair(const CollideIn& c, const Mrt& m, int a, float& pa, float& pb) {
    mrt_pair_c(c, m, float(cx(a)), float(cy(a)), float(cz(a)), wsplit(a), pa, pb);
}

// the pairs with c_x != 0 (their odd member has c_x = +1): 1, 7, 9, 11, 13
__host__ __device__ constexpr int xpair(int m) { return m == 0 ? 1 : 5 + 2 * m; }
__host__ __device__ constexpr int xpair_index(int a) { return a == 1 ? 0 : (a - 5) / 2; }

// Moment contributions of one value v that arrives at a node as population a: delta rho
// gains v, j gains c_a v (acc = delta rho, j_x, j_y, j_z; c_a is a compile-time constant).
__device__ __forceinline__ void add_moments(float (&acc)[4], int a, float v) {
    acc[0] += v;
    if (cx(a) > 0) acc[1] += v;
    if (cx(a) < 0) acc[1] -= v;
    if (cy(a) > 0) acc[2] += v;
    if (cy(a) < 0) acc[2] -= v;
    if (cz(a) > 0) acc[3] += v;
    if (cz(a) < 0) acc[3] -= v;
}

// The five populations a row sends into the row above it (directions 3, 7, 10, 15, 17,
// c_y = +1), folded to what the moments of the receiving nodes need: the sum and the
// x-momentum of the three in-plane ones, then the one going to plane +1 and to plane -1.
__device__ __forceinline__ void fold_up(float v3, float v7, float v10, float v15, float v17, float (&o)[4]) {
    o[0] = (v3 + v7) + v10;
    o[1] = v7 - v10;
    o[2] = v15;
    o[3] = v17;
}
// ... and into the row below it (directions 4, 8, 9, 18, 16, c_y = -1).
__device__ __forceinline__ void fold_dn(float v4, float v8, float v9, float v16, float v18, float (&o)[4]) {
    o[0] = (v4 + v8) + v9;
    o[1] = v9 - v8;
    o[2] = v18;
    o[3] = v16;
}

// One workgroup's share of a step: tile [x0, x0+TX) x [y0, y0+TY), planes [z0, z1).
// TP = false: single pass, the moments are formed here from the populations of the tile
// and its halo.  TP = true: second pass of the two-pass step, delta rho and j of every
// node come from `mom` (written by the moments pass over the same time level), so only the
// tile's own populations are read, once, for the collision.
// MO (with TP, 64-wide tiles): the tile also forms delta rho and j of the next time level
// for its own nodes and writes them to `mom_out`, so the next step needs no moments pass.
// A node's new populations come from itself and its 18 neighbours, so the tile also
// collides, without storing anything,
//   * the planes z0-1 and z1 next to its chunk (only what crosses into the chunk is kept),
//   * the rows y0-1 and y0+TY next to it (the five directions entering the tile), and
//   * the corner nodes of those rows (the diagonal entering the tile's corner),
// with the same fixed-fma collision as own nodes.  Every moment is therefore the same sum
// of the same values, added in the same order, whatever the tile position and z-chunk.
// What a thread receives in its own row goes into a ring of three partial moments in
// registers (planes p-1, p, p+1 of the source plane p); what goes to the rows above and
// below is folded to four values per row and passed on through LDS.
// FE: 0 the upwind/Euler FENE-P update, 1 the Cholesky-log Adams-Bashforth-2 integrator with
// central differences and artificial diffusivity (the rate of the previous step read from
// `ab`, this step's written to `abn`, at the own node only).
template <int NC, int TX, int TY, bool TP, bool MO, int FE = 0, int CO = 0>
__device__ __forceinline__ void fused_tile(const DevParams& p, const float* __restrict__ h,
                                           float* __restrict__ hn, const float* __restrict__ D,
                                           float* __restrict__ Dn, unsigned* __restrict__ flags,
                                           FusedTile<NC, TX, TY, TP, MO>& L, int x0, int y0, int z0, int z1,
                                           const float* __restrict__ mom, float* __restrict__ mom_out,
                                           const float* __restrict__ ab = nullptr,
                                           float* __restrict__ abn = nullptr) {
    using T = FusedTile<NC, TX, TY, TP, MO>;
    static_assert(FE == 0 || MO, "the Cholesky integrator runs in the chained body only");
    static_assert(CO == 0 || MO, "the MRT collision runs in the chained body only");
    static_assert(!MO || (TP && (TX == 64 || TX == 32)),
                  "next-level moments: two-pass body, one or two tile rows per wavefront");
    static_assert(T::NH2 <= T::NT, "one R2 halo node per thread at most");
    static_assert(T::A1 <= 2 * T::NTH, "phase B covers the R1 region in two passes at most");
    static_assert(T::NT % 64 == 0, "a wavefront never straddles two components");

    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const uint32_t N = (uint32_t)p.N;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;

    const int tid = threadIdx.x;
    // component this thread loads and collides; uniform across the wavefront
    const int comp = __builtin_amdgcn_readfirstlane(tid / T::NT);
    const int nid = tid % T::NT;    // tile node of this thread
    const int olx = nid % TX, oly = nid / TX;
    const int ogx = x0 + olx, ogy = y0 + oly;
    const bool active = ogx < nx && ogy < ny;
    const int oi2 = (oly + 2) * T::W2 + olx + 2;
    const int oi1 = (oly + 1) * T::W1 + olx + 1;
    const int ogxw = wrapn(ogx, nx);
    const uint32_t own_xy = (uint32_t)min(ogy, ny - 1) * (uint32_t)nx + (uint32_t)ogxw;
    const float* hs = h + (size_t)comp * kQ * N;
    float* hns = hn + (size_t)comp * kQ * N;
    const bool fene = comp == 0;            // FENE-P and own C handled by component-0 threads
    const bool halo_d = comp == NC - 1;      // halo C loaded by the last component's threads

    // R2 halo node of this thread (fixed in x, y for the whole march)
    const bool has_halo = nid < T::NH2;
    int hlx = 0, hly = 0;
    if (has_halo) halo2_pos<TX, TY>(nid, hlx, hly);
    const int hgy = y0 + hly;
    const uint32_t halo_xy = (uint32_t)(hgy < 0 ? 0 : (hgy >= ny ? ny - 1 : hgy)) * (uint32_t)nx +
                             (uint32_t)wrapn(x0 + hlx, nx);

    // streaming targets of the own node that do not depend on the plane
    const uint32_t xcol[3] = {(uint32_t)(ogxw == 0 ? nx - 1 : ogxw - 1), (uint32_t)ogxw,
                              (uint32_t)(ogxw + 1 == nx ? 0 : ogxw + 1)};
    const uint32_t yrow = (uint32_t)min(ogy, ny - 1) * (uint32_t)nx;

    // own-column values of plane q-3 (their LDS ring slots are reused by plane q)
    float c_old[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float u_old[3] = {0.f, 0.f, 0.f};
    unsigned bad = 0u;

    // MO: partial next-level moments of the own node (delta rho, j) on planes p-1, p, p+1
    // (mm, m0, mp) for the plane p collided last; the momentum of a completed plane td waits in jd for
    // the other component's share
    float mm[4] = {0.f, 0.f, 0.f, 0.f}, m0[4] = {0.f, 0.f, 0.f, 0.f}, mp[4] = {0.f, 0.f, 0.f, 0.f};
    float jd[3] = {0.f, 0.f, 0.f};
    int td = -1;
    // MO: the wavefront that collides a neighbouring row (-1: the row below the tile, TY:
    // the row above, 0: none); one per component and side, on four different SIMDs
    int hrow = 0;
    if (MO) {
        const int wv = tid >> 6;
        if ((wv == 0 || wv == 10) && y0 >= 1) hrow = -1;
        if ((wv == 1 || wv == 11) && y0 + TY < ny) hrow = TY;
    }

    // plane q+1 is loaded while plane q is processed; the loads land in the registers that
    // phase A1 has just emptied, so no copy (and no early wait) sits on the loop edge
    NodeLoad pf_own, pf_halo;
    // two-pass: positions of the tile + halo this thread loads (moments and D), and the own
    // populations of the plane collided next
    constexpr int KP = (T::A2 + T::NTH - 1) / T::NTH;
    MomLoad<NC> mpf[KP];
    uint32_t mpos[KP];
    if (TP) {
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const int k = tid + i * T::NTH;
            const int lx = k % T::W2 - 2, ly = k / T::W2 - 2;
            const int gy = min(max(y0 + ly, 0), ny - 1);
            mpos[i] = (uint32_t)gy * (uint32_t)nx + (uint32_t)wrapn(x0 + lx, nx);
        }
    }
    auto issue_mom = [&](int zq) {
        const uint32_t zoff = (uint32_t)wrapn(zq, nz) * plane;
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            if (tid + i * T::NTH < T::A2) {
                const uint32_t bo = (zoff + mpos[i]) * 4u;
#pragma unroll
                for (int c = 0; c < NC; ++c) mpf[i].r[c] = ld_off(mom + (size_t)c * N, bo);
#pragma unroll
                for (int d = 0; d < 3; ++d) mpf[i].j[d] = ld_off(mom + (size_t)(NC + d) * N, bo);
#pragma unroll
                for (int k = 0; k < 6; ++k) mpf[i].d[k] = ld_off(D + (size_t)k * N, bo);
            }
        }
    };
    if (TP) {
        issue_mom(z0 - 2);
    } else {
        const uint32_t zoff = (uint32_t)wrapn(z0 - 2, nz) * plane;
        issue_load(hs, D, N, zoff + own_xy, fene, pf_own);
        if (has_halo) issue_load(hs, D, N, zoff + halo_xy, halo_d, pf_halo);
    }

    for (int q = z0 - 2; q <= z1 + 1; ++q) {
        // Two-pass bodies: the lane-dependent indices are derived again in every plane
        // from a copy of the thread index that the compiler cannot see through (an empty
        // asm statement).  Otherwise it keeps every LDS and global address it can form
        // from them live across the loop; at 128 VGPRs per thread (four waves per SIMD)
        // those addresses would be spilled to scratch, whose reloads cost HBM traffic.
        // The single-pass body runs two waves per SIMD and keeps them in registers.
        int tq = tid;
        if constexpr (TP) asm volatile("" : "+v"(tq));
        const int nid = tq % T::NT;
        const int olx = nid % TX, oly = nid / TX;
        const int ogx = x0 + olx, ogy = y0 + oly;
        const bool active = ogx < nx && ogy < ny;
        const int oi2 = (oly + 2) * T::W2 + olx + 2;
        const int oi1 = (oly + 1) * T::W1 + olx + 1;
        const uint32_t yrow = (uint32_t)min(ogy, ny - 1) * (uint32_t)nx;
        const uint32_t own_xy = yrow + xcol[1];
        const int sq = ((q % 3) + 3) % 3;
        const int s2 = q & 1;

        // ---------------- A1: consume plane q, then request plane q+1 ----------------
        if constexpr (TP) {
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const int k = tq + i * T::NTH;
                if (k < T::A2) {
                    const int lx = k % T::W2 - 2, ly = k / T::W2 - 2;
#pragma unroll
                    for (int c = 0; c < NC; ++c) L.rho[sq][c][k] = mpf[i].r[c];
#pragma unroll
                    for (int kk = 0; kk < 6; ++kk) L.cs[sq][kk][k] = mpf[i].d[kk];
                    if (lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) {
                        const int i1 = (ly + 1) * T::W1 + lx + 1;
#pragma unroll
                        for (int d = 0; d < 3; ++d) L.u[sq][d][i1] = mpf[i].j[d];
                    }
                }
            }
            if (q + 1 <= z1 + 1) issue_mom(q + 1);
        } else {
            phase_a1<NC, TX, TY, true>(L, sq, s2, comp, nid, olx, oly, fene, pf_own);
            if (has_halo) phase_a1<NC, TX, TY, false>(L, sq, s2, comp, nid, hlx, hly, halo_d, pf_halo);
            if (q + 1 <= z1 + 1) {
                const uint32_t zoff = (uint32_t)wrapn(q + 1, nz) * plane;
                issue_load(hs, D, N, zoff + own_xy, fene, pf_own);
                if (has_halo) issue_load(hs, D, N, zoff + halo_xy, halo_d, pf_halo);
            }
        }
        lds_barrier();

        // ---------------- A2: ghosts, f+, stress coefficients, total momentum ----------------
        for (int k = tq; k < T::A2; k += T::NTH) phase_a2<NC, TX, TY, TP>(p, L, sq, s2, y0, k, bad);
        if constexpr (MO) {
            // momentum of the plane completed last, second component's share (the exchange
            // reads of that plane ended at the barrier above)
            if (NC == 2 && comp == NC - 1 && td >= 0) {
                if (active) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) L.X[T::NFO + d * T::NT + nid] = jd[d];
                }
                td = -1;
            }
        }
        lds_barrier();

        // ---------------- B: forces and velocity on plane q-1 (tile + 1 halo) -------------
        if (q >= z0) {
            const int sr = ((q - 1) % 3 + 3) % 3;
            const int sp = ((q - 2) % 3 + 3) % 3;
            for (int k = tq; k < T::A1; k += T::NTH) {
                int lx, ly;
                if (k < T::NT) {
                    lx = k % TX;
                    ly = k / TX;
                } else {
                    halo1_pos<TX, TY>(k - T::NT, lx, ly);
                }
                const int gy = y0 + ly;
                if (gy < 0 || gy >= ny) continue;  // ghost velocities come from the wall rule
                float Fs[2][3];
                phase_b<NC, TX, TY, TP>(p, L, sp, sr, sq, lx, ly, Fs);
                const int i1 = (ly + 1) * T::W1 + lx + 1;
#pragma unroll
                for (int s = 0; s < NC; ++s)
#pragma unroll
                    for (int d = 0; d < 3; ++d) L.Fo[s][d][i1] = Fs[s][d];
            }
        }
        if constexpr (MO) {
            // momentum of the plane completed last: both components' shares, written out
            // (the forces written above lie below offset NFO)
            if (comp == 0 && td >= 0) {
                if (active) {
                    const uint32_t bt = ((uint32_t)td * plane + own_xy) * 4u;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        float jv = jd[d];
                        if (NC == 2) jv += L.X[T::NFO + d * T::NT + nid];
                        st_off(mom_out + (size_t)(NC + d) * N, bt, jv);
                    }
                }
                td = -1;
            }
        }
        lds_barrier();

        // ---------------- D: FENE-P on plane q-2 (own node, component-0 threads) ----------
        // (independent of C: it reads C - I and u from LDS and writes only Dn)
        auto phase_d = [&]() {
            if (fene && q >= z0 + 2 && active) {
                const int t = wrapn(q - 2, nz);
                const int st = ((q - 2) % 3 + 3) % 3;
                const int st1 = ((q - 1) % 3 + 3) % 3;
                const uint32_t bt = ((uint32_t)t * plane + own_xy) * 4u;
                // the previous step's rate (Cholesky integrator), requested first so that
                // its latency hides behind the stencil
                float yp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if constexpr (FE == 1) {
                    if (p.ab_hist) {
#pragma unroll
                        for (int k = 0; k < 6; ++k) yp[k] = ld_off(ab + (size_t)k * N, bt);
                    }
                }
                float d0[6], u0[3];
#pragma unroll
                for (int k = 0; k < 6; ++k) d0[k] = L.cs[st][k][oi2];
#pragma unroll
                for (int d = 0; d < 3; ++d) u0[d] = L.u[st][d][oi1];
                float Gm[3][3];
                float adv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    float up[3], um[3];
                    if (i == 2) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            up[d] = L.u[st1][d][oi1];
                            um[d] = u_old[d];
                        }
                    } else {
                        const int off = i == 0 ? 1 : T::W1;
                        const bool top = i == 1 && ogy == ny - 1;
                        const bool bot = i == 1 && ogy == 0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const float vp = L.u[st][d][oi1 + off];
                            const float vm = L.u[st][d][oi1 - off];
                            up[d] = top ? 2.0f * p.ut[d] - u0[d] : vp;
                            um[d] = bot ? 2.0f * p.ub[d] - u0[d] : vm;
                        }
                    }
#pragma unroll
                    for (int d = 0; d < 3; ++d) Gm[i][d] = 0.5f * (up[d] - um[d]);
                    if constexpr (FE == 1) {
                        // central difference and artificial diffusivity along i (the wall
                        // ghosts in the rings are the linear extrapolations)
                        float dpl[6], dmi[6];
                        if (i == 2) {
#pragma unroll
                            for (int k = 0; k < 6; ++k) {
                                dpl[k] = L.cs[st1][k][oi2];
                                dmi[k] = c_old[k];
                            }
                        } else {
                            const int off = i == 0 ? 1 : T::W2;
#pragma unroll
                            for (int k = 0; k < 6; ++k) {
                                dpl[k] = L.cs[st][k][oi2 + off];
                                dmi[k] = L.cs[st][k][oi2 - off];
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            adv[k] += u0[i] * (0.5f * (dpl[k] - dmi[k])) - p.kappa * (dpl[k] - 2.0f * d0[k] + dmi[k]);
                        continue;
                    }
                    float dn[6];
                    const bool bwd = u0[i] >= 0.0f;  // upwind: backward difference for u_i >= 0
                    if (i == 2) {
#pragma unroll
                        for (int k = 0; k < 6; ++k) dn[k] = bwd ? c_old[k] : L.cs[st1][k][oi2];
                    } else {
                        const int off = i == 0 ? 1 : T::W2;
                        const int in = bwd ? oi2 - off : oi2 + off;
#pragma unroll
                        for (int k = 0; k < 6; ++k) dn[k] = L.cs[st][k][in];
                    }
#pragma unroll
                    for (int k = 0; k < 6; ++k) adv[k] += bwd ? u0[i] * (d0[k] - dn[k]) : u0[i] * (dn[k] - d0[k]);
                }
                const float trd = d0[0] + d0[1] + d0[2];
                const float den = p.L2m3 - trd;
                if (!(den > 0.0f)) bad |= 2u;
                const float inv = 1.0f / den;
                const float f = p.L2m3 * inv;
                const float fm1 = trd * inv;
                float dnew[6], rate[6];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
#pragma unroll
                    for (int b = a; b < 3; ++b) {
                        const int kk = sidx(a, b);
                        float stv = Gm[b][a] + Gm[a][b];
#pragma unroll
                        for (int k = 0; k < 3; ++k) stv += Gm[k][a] * d0[sidx(k, b)] + d0[sidx(a, k)] * Gm[k][b];
                        const float relax = (f * d0[kk] + (a == b ? fm1 : 0.0f)) * p.inv_tau_p;
                        rate[kk] = -adv[kk] + stv - relax;
                        dnew[kk] = d0[kk] + rate[kk];
                    }
                }
                if constexpr (FE == 1) {
                    // the same rate taken through the Cholesky factor of f C, one AB2 step
                    if (den > 0.0f) {
                        float dn6[6], yd[6];
                        if (cholesky_ab2_step(p.L2, p.L2m3, d0, rate, yp, p.ab_hist != 0, dn6, yd)) {
#pragma unroll
                            for (int k = 0; k < 6; ++k) {
                                dnew[k] = dn6[k];
                                st_off(abn + (size_t)k * N, bt, yd[k]);
                            }
                        } else {
                            bad |= 4u;
                        }
                    }
                }
                float check = 0.0f;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    st_off(Dn + (size_t)k * N, bt, dnew[k]);
                    check += dnew[k];
                }
                if (!isfinite(check)) bad |= 1u;
                const float c0 = 1.0f + dnew[0], c1 = 1.0f + dnew[1], c2 = 1.0f + dnew[2];
                if (!(c0 + c1 + c2 < p.L2)) bad |= 2u;
                const float m2 = c0 * c1 - dnew[3] * dnew[3];
                const float m3 = c0 * (c1 * c2 - dnew[5] * dnew[5]) - dnew[3] * (dnew[3] * c2 - dnew[5] * dnew[4]) +
                                 dnew[4] * (dnew[3] * dnew[5] - c1 * dnew[4]);
                if (!(c0 > 0.0f && m2 > 0.0f && m3 > 0.0f)) bad |= 4u;
            }
        };

        // ---------------- C: collide + stream plane q-1 (own node, own component) ----------
        // BGK with the forcing source (eq. LB, Lambda = I/tau(phi)), per opposite pair.
        // Streaming stores are x-aligned: a lane stores, at its own x, the value arriving
        // from x - c_x, taken from the neighbouring lane of its row; the edge lane of a row
        // collides the halo node's inbound directions itself (same arithmetic, same inputs),
        // so every row of every direction is written as whole lines by one workgroup.
        // MO also collides the planes z0-1 and z1 (no stores) and a neighbouring row.
        const bool cplane = MO ? (q >= z0 && q <= z1 + 1) : (q >= z0 + 1 && q <= z1);
        const bool store = q >= z0 + 1 && q <= z1;
        const bool own_ok = ogy < ny;
        float up[4] = {0.f, 0.f, 0.f, 0.f}, dn[4] = {0.f, 0.f, 0.f, 0.f}, hj[4] = {0.f, 0.f, 0.f, 0.f};
        if (MO) phase_d();
        if (cplane && (own_ok || (MO && hrow != 0))) {
            const int sr = ((q - 1) % 3 + 3) % 3;
            const int p2 = s2 ^ 1;
            const int r = wrapn(q - 1, nz);
            const int txe = min(TX, nx - x0);  // columns of this tile inside the lattice
            const bool left_edge = olx == 0;
            const bool right_edge = olx == txe - 1;
            const uint32_t zrow[3] = {(uint32_t)(r == 0 ? nz - 1 : r - 1) * plane, (uint32_t)r * plane,
                                      (uint32_t)(r + 1 == nz ? 0 : r + 1) * plane};
            const uint32_t bself = (zrow[1] + yrow + xcol[1]) * 4u;
            // the halo nodes' post-collision values that stream into this row's edge nodes:
            // lane m < 5 of the row collides direction xpair(m) (c_x = +1) of the left halo
            // node, lane 5 + m direction xpair(m) + 1 (c_x = -1) of the right one.  MO: lanes
            // 10 and 11 collide the diagonal that enters the tile's corner from the corner
            // node of the neighbouring row (left: c_x = +1, right: c_x = -1)
            float hval = 0.0f;
            const bool e_own = own_ok && olx < 10;
            const bool e_corner = MO && hrow != 0 && (olx == 10 || olx == 11);
            if (e_own || e_corner) {
                int ap, nlx, nly;
                bool take_a;
                if (e_own) {
                    const bool lside = olx < 5;
                    const int m = lside ? olx : olx - 5;
                    ap = m == 0 ? 1 : 5 + 2 * m;  // xpair(m)
                    take_a = lside;
                    nlx = lside ? -1 : txe;
                    nly = oly;
                } else {
                    const bool left = olx == 10;
                    ap = ((hrow < 0) == left) ? 7 : 9;
                    take_a = left;
                    nlx = left ? -1 : txe;
                    nly = hrow;
                }
                const float ex = 1.0f;
                const float ey = ap == 7 ? 1.0f : (ap == 9 ? -1.0f : 0.0f);
                const float ez = ap == 11 ? 1.0f : (ap == 13 ? -1.0f : 0.0f);
                const Wt w = ap == 1 ? wsplit(1) : wsplit(7);
                const uint32_t hx = (uint32_t)wrapn(x0 + nlx, nx);  // halo column
                const uint32_t bo = (zrow[1] + (uint32_t)(y0 + nly) * (uint32_t)nx + hx) * 4u;
                const CollideIn in = collide_in<NC, TX, TY, TP>(p, L, sr, p2, comp, (nly + 1) * T::W1 + nlx + 1,
                                                                (nly + 2) * T::W2 + nlx + 2);
                if constexpr (CO == 1) {
                    float hh[kQ];
#pragma unroll
                    for (int a = 0; a < kQ; ++a) hh[a] = ld_off(hs + (size_t)a * N, bo);
                    const Mrt mc = mrt_coef(in, hh);
                    float pa, pb;
                    mrt_pair_c(in, mc, ex, ey, ez, w, pa, pb);
                    hval = take_a ? pa : pb;
                } else {
                    const float hv = ld_off(hs + (size_t)(take_a ? ap : ap + 1) * N, bo);
                    float pa, pb;
                    collide_pair_c(in, ex, ey, ez, w, hv, hv, pa, pb);
                    hval = take_a ? pa : pb;
                }
            }
            float lin[5], rin[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                lin[m] = __shfl(hval, m, TX);
                rin[m] = __shfl(hval, 5 + m, TX);
            }
            float cl = 0.0f, cr = 0.0f;
            if constexpr (MO) {
                cl = __shfl(hval, 10, TX);
                cr = __shfl(hval, 11, TX);
            }
            if (own_ok) {
                float hpop[kQ];
                if constexpr (TP) {
#pragma unroll
                    for (int a = 0; a < kQ; ++a) hpop[a] = ld_off(hs + (size_t)a * N, bself);
                } else {
#pragma unroll
                    for (int a = 0; a < kQ; ++a) hpop[a] = L.pop[TP ? 0 : p2][TP ? 0 : comp][a][TP ? 0 : nid];
                }
                const CollideIn own = collide_in<NC, TX, TY, TP>(p, L, sr, p2, comp, oi1, oi2);
                const bool stx = ogx < nx;  // lanes past a ragged edge compute but do not store
                float xv[kQ];               // MO: values leaving the row (c_y != 0), as stored
                float check;
                Mrt mo{};
                if constexpr (CO == 1) mo = mrt_coef(own, hpop);
                {
                    float post;
                    if constexpr (CO == 1) {
                        float junk;
                        mrt_pair(own, mo, 0, post, junk);
                    } else {
                        post = collide_rest(own, hpop[0]);
                    }
                    if (store && stx) st_off(hns, bself, post);
                    check = post;
                    if constexpr (MO) add_moments(m0, 0, post);
                }
#pragma unroll
                for (int a = 1; a < kQ; a += 2) {
                    float pp, pm;
                    if constexpr (CO == 1) {
                        mrt_pair(own, mo, a, pp, pm);
                    } else {
                        collide_pair(own, a, hpop[a], hpop[a + 1], pp, pm);
                    }
                    check += pp + pm;
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int bq = a + e;
                        const float post = e == 0 ? pp : pm;
                        float v = post;
                        if (cx(bq) > 0) {
                            v = __shfl_up(post, 1, TX);
                            if (left_edge) v = lin[xpair_index(a)];
                        } else if (cx(bq) < 0) {
                            v = __shfl_down(post, 1, TX);
                            if (right_edge) v = rin[xpair_index(a)];
                        }
                        const int yd = ogy + cy(bq);
                        if (yd >= 0 && yd < ny) {
                            const uint32_t dst = zrow[cz(bq) + 1] + yrow + (uint32_t)(cy(bq) * nx) + xcol[1];
                            if (store && stx) st_off(hns + (size_t)bq * N, dst * 4u, v);
                            if constexpr (MO) {
                                if (cy(bq) != 0) xv[bq] = v;
                                else if (cz(bq) > 0) add_moments(mp, bq, v);
                                else if (cz(bq) < 0) add_moments(mm, bq, v);
                                else add_moments(m0, bq, v);
                            }
                        } else {
                            // moving-wall bounce-back (Sec. 3.1 walls): the link returns as opp(bq)
                            const float* uw = yd < 0 ? p.ub : p.ut;
                            const float bb = post - 6.0f * wgt(bq) * own.rs * wall_cu(bq, uw);
                            if (store && stx) st_off(hns + (size_t)opp(bq) * N, bself, bb);
                            if constexpr (MO) {
                                add_moments(m0, opp(bq), bb);
                                xv[bq] = 0.0f;
                            }
                        }
                    }
                }
                if (store && stx && !isfinite(check)) bad |= 1u;
                if constexpr (MO) {
                    fold_up(xv[3], xv[7], xv[10], xv[15], xv[17], up);
                    fold_dn(xv[4], xv[8], xv[9], xv[16], xv[18], dn);
                }
            }
            if constexpr (MO) {
                // the neighbouring row's directions that enter the tile, x-aligned like the
                // own stores (lane 0 / the last lane take the corner values of lanes 10 / 11)
                if (hrow != 0) {
                    const int hy = hrow;
                    const uint32_t bh = (zrow[1] + (uint32_t)(y0 + hy) * (uint32_t)nx + xcol[1]) * 4u;
                    const CollideIn hin = collide_in<NC, TX, TY, TP>(p, L, sr, p2, comp, (hy + 1) * T::W1 + olx + 1,
                                                                     (hy + 2) * T::W2 + olx + 2);
                    float junk;
                    if constexpr (CO == 1) {
                        float hh[kQ];
#pragma unroll
                        for (int a = 0; a < kQ; ++a) hh[a] = ld_off(hs + (size_t)a * N, bh);
                        const Mrt mh = mrt_coef(hin, hh);
                        float p3, p4, p7, p8, p9, p10, p15, p16, p17, p18;
                        mrt_pair(hin, mh, 3, p3, p4);
                        mrt_pair(hin, mh, 7, p7, p8);
                        mrt_pair(hin, mh, 9, p9, p10);
                        mrt_pair(hin, mh, 15, p15, p16);
                        mrt_pair(hin, mh, 17, p17, p18);
                        if (hy < 0) {
                            float s7 = __shfl_up(p7, 1, TX);
                            if (left_edge) s7 = cl;
                            float s10 = __shfl_down(p10, 1, TX);
                            if (right_edge) s10 = cr;
                            fold_up(p3, s7, s10, p15, p17, hj);
                        } else {
                            float s9 = __shfl_up(p9, 1, TX);
                            if (left_edge) s9 = cl;
                            float s8 = __shfl_down(p8, 1, TX);
                            if (right_edge) s8 = cr;
                            fold_dn(p4, s8, s9, p16, p18, hj);
                        }
                    } else if (hy < 0) {
                        const float h3 = ld_off(hs + (size_t)3 * N, bh), h7 = ld_off(hs + (size_t)7 * N, bh);
                        const float h10 = ld_off(hs + (size_t)10 * N, bh), h15 = ld_off(hs + (size_t)15 * N, bh);
                        const float h17 = ld_off(hs + (size_t)17 * N, bh);
                        float v3, v7, v10, v15, v17;
                        collide_pair(hin, 3, h3, h3, v3, junk);
                        collide_pair(hin, 7, h7, h7, v7, junk);
                        collide_pair(hin, 9, h10, h10, junk, v10);
                        collide_pair(hin, 15, h15, h15, v15, junk);
                        collide_pair(hin, 17, h17, h17, v17, junk);
                        float s7 = __shfl_up(v7, 1, TX);
                        if (left_edge) s7 = cl;
                        float s10 = __shfl_down(v10, 1, TX);
                        if (right_edge) s10 = cr;
                        fold_up(v3, s7, s10, v15, v17, hj);
                    } else {
                        const float h4 = ld_off(hs + (size_t)4 * N, bh), h8 = ld_off(hs + (size_t)8 * N, bh);
                        const float h9 = ld_off(hs + (size_t)9 * N, bh), h16 = ld_off(hs + (size_t)16 * N, bh);
                        const float h18 = ld_off(hs + (size_t)18 * N, bh);
                        float v4, v8, v9, v16, v18;
                        collide_pair(hin, 3, h4, h4, junk, v4);
                        collide_pair(hin, 7, h8, h8, junk, v8);
                        collide_pair(hin, 9, h9, h9, v9, junk);
                        collide_pair(hin, 15, h16, h16, junk, v16);
                        collide_pair(hin, 17, h18, h18, junk, v18);
                        float s9 = __shfl_up(v9, 1, TX);
                        if (left_edge) s9 = cl;
                        float s8 = __shfl_down(v8, 1, TX);
                        if (right_edge) s8 = cr;
                        fold_dn(v4, s8, s9, v16, v18, hj);
                    }
                }
            }
        }
        if (!MO) phase_d();

        // plane q-2 becomes plane q-3 of the next iteration (C and D write no LDS; the
        // barrier after these reads protects the slots the next phase A overwrites)
        if (fene) {
            const int st = ((q - 2) % 3 + 3) % 3;
#pragma unroll
            for (int k = 0; k < 6; ++k) c_old[k] = L.cs[st][k][oi2];
#pragma unroll
            for (int d = 0; d < 3; ++d) u_old[d] = L.u[st][d][oi1];
        }
        lds_barrier();

        if constexpr (MO) {
            // ---------------- exchange: partial moments for the rows above and below ------
            if (cplane) {
                const int cb = comp * 8;
                if (own_ok) {
                    if (oly + 1 < TY) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) L.X[((cb + k) * TY + oly + 1) * TX + olx] = up[k];
                    }
                    if (oly >= 1) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) L.X[((cb + 4 + k) * TY + oly - 1) * TX + olx] = dn[k];
                    }
                }
                if (hrow < 0) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) L.X[(cb + k) * TY * TX + olx] = hj[k];
                } else if (hrow == TY) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) L.X[((cb + 4 + k) * TY + TY - 1) * TX + olx] = hj[k];
                }
            }
            lds_barrier();
            if (cplane) {
                const int cb = comp * 8;
                if (own_ok && ogy >= 1) {  // from the row below (c_y = +1)
                    float o[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) o[k] = L.X[((cb + k) * TY + oly) * TX + olx];
                    m0[0] += o[0];
                    m0[1] += o[1];
                    m0[2] += o[0];
                    mp[0] += o[2];
                    mp[2] += o[2];
                    mp[3] += o[2];
                    mm[0] += o[3];
                    mm[2] += o[3];
                    mm[3] -= o[3];
                }
                if (own_ok && ogy + 1 < ny) {  // from the row above (c_y = -1)
                    float o[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) o[k] = L.X[((cb + 4 + k) * TY + oly) * TX + olx];
                    m0[0] += o[0];
                    m0[1] += o[1];
                    m0[2] -= o[0];
                    mp[0] += o[2];
                    mp[2] -= o[2];
                    mp[3] += o[2];
                    mm[0] += o[3];
                    mm[2] -= o[3];
                    mm[3] -= o[3];
                }
                // plane q-2 has received all its populations
                const int t = q - 2;
                if (t >= z0 && t < z1) {
                    const int tw = wrapn(t, nz);
                    if (active) st_off(mom_out + (size_t)comp * N, ((uint32_t)tw * plane + own_xy) * 4u, mm[0]);
#pragma unroll
                    for (int d = 0; d < 3; ++d) jd[d] = mm[d + 1];
                    td = tw;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    mm[k] = m0[k];
                    m0[k] = mp[k];
                    mp[k] = 0.0f;
                }
            }
        }
    }
    if constexpr (MO) {
        // the last completed plane's momentum (td is the same in every thread)
        if (td >= 0) {
            lds_barrier();
            if (NC == 2 && comp == NC - 1 && active) {
#pragma unroll
                for (int d = 0; d < 3; ++d) L.X[T::NFO + d * T::NT + nid] = jd[d];
            }
            lds_barrier();
            if (comp == 0 && active) {
                const uint32_t bt = ((uint32_t)td * plane + own_xy) * 4u;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    float jv = jd[d];
                    if (NC == 2) jv += L.X[T::NFO + d * T::NT + nid];
                    st_off(mom_out + (size_t)(NC + d) * N, bt, jv);
                }
            }
        }
    }
    if (bad) atomicOr(flags, bad);
}

template <int NC, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY, 1) void k_fused(
    DevParams p, const float* __restrict__ h, float* __restrict__ hn, const float* __restrict__ D,
    float* __restrict__ Dn, unsigned* __restrict__ flags, int zchunk) {
    __shared__ FusedTile<NC, TX, TY, false> L;
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    // groups of about 256 x 32 nodes
    const int gxw = min(ntx, 256 / TX);
    const int gyh = min(nty, max(1, 32 / gxw));
    int tx_i, ty_i, zc_i;
    tile_of_block(blockIdx.x, gridDim.x, ntx, nty, gxw, gyh, tx_i, ty_i, zc_i);
    const int z0 = zc_i * zchunk;
    fused_tile<NC, TX, TY, false, false>(p, h, hn, D, Dn, flags, L, tx_i * TX, ty_i * TY, z0,
                                         min(z0 + zchunk, p.nz), nullptr, nullptr);
}

// Second pass of the two-pass step: the moments of the whole lattice at time level n are
// in `mom` (delta rho per component, then j), written by the moments pass.  Without the
// population ring its LDS (72 KB for 32x8, two components) admits two workgroups per CU;
// the launch bound asks for 4 waves per SIMD (128 VGPRs) so that both fit.
template <int NC, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY, NC == 2 ? 4 : 2) void k_fused2(
    DevParams p, const float* __restrict__ h, float* __restrict__ hn, const float* __restrict__ D,
    float* __restrict__ Dn, const float* __restrict__ mom, unsigned* __restrict__ flags, int zchunk) {
    __shared__ FusedTile<NC, TX, TY, true> L;
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const int gxw = min(ntx, 256 / TX);
    const int gyh = min(nty, max(1, 32 / gxw));
    int tx_i, ty_i, zc_i;
    tile_of_block(blockIdx.x, gridDim.x, ntx, nty, gxw, gyh, tx_i, ty_i, zc_i);
    const int z0 = zc_i * zchunk;
    fused_tile<NC, TX, TY, true, false>(p, h, hn, D, Dn, flags, L, tx_i * TX, ty_i * TY, z0,
                                        min(z0 + zchunk, p.nz), mom, nullptr);
}

// Chained two-pass step: the second pass of step n, which also writes the moments of
// level n+1 to `mom_out`, so that step n+1 starts from them without a moments pass.
// 64x8 tiles only (one tile row per wavefront); 156 KB of LDS for two components.
// FE selects the FENE-P integrator (0 upwind/Euler, 1 Cholesky-log AB2, its rate history
// read from ab and written to abn); CO the collision (0 BGK, 1 MRT).
template <int NC, int FE, int CO>
__global__ __launch_bounds__(NC * 64 * 8, NC == 2 ? 4 : 2) void k_fused3(
    DevParams p, const float* __restrict__ h, float* __restrict__ hn, const float* __restrict__ D,
    float* __restrict__ Dn, const float* __restrict__ mom, float* __restrict__ mom_out, unsigned* __restrict__ flags,
    int zchunk, const float* __restrict__ ab, float* __restrict__ abn) {
    constexpr int TX = 64, TY = 8;
    __shared__ FusedTile<NC, TX, TY, true, true> L;
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const int gxw = min(ntx, 256 / TX);
    const int gyh = min(nty, max(1, 32 / gxw));
    int tx_i, ty_i, zc_i;
    tile_of_block(blockIdx.x, gridDim.x, ntx, nty, gxw, gyh, tx_i, ty_i, zc_i);
    const int z0 = zc_i * zchunk;
    fused_tile<NC, TX, TY, true, true, FE, CO>(p, h, hn, D, Dn, flags, L, tx_i * TX, ty_i * TY, z0,
                                               min(z0 + zchunk, p.nz), mom, mom_out, ab, abn);
}

// Many independent lattices in one launch: each workgroup takes one entry of the work
// table (instance, tile, z range) and steps that part of its instance.  The instance's
// buffer holding time level n is cur ^ parity, so a two-launch graph (parity 0, 1)
// replays any even number of steps.
template <int NC, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY, 1) void k_fused_batch(
    const BatchInstance* __restrict__ inst, const WorkItem* __restrict__ work, int parity) {
    __shared__ FusedTile<NC, TX, TY, false> L;
    const int64_t bid = xcd_remap_f(blockIdx.x, gridDim.x);
    const WorkItem w = work[bid];
    const BatchInstance& bi = inst[w.inst];
    const DevParams p = bi.p;
    const int c = bi.cur ^ parity;
    fused_tile<NC, TX, TY, false, false>(p, bi.h[c], bi.h[c ^ 1], bi.D[c], bi.D[c ^ 1], bi.flags, L, w.x0, w.y0,
                                         w.z0, w.z1, nullptr, nullptr);
}

// Chained step for many lattices: the k_fused_batch work table, and each instance's moments
// carried in mom[cur ^ parity] -> mom[cur ^ parity ^ 1] (and, with the Cholesky integrator,
// its rate history in ab the same way).  FE and CO as for k_fused3, shared by every instance
// of the batch.  TX = 64: 64x8 tiles, one tile row per wavefront; TX = 32: 32x16 tiles for
// lattices 32 or 96 nodes wide, where a 64-wide tile would run half or a quarter empty (two
// tile rows per wavefront, the shuffles 32 lanes wide; the wavefronts that collide a
// neighbouring row run it in both halves, which form the same values).  The collisions and
// the order in which each node's moments are summed do not depend on the tile, so both
// shapes give the same results bit for bit.
template <int NC, int FE, int CO, int TX>
__global__ __launch_bounds__(NC * 64 * 8, NC == 2 ? 4 : 2) void k_fused3_batch(
    const BatchInstance* __restrict__ inst, const WorkItem* __restrict__ work, int parity) {
    constexpr int TY = 512 / TX;
    __shared__ FusedTile<NC, TX, TY, true, true> L;
    const int64_t bid = xcd_remap_f(blockIdx.x, gridDim.x);
    const WorkItem w = work[bid];
    const BatchInstance& bi = inst[w.inst];
    const DevParams p = bi.p;
    const int c = bi.cur ^ parity;
    fused_tile<NC, TX, TY, true, true, FE, CO>(p, bi.h[c], bi.h[c ^ 1], bi.D[c], bi.D[c ^ 1], bi.flags, L, w.x0, w.y0,
                                               w.z0, w.z1, bi.mom[c], bi.mom[c ^ 1], bi.ab[c], bi.ab[c ^ 1]);
}

template <int NC, int TX, int TY>
static hipError_t launch_fused_t(const DevParams& p, const Buffers& b, int zchunk, hipStream_t s) {
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const int nzc = (p.nz + zchunk - 1) / zchunk;
    const int64_t nblk = (int64_t)ntx * nty * nzc;
    hipLaunchKernelGGL((k_fused<NC, TX, TY>), dim3((unsigned)nblk), dim3(NC * TX * TY), 0, s, p, b.h, b.hn, b.D,
                       b.Dn, b.flags, zchunk);
    return hipGetLastError();
}

template <int NC, int TX, int TY>
static hipError_t launch_fused2_t(const DevParams& p, const Buffers& b, int zchunk, hipStream_t s) {
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const int nzc = (p.nz + zchunk - 1) / zchunk;
    const int64_t nblk = (int64_t)ntx * nty * nzc;
    hipLaunchKernelGGL((k_fused2<NC, TX, TY>), dim3((unsigned)nblk), dim3(NC * TX * TY), 0, s, p, b.h, b.hn, b.D,
                       b.Dn, b.mom, b.flags, zchunk);
    return hipGetLastError();
}

hipError_t launch_fused2(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s) {
    const int zc = t.zchunk > 0 ? t.zchunk : p.nz;
    if (p.nc == 2) {
        if (t.tile == 2) return launch_fused2_t<2, 16, 16>(p, b, zc, s);
        if (t.tile == 3) return launch_fused2_t<2, 64, 8>(p, b, zc, s);
        return launch_fused2_t<2, 32, 8>(p, b, zc, s);
    }
    if (t.tile == 2) return launch_fused2_t<1, 16, 16>(p, b, zc, s);
    if (t.tile == 3) return launch_fused2_t<1, 64, 8>(p, b, zc, s);
    return launch_fused2_t<1, 32, 8>(p, b, zc, s);
}

template <int NC, int FE, int CO>
static hipError_t launch_fused3_t(const DevParams& p, const Buffers& b, int zchunk, hipStream_t s) {
    const int ntx = (p.nx + 63) / 64, nty = (p.ny + 7) / 8;
    const int nzc = (p.nz + zchunk - 1) / zchunk;
    const int64_t nblk = (int64_t)ntx * nty * nzc;
    hipLaunchKernelGGL((k_fused3<NC, FE, CO>), dim3((unsigned)nblk), dim3(NC * 64 * 8), 0, s, p, b.h, b.hn, b.D, b.Dn,
                       b.mom, b.mom_next, b.flags, zchunk, b.ab, b.ab_next);
    return hipGetLastError();
}

hipError_t launch_fused3(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s) {
    const int zc = t.zchunk > 0 ? t.zchunk : p.nz;
    if (p.collision == 1) {
        if (p.fene == 1) return p.nc == 2 ? launch_fused3_t<2, 1, 1>(p, b, zc, s) : launch_fused3_t<1, 1, 1>(p, b, zc, s);
        return p.nc == 2 ? launch_fused3_t<2, 0, 1>(p, b, zc, s) : launch_fused3_t<1, 0, 1>(p, b, zc, s);
    }
    if (p.fene == 1) return p.nc == 2 ? launch_fused3_t<2, 1, 0>(p, b, zc, s) : launch_fused3_t<1, 1, 0>(p, b, zc, s);
    return p.nc == 2 ? launch_fused3_t<2, 0, 0>(p, b, zc, s) : launch_fused3_t<1, 0, 0>(p, b, zc, s);
}

hipError_t launch_fused_batch(const BatchInstance* inst, const WorkItem* work, int64_t nwork, int ncomp, int tile,
                              int parity, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    const dim3 grid((unsigned)nwork);
    if (ncomp == 2) {
        if (tile == 2)
            hipLaunchKernelGGL((k_fused_batch<2, 16, 16>), grid, dim3(512), 0, s, inst, work, parity);
        else
            hipLaunchKernelGGL((k_fused_batch<2, 32, 8>), grid, dim3(512), 0, s, inst, work, parity);
    } else {
        if (tile == 2)
            hipLaunchKernelGGL((k_fused_batch<1, 16, 16>), grid, dim3(256), 0, s, inst, work, parity);
        else
            hipLaunchKernelGGL((k_fused_batch<1, 32, 8>), grid, dim3(256), 0, s, inst, work, parity);
    }
    return hipGetLastError();
}

template <int NC, int FE, int CO>
static void launch_fused3_batch_t(const BatchInstance* inst, const WorkItem* work, int64_t nwork, int tx, int parity,
                                  hipStream_t s) {
    if (tx == 32)
        hipLaunchKernelGGL((k_fused3_batch<NC, FE, CO, 32>), dim3((unsigned)nwork), dim3(NC * 512), 0, s, inst, work,
                           parity);
    else
        hipLaunchKernelGGL((k_fused3_batch<NC, FE, CO, 64>), dim3((unsigned)nwork), dim3(NC * 512), 0, s, inst, work,
                           parity);
}

hipError_t launch_fused3_batch(const BatchInstance* inst, const WorkItem* work, int64_t nwork, int ncomp, int fene,
                               int collision, int tx, int parity, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    if (tx != 32 && tx != 64) return hipErrorInvalidValue;
    const int sel = (ncomp == 2 ? 4 : 0) + (fene == 1 ? 2 : 0) + (collision == 1 ? 1 : 0);
    switch (sel) {
        case 0: launch_fused3_batch_t<1, 0, 0>(inst, work, nwork, tx, parity, s); break;
        case 1: launch_fused3_batch_t<1, 0, 1>(inst, work, nwork, tx, parity, s); break;
        case 2: launch_fused3_batch_t<1, 1, 0>(inst, work, nwork, tx, parity, s); break;
        case 3: launch_fused3_batch_t<1, 1, 1>(inst, work, nwork, tx, parity, s); break;
        case 4: launch_fused3_batch_t<2, 0, 0>(inst, work, nwork, tx, parity, s); break;
        case 5: launch_fused3_batch_t<2, 0, 1>(inst, work, nwork, tx, parity, s); break;
        case 6: launch_fused3_batch_t<2, 1, 0>(inst, work, nwork, tx, parity, s); break;
        default: launch_fused3_batch_t<2, 1, 1>(inst, work, nwork, tx, parity, s); break;
    }
    return hipGetLastError();
}

// tile extent of the chained batch body for a tuning choice: 32x16 when asked for, else 64x8
void chained_batch_tile_shape(int tile, int* tx, int* ty) {
    *tx = tile == 1 ? 32 : 64;
    *ty = tile == 1 ? 16 : 8;
}

// tile extent of a tuning choice (the 32x16 choice runs as 32x8: a 32x16 tile with its
// two planes of own populations would not fit in LDS)
void fused_tile_shape(int ncomp, int tile, int* tx, int* ty) {
    (void)ncomp;
    *tx = tile == 2 ? 16 : 32;
    *ty = tile == 2 ? 16 : 8;
}

hipError_t launch_fused(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s) {
    const int zc = t.zchunk > 0 ? t.zchunk : p.nz;
    if (p.nc == 2) {
        if (t.tile == 2) return launch_fused_t<2, 16, 16>(p, b, zc, s);
        return launch_fused_t<2, 32, 8>(p, b, zc, s);
    }
    if (t.tile == 2) return launch_fused_t<1, 16, 16>(p, b, zc, s);
    return launch_fused_t<1, 32, 8>(p, b, zc, s);
}

}  // namespace lbfd

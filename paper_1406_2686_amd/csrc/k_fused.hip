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
//   C  collides plane q-1 (BGK with the forcing source, eq. LB with Lambda = I/tau(phi))
//      and pushes the post-collision populations to their neighbours, bouncing links that
//      leave through a wall back with the moving-wall correction;
//   D  advances C on plane q-2 with the explicit FENE-P update (eq. FENE): first-order
//      upwind advection, G^T C + C G with central G_ij = d_i u_j, Peterlin relaxation.
// Every stage reads time level n only, so HBM sees each population and C component read
// once and written once per step: 2 x ncomp x 19 x 4 + 2 x 6 x 4 bytes per node.  The halo
// re-reads of neighbouring tiles hit L2: blocks are remapped so that each XCD owns a
// contiguous range of tiles, x-tile fastest.
//
// Ghost rules at the y walls (same as the host-visible definition of the method):
// densities copy the wall layer, C is extrapolated linearly, u is reflected through the
// wall velocity; x and z are periodic.
#include "d3q19.h"
#include "lbfd_internal.h"

namespace lbfd {

namespace {

__device__ __forceinline__ int64_t xcd_remap_f(int64_t b, int64_t nb) {
    const int64_t per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
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

__device__ __forceinline__ float modulation_f(int phase, float phi, float inv_delta) {
    if (phase == 3) return 1.0f;
    if (phase == 0) return 0.0f;
    const float t = tanhf(phi * inv_delta);
    return phase == 1 ? 0.5f * (1.0f + t) : 0.5f * (1.0f - t);
}

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

template <int NC, int TX, int TY>
struct FusedTile {
    static constexpr int NT = TX * TY;    // nodes per tile
    static constexpr int NTH = NC * NT;   // threads: one per (node, component)
    static constexpr int W2 = TX + 4, H2 = TY + 4, A2 = W2 * H2;
    static constexpr int W1 = TX + 2, H1 = TY + 2, A1 = W1 * H1;
    static constexpr int NH2 = A2 - NT;  // R2 halo nodes
    static constexpr int NH1 = A1 - NT;  // R1 halo nodes
    float rho[3][NC][A2];  // delta rho per component (ring over planes)
    float cs[3][8][A2];    // D = C - I (6), s, s1 (ring over planes)
    float u[3][3][A1];     // total j (after A2), u (after B) (ring over planes)
    float jc[NC][3][A1];   // momentum per component of the entering plane
    float Fo[NC][3][NT];   // species forces of the tile nodes, phase B -> C
};

// Populations of one component and (optionally) D of one node, as loaded.
struct NodeLoad {
    float f[kQ];
    float d[6];
};

__device__ __forceinline__ void issue_load(const float* __restrict__ hs, const float* __restrict__ D, int64_t N,
                                           int64_t n, bool with_d, NodeLoad& v) {
#pragma unroll
    for (int a = 0; a < kQ; ++a) v.f[a] = hs[a * N + n];
    if (with_d) {
#pragma unroll
        for (int k = 0; k < 6; ++k) v.d[k] = D[k * N + n];
    }
}

// Phase A1 for one (node, component) of plane q: delta rho and momentum of this component,
// D when with_d.  Positions beyond a wall hold the wall layer's values (densities copy
// the wall layer; C and the stress are replaced in phase A2).
template <int NC, int TX, int TY>
__device__ __forceinline__ void phase_a1(FusedTile<NC, TX, TY>& L, int sq, int c, int lx, int ly, bool with_d,
                                         const NodeLoad& v) {
    using T = FusedTile<NC, TX, TY>;
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
}

// Phase A2 for one R2 position of plane q: wall ghosts of C (linear extrapolation from the
// two wall-adjacent layers, Sec. 2 boundary condition of C), the stress coefficients
// s = (eta_p/tau_p) m(phi) f(r), s1 = (eta_p/tau_p) m(phi) (f(r) - 1), and the total momentum.
template <int NC, int TX, int TY>
__device__ __forceinline__ void phase_a2(const DevParams& p, FusedTile<NC, TX, TY>& L, int sq, int y0, int k,
                                         unsigned& bad) {
    using T = FusedTile<NC, TX, TY>;
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
    const float trd = dv[0] + dv[1] + dv[2];
    const float den = p.L2m3 - trd;
    if (!(den > 0.0f) && gy >= -1 && gy <= p.ny) bad |= 2u;
    const float inv = 1.0f / den;
    const float pm = p.pstress * modulation_f(p.phase, phi, p.inv_delta);
    // ghost rows are written only by this thread and read after the next barrier
    if (gy == -1 || gy == p.ny) {
#pragma unroll
        for (int c = 0; c < 6; ++c) L.cs[sq][c][i2] = dv[c];
    }
    L.cs[sq][6][i2] = pm * p.L2m3 * inv;
    L.cs[sq][7][i2] = pm * trd * inv;
    if (lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) {
        const int i1 = (ly + 1) * T::W1 + lx + 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) L.u[sq][d][i1] = NC == 2 ? L.jc[0][d][i1] + L.jc[NC - 1][d][i1] : L.jc[0][d][i1];
    }
}

// Phase B for one in-domain node of plane q-1 at local (lx, ly): Shan-Chen force, polymer
// stress divergence, species forces and velocity; u replaces j in LDS slot sr.
template <int NC, int TX, int TY>
__device__ __forceinline__ void phase_b(const DevParams& p, FusedTile<NC, TX, TY>& L, int sp, int sr,
                                        int sn, int lx, int ly, float (&Fs)[2][3]) {
    using T = FusedTile<NC, TX, TY>;
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
    if (p.pstress != 0.0f) {
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

// One workgroup's share of a step: tile [x0, x0+TX) x [y0, y0+TY), planes [z0, z1).
template <int NC, int TX, int TY>
__device__ __forceinline__ void fused_tile(const DevParams& p, const float* __restrict__ h,
                                           float* __restrict__ hn, const float* __restrict__ D,
                                           float* __restrict__ Dn, unsigned* __restrict__ flags,
                                           FusedTile<NC, TX, TY>& L, int x0, int y0, int z0, int z1) {
    using T = FusedTile<NC, TX, TY>;
    static_assert(T::NH2 <= T::NT, "one R2 halo node per thread at most");
    static_assert(T::A1 <= 2 * T::NTH, "phase B covers the R1 region in two passes at most");

    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t N = p.N;
    const int64_t plane = (int64_t)nx * ny;

    const int tid = threadIdx.x;
    const int comp = tid / T::NT;   // component this thread loads and collides
    const int nid = tid % T::NT;    // tile node of this thread
    const int olx = nid % TX, oly = nid / TX;
    const int ogx = x0 + olx, ogy = y0 + oly;
    const bool active = ogx < nx && ogy < ny;
    const int oi2 = (oly + 2) * T::W2 + olx + 2;
    const int oi1 = (oly + 1) * T::W1 + olx + 1;
    const int ogxw = wrapn(ogx, nx);
    const int64_t own_xy = (int64_t)min(ogy, ny - 1) * nx + ogxw;
    const float* hs = h + (int64_t)comp * kQ * N;
    const bool fene = comp == 0;            // FENE-P and own C handled by component-0 threads
    const bool halo_d = comp == NC - 1;      // halo C loaded by the last component's threads

    // R2 halo node of this thread (fixed in x, y for the whole march)
    const bool has_halo = nid < T::NH2;
    int hlx = 0, hly = 0;
    if (has_halo) halo2_pos<TX, TY>(nid, hlx, hly);
    const int hgy = y0 + hly;
    const int64_t halo_xy = (int64_t)(hgy < 0 ? 0 : (hgy >= ny ? ny - 1 : hgy)) * nx + wrapn(x0 + hlx, nx);

    // own-column values of plane q-3 (their LDS ring slots are reused by plane q)
    float c_old[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float u_old[3] = {0.f, 0.f, 0.f};
    unsigned bad = 0u;

    NodeLoad pf_own, pf_halo;
    float held[kQ];  // own populations of plane q-1 (collided in phase C)
#pragma unroll
    for (int a = 0; a < kQ; ++a) held[a] = 0.0f;
    {
        const int64_t zoff = (int64_t)wrapn(z0 - 2, nz) * plane;
        issue_load(hs, D, N, zoff + own_xy, fene, pf_own);
        if (has_halo) issue_load(hs, D, N, zoff + halo_xy, halo_d, pf_halo);
    }

    for (int q = z0 - 2; q <= z1 + 1; ++q) {
        const int sq = ((q % 3) + 3) % 3;
        const bool do_c = q >= z0 + 1 && q <= z1 && active;

        // ---------------- A1: consume plane q (prefetched) ----------------
        phase_a1<NC, TX, TY>(L, sq, comp, olx, oly, fene, pf_own);
        if (has_halo) phase_a1<NC, TX, TY>(L, sq, comp, hlx, hly, halo_d, pf_halo);
        // own populations: plane q-1 (held since the previous plane) is collided in phase C,
        // plane q is kept for the next one; each population is read from HBM once per step
        float hv[kQ], cur[kQ];
#pragma unroll
        for (int a = 0; a < kQ; ++a) {
            hv[a] = held[a];
            cur[a] = pf_own.f[a];
        }
        const int r = wrapn(q - 1, nz);
        const int64_t nself = (int64_t)r * plane + own_xy;
        // prefetch plane q+1
        if (q + 1 <= z1 + 1) {
            const int64_t zoff = (int64_t)wrapn(q + 1, nz) * plane;
            issue_load(hs, D, N, zoff + own_xy, fene, pf_own);
            if (has_halo) issue_load(hs, D, N, zoff + halo_xy, halo_d, pf_halo);
        }
        lds_barrier();

        // ---------------- A2: ghosts, stress coefficients, total momentum ----------------
        for (int k = tid; k < T::A2; k += T::NTH) phase_a2<NC, TX, TY>(p, L, sq, y0, k, bad);
        lds_barrier();

        // ---------------- B: forces and velocity on plane q-1 (tile + 1 halo) -------------
        if (q >= z0) {
            const int sr = ((q - 1) % 3 + 3) % 3;
            const int sp = ((q - 2) % 3 + 3) % 3;
            for (int k = tid; k < T::A1; k += T::NTH) {
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
                phase_b<NC, TX, TY>(p, L, sp, sr, sq, lx, ly, Fs);
                if (k < T::NT) {
#pragma unroll
                    for (int s = 0; s < NC; ++s)
#pragma unroll
                        for (int d = 0; d < 3; ++d) L.Fo[s][d][k] = Fs[s][d];
                }
            }
        }
        lds_barrier();

        // ---------------- C: collide + stream plane q-1 (own node, own component) ----------
        if (do_c) {
            const int sr = ((q - 1) % 3 + 3) % 3;
            float u[3], F[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                u[d] = L.u[sr][d][oi1];
                F[d] = L.Fo[comp][d][nid];
            }
            const float drA = L.rho[sr][0][oi2];
            const float drB = NC == 2 ? L.rho[sr][NC - 1][oi2] : 0.0f;
            const float drs = comp == 0 ? drA : drB;
            const float rA = p.rho0[0] + drA;
            const float rB = NC == 2 ? p.rho0[1] + drB : 0.0f;
            const float rs = comp == 0 ? rA : rB;
            const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            float tau = p.tauA;
            if (NC == 2) {
                const float phi = (rA - rB) / (rA + rB);
                tau = p.tauB + (p.tauA - p.tauB) * 0.5f * (1.0f + tanhf(phi * p.inv_delta));
            }
            const float om = 1.0f / tau;
            const float cfac = 1.0f - 0.5f * om;
            const int xp = ogxw + 1 == nx ? 0 : ogxw + 1;
            const int xm = ogxw == 0 ? nx - 1 : ogxw - 1;
            const int zp = r + 1 == nz ? 0 : r + 1;
            const int zm = r == 0 ? nz - 1 : r - 1;
            const float uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
            float* hns = hn + (int64_t)comp * kQ * N;
            float check = 0.0f;
#pragma unroll
            for (int a = 0; a < kQ; ++a) {
                const float ha = hv[a];
                const float cu = cx(a) * u[0] + cy(a) * u[1] + cz(a) * u[2];
                const float cF = cx(a) * F[0] + cy(a) * F[1] + cz(a) * F[2];
                const float heq = wgt(a) * (drs + rs * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
                const float src = wgt(a) * (3.0f * (cF - uF) + 9.0f * cu * cF);
                const float post = ha - om * (ha - heq) + cfac * src;
                check += post;
                const int yd = ogy + cy(a);
                if (yd >= 0 && yd < ny) {
                    const int xd = cx(a) == 0 ? ogxw : (cx(a) > 0 ? xp : xm);
                    const int zd = cz(a) == 0 ? r : (cz(a) > 0 ? zp : zm);
                    // streaming stores: the next step reads them, this launch does not
                    __builtin_nontemporal_store(post, &hns[a * N + (int64_t)zd * plane + (int64_t)yd * nx + xd]);
                } else {
                    const float* uw = yd < 0 ? p.ub : p.ut;
                    const float cuw = cx(a) * uw[0] + cz(a) * uw[2];
                    __builtin_nontemporal_store(post - 6.0f * wgt(a) * rs * cuw, &hns[opp(a) * N + nself]);
                }
            }
            if (!isfinite(check)) bad |= 1u;
        }
#pragma unroll
        for (int a = 0; a < kQ; ++a) held[a] = cur[a];

        // ---------------- D: FENE-P on plane q-2 (own node, component-0 threads) ----------
        if (fene && q >= z0 + 2 && active) {
            const int t = wrapn(q - 2, nz);
            const int st = ((q - 2) % 3 + 3) % 3;
            const int st1 = ((q - 1) % 3 + 3) % 3;
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
            float dnew[6];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
#pragma unroll
                for (int b = a; b < 3; ++b) {
                    const int kk = sidx(a, b);
                    float stv = Gm[b][a] + Gm[a][b];
#pragma unroll
                    for (int k = 0; k < 3; ++k) stv += Gm[k][a] * d0[sidx(k, b)] + d0[sidx(a, k)] * Gm[k][b];
                    const float relax = (f * d0[kk] + (a == b ? fm1 : 0.0f)) * p.inv_tau_p;
                    dnew[kk] = d0[kk] + (-adv[kk] + stv - relax);
                }
            }
            const int64_t nt = (int64_t)t * plane + own_xy;
            float check = 0.0f;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                __builtin_nontemporal_store(dnew[k], &Dn[k * N + nt]);
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
    }
    if (bad) atomicOr(flags, bad);
}

template <int NC, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY, (NC == 1 ? 2 : 1)) void k_fused(
    DevParams p, const float* __restrict__ h, float* __restrict__ hn, const float* __restrict__ D,
    float* __restrict__ Dn, unsigned* __restrict__ flags, int zchunk) {
    __shared__ FusedTile<NC, TX, TY> L;
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const int64_t bid = xcd_remap_f(blockIdx.x, gridDim.x);
    const int tx_i = (int)(bid % ntx);
    const int64_t rem = bid / ntx;
    const int ty_i = (int)(rem % nty);
    const int zc_i = (int)(rem / nty);
    const int z0 = zc_i * zchunk;
    fused_tile<NC, TX, TY>(p, h, hn, D, Dn, flags, L, tx_i * TX, ty_i * TY, z0, min(z0 + zchunk, p.nz));
}

// Many independent lattices in one launch: each workgroup takes one entry of the work
// table (instance, tile, z range) and steps that part of its instance.  The instance's
// buffer holding time level n is cur ^ parity, so a two-launch graph (parity 0, 1)
// replays any even number of steps.
template <int NC, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY, (NC == 1 ? 2 : 1)) void k_fused_batch(
    const BatchInstance* __restrict__ inst, const WorkItem* __restrict__ work, int parity) {
    __shared__ FusedTile<NC, TX, TY> L;
    const int64_t bid = xcd_remap_f(blockIdx.x, gridDim.x);
    const WorkItem w = work[bid];
    const BatchInstance& bi = inst[w.inst];
    const DevParams p = bi.p;
    const int c = bi.cur ^ parity;
    fused_tile<NC, TX, TY>(p, bi.h[c], bi.h[c ^ 1], bi.D[c], bi.D[c ^ 1], bi.flags, L, w.x0, w.y0, w.z0, w.z1);
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
        if (tile == 1)
            hipLaunchKernelGGL((k_fused_batch<1, 32, 16>), grid, dim3(512), 0, s, inst, work, parity);
        else if (tile == 2)
            hipLaunchKernelGGL((k_fused_batch<1, 16, 16>), grid, dim3(256), 0, s, inst, work, parity);
        else
            hipLaunchKernelGGL((k_fused_batch<1, 32, 8>), grid, dim3(256), 0, s, inst, work, parity);
    }
    return hipGetLastError();
}

// tile extent of a tuning choice (two components run the 32x16 choice as 32x8)
void fused_tile_shape(int ncomp, int tile, int* tx, int* ty) {
    *tx = tile == 2 ? 16 : 32;
    *ty = tile == 2 ? 16 : ((tile == 1 && ncomp == 1) ? 16 : 8);
}

hipError_t launch_fused(const DevParams& p, const Buffers& b, const Tuning& t, hipStream_t s) {
    const int zc = t.zchunk > 0 ? t.zchunk : p.nz;
    if (p.nc == 2) {
        // two components run one thread per (node, component): the 32x16 tile would need
        // 1024 threads at half the registers, so it maps to 32x8
        if (t.tile == 2) return launch_fused_t<2, 16, 16>(p, b, zc, s);
        return launch_fused_t<2, 32, 8>(p, b, zc, s);
    }
    if (t.tile == 1) return launch_fused_t<1, 32, 16>(p, b, zc, s);
    if (t.tile == 2) return launch_fused_t<1, 16, 16>(p, b, zc, s);
    return launch_fused_t<1, 32, 8>(p, b, zc, s);
}

}  // namespace lbfd

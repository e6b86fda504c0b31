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
// re-reads of neighbouring tiles are meant to hit a cache: blocks are mapped so that the
// tiles running together on one XCD form a compact group and the groups running together
// on the chip form a band (tile_of_block).
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
template <int NC, int TX, int TY, bool TP>
struct FusedTile {
    static constexpr int NT = TX * TY;    // nodes per tile
    static constexpr int NTH = NC * NT;   // threads: one per (node, component)
    static constexpr int W2 = TX + 4, H2 = TY + 4, A2 = W2 * H2;
    static constexpr int W1 = TX + 2, H1 = TY + 2, A1 = W1 * H1;
    static constexpr int NH2 = A2 - NT;  // R2 halo nodes
    static constexpr int NH1 = A1 - NT;  // R1 halo nodes
    float rho[3][NC][A2];       // delta rho per component (ring over planes)
    float cs[3][8][A2];         // D = C - I (6), s, s1 (ring over planes)
    float u[3][3][A1];          // total j (after A2), u (after B) (ring over planes)
    float Fo[NC][3][NT];        // species forces of the tile nodes, phase B -> C
    float fpl[2][NT];           // f+(phi) of the tile nodes, planes q and q-1
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
template <int NC, int TX, int TY, bool TP>
__device__ __forceinline__ void phase_a2(const DevParams& p, FusedTile<NC, TX, TY, TP>& L, int sq, int s2, int y0, int k,
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
    if (NC == 2 && lx >= 0 && lx < TX && ly >= 0 && ly < TY) L.fpl[s2][ly * TX + lx] = 0.5f * (1.0f + th);
    if (!TP && lx >= -1 && lx <= TX && ly >= -1 && ly <= TY) {
        const int i1 = (ly + 1) * T::W1 + lx + 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) L.u[sq][d][i1] = NC == 2 ? L.jc[0][d][i1] + L.jc[NC - 1][d][i1] : L.jc[0][d][i1];
    }
}

// Phase B for one in-domain node of plane q-1 at local (lx, ly): Shan-Chen force, polymer
// stress divergence, species forces and velocity; u replaces j in LDS slot sr.
template <int NC, int TX, int TY, bool TP>
__device__ __forceinline__ void phase_b(const DevParams& p, FusedTile<NC, TX, TY, TP>& L, int sp, int sr,
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

// One workgroup's share of a step: tile [x0, x0+TX) x [y0, y0+TY), planes [z0, z1).
// TP = false: single pass, the moments are formed here from the populations of the tile
// and its halo.  TP = true: second pass of the two-pass step, delta rho and j of every
// node come from `mom` (written by the moments pass over the same time level), so only the
// tile's own populations are read, once, for the collision.
template <int NC, int TX, int TY, bool TP>
__device__ __forceinline__ void fused_tile(const DevParams& p, const float* __restrict__ h,
                                           float* __restrict__ hn, const float* __restrict__ D,
                                           float* __restrict__ Dn, unsigned* __restrict__ flags,
                                           FusedTile<NC, TX, TY, TP>& L, int x0, int y0, int z0, int z1,
                                           const float* __restrict__ mom) {
    using T = FusedTile<NC, TX, TY, TP>;
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

    // plane q+1 is loaded while plane q is processed; the loads land in the registers that
    // phase A1 has just emptied, so no copy (and no early wait) sits on the loop edge
    NodeLoad pf_own, pf_halo;
    // two-pass: positions of the tile + halo this thread loads (moments and D), and the own
    // populations of the plane collided next
    constexpr int KP = (T::A2 + T::NTH - 1) / T::NTH;
    MomLoad<NC> mpf[KP];
    uint32_t mpos[KP];
    float own_pop[kQ];
    if (TP) {
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const int k = tid + i * T::NTH;
            const int lx = k % T::W2 - 2, ly = k / T::W2 - 2;
            const int gy = min(max(y0 + ly, 0), ny - 1);
            mpos[i] = (uint32_t)gy * (uint32_t)nx + (uint32_t)wrapn(x0 + lx, nx);
        }
#pragma unroll
        for (int a = 0; a < kQ; ++a) own_pop[a] = 0.0f;
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
        const int sq = ((q % 3) + 3) % 3;
        const int s2 = q & 1;
        const bool do_c = q >= z0 + 1 && q <= z1 && active;

        // ---------------- A1: consume plane q, then request plane q+1 ----------------
        if constexpr (TP) {
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const int k = tid + i * T::NTH;
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
        for (int k = tid; k < T::A2; k += T::NTH) phase_a2<NC, TX, TY, TP>(p, L, sq, s2, y0, k, bad);
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
                phase_b<NC, TX, TY, TP>(p, L, sp, sr, sq, lx, ly, Fs);
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
        // BGK with the forcing source (eq. LB, Lambda = I/tau(phi)).  For an opposite pair
        // (a, a+1) the equilibrium and the source split into parts even and odd in c, formed
        // once per pair; each population is then relaxed as h - (h - h_eq)/tau + (1 -
        // 1/(2 tau)) S, the form whose rounding keeps the species mass drift smallest.
        if (do_c) {
            const int sr = ((q - 1) % 3 + 3) % 3;
            const int p2 = s2 ^ 1;
            const int r = wrapn(q - 1, nz);
            float u[3], F[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                u[d] = L.u[sr][d][oi1];
                F[d] = L.Fo[comp][d][nid];
            }
            const float drs = L.rho[sr][comp][oi2];
            const float rs = (comp == 0 ? p.rho0[0] : p.rho0[1]) + drs;
            const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const float tau = NC == 2 ? p.tauB + (p.tauA - p.tauB) * L.fpl[p2][nid] : p.tauA;
            const float om = 1.0f / tau;
            const float cfac = 1.0f - 0.5f * om;
            const float uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
            const float b = -1.5f * uu;
            // stress coupling (eq. MODEtransformation): T_s = (rho_s/rho) T lowers the second
            // moment of this species' equilibrium by -4.5 w (c.T_s.c - tr T_s/3) per direction
            const bool stress_eq = p.coupling == 1 && p.pstress != 0.0f;
            float Ts[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (stress_eq) {
                const float rtot = p.rho0[0] + L.rho[sr][0][oi2] + (NC == 2 ? p.rho0[1] + L.rho[sr][NC - 1][oi2] : 0.0f);
                const float share = rs / rtot;
                const float sv = share * L.cs[sr][6][oi2], s1v = share * L.cs[sr][7][oi2];
#pragma unroll
                for (int k = 0; k < 6; ++k) Ts[k] = sv * L.cs[sr][k][oi2] + (k < 3 ? s1v : 0.0f);
            }
            const float trs3 = (Ts[0] + Ts[1] + Ts[2]) * (1.0f / 3.0f);
            const uint32_t zrow[3] = {(uint32_t)(r == 0 ? nz - 1 : r - 1) * plane, (uint32_t)r * plane,
                                      (uint32_t)(r + 1 == nz ? 0 : r + 1) * plane};
            const uint32_t bself = (zrow[1] + yrow + xcol[1]) * 4u;
            float check;
            {
                const float w = wgt(0);
                const float ha = TP ? own_pop[0] : L.pop[TP ? 0 : p2][TP ? 0 : comp][0][TP ? 0 : nid];
                const float heq0 = w * (drs + rs * b) + (stress_eq ? 4.5f * w * trs3 : 0.0f);
                const float post = ha - om * (ha - heq0) + cfac * (w * (-3.0f * uF));
                st_off(hns, bself, post);
                check = post;
            }
#pragma unroll
            for (int a = 1; a < kQ; a += 2) {
                const float w = wgt(a);
                const float cu = cx(a) * u[0] + cy(a) * u[1] + cz(a) * u[2];
                const float cF = cx(a) * F[0] + cy(a) * F[1] + cz(a) * F[2];
                float ee = w * (drs + rs * (4.5f * cu * cu + b));  // equilibrium, even part
                if (stress_eq) {
                    const float cTc = float(cx(a) * cx(a)) * Ts[0] + float(cy(a) * cy(a)) * Ts[1] +
                                      float(cz(a) * cz(a)) * Ts[2] +
                                      2.0f * (float(cx(a) * cy(a)) * Ts[3] + float(cx(a) * cz(a)) * Ts[4] +
                                              float(cy(a) * cz(a)) * Ts[5]);
                    ee -= 4.5f * w * (cTc - trs3);
                }
                const float eo = (3.0f * w) * rs * cu;                   // equilibrium, odd part
                const float se = w * (9.0f * cu * cF - 3.0f * uF);       // source, even part
                const float so = (3.0f * w) * cF;                        // source, odd part
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int bq = a + e;
                    const float ha = TP ? own_pop[bq] : L.pop[TP ? 0 : p2][TP ? 0 : comp][bq][TP ? 0 : nid];
                    const float heq = e == 0 ? ee + eo : ee - eo;
                    const float src = e == 0 ? se + so : se - so;
                    const float post = ha - om * (ha - heq) + cfac * src;
                    check += post;
                    const int yd = ogy + cy(bq);
                    if (yd >= 0 && yd < ny) {
                        const uint32_t dst = zrow[cz(bq) + 1] + yrow + (uint32_t)(cy(bq) * nx) + xcol[cx(bq) + 1];
                        st_off(hns + (size_t)bq * N, dst * 4u, post);
                    } else {
                        // moving-wall bounce-back (Sec. 3.1 walls): the link returns as opp(bq)
                        const float* uw = yd < 0 ? p.ub : p.ut;
                        const float cuw = cx(bq) * uw[0] + cz(bq) * uw[2];
                        st_off(hns + (size_t)opp(bq) * N, bself, post - 6.0f * wgt(bq) * rs * cuw);
                    }
                }
            }
            if (!isfinite(check)) bad |= 1u;
        }
        if (TP && q >= z0 && q < z1) {
            // own populations of plane q, collided in the next iteration; the registers were
            // emptied by phase C just above
            const uint32_t bo = ((uint32_t)wrapn(q, nz) * plane + own_xy) * 4u;
#pragma unroll
            for (int a = 0; a < kQ; ++a) own_pop[a] = ld_off(hs + (size_t)a * N, bo);
        }

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
            const uint32_t bt = ((uint32_t)t * plane + own_xy) * 4u;
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
    fused_tile<NC, TX, TY, false>(p, h, hn, D, Dn, flags, L, tx_i * TX, ty_i * TY, z0, min(z0 + zchunk, p.nz),
                                  nullptr);
}

// Second pass of the two-pass step: the moments of the whole lattice at time level n are
// in `mom` (delta rho per component, then j), written by the moments pass.  Without the
// population ring its LDS (72 KB for 32x8, two components) admits two workgroups per CU;
// the launch bound asks for 4 waves per SIMD (128 VGPRs) so that both fit.
template <int NC, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY, 4) void k_fused2(
    DevParams p, const float* __restrict__ h, float* __restrict__ hn, const float* __restrict__ D,
    float* __restrict__ Dn, const float* __restrict__ mom, unsigned* __restrict__ flags, int zchunk) {
    __shared__ FusedTile<NC, TX, TY, true> L;
    const int ntx = (p.nx + TX - 1) / TX, nty = (p.ny + TY - 1) / TY;
    const int gxw = min(ntx, 256 / TX);
    const int gyh = min(nty, max(1, 32 / gxw));
    int tx_i, ty_i, zc_i;
    tile_of_block(blockIdx.x, gridDim.x, ntx, nty, gxw, gyh, tx_i, ty_i, zc_i);
    const int z0 = zc_i * zchunk;
    fused_tile<NC, TX, TY, true>(p, h, hn, D, Dn, flags, L, tx_i * TX, ty_i * TY, z0, min(z0 + zchunk, p.nz), mom);
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
    fused_tile<NC, TX, TY, false>(p, bi.h[c], bi.h[c ^ 1], bi.D[c], bi.D[c ^ 1], bi.flags, L, w.x0, w.y0, w.z0, w.z1,
                                  nullptr);
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
        return launch_fused2_t<2, 32, 8>(p, b, zc, s);
    }
    if (t.tile == 2) return launch_fused2_t<1, 16, 16>(p, b, zc, s);
    return launch_fused2_t<1, 32, 8>(p, b, zc, s);
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

// d3q19.h -- D3Q19 lattice constants and index helpers for the gfx950 kernels.
//
// Velocity ordering (a convention; the paper fixes only the weights, Sec. 2):
//   0: rest; 1-6: +-x, +-y, +-z; 7-18: the 12 edge diagonals in the xy, xz, yz planes.
// Opposite directions are adjacent pairs (1,2), (3,4), ..., (17,18), so the odd index
// of each pair is the "+" member.  Weights 1/3, 1/18, 1/36 (Sec. 2, D3Q19 weights).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfd {

constexpr int kQ = 19;
constexpr float kCs2 = 1.0f / 3.0f;

__host__ __device__ constexpr int cx(int a) {
    constexpr int t[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[a];
}
__host__ __device__ constexpr int cy(int a) {
    constexpr int t[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[a];
}
__host__ __device__ constexpr int cz(int a) {
    constexpr int t[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[a];
}
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
__host__ __device__ constexpr float wgt(int a) {
    return a == 0 ? 1.0f / 3.0f : (a <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}

// A weight as the FP32 pair w = hi + lo (hi the FP32 value nearest the weight, lo the rest),
// and the same for 3w.  Products with the weights are formed as fma(hi, x, lo x): the exact
// product hi x plus the small lo x, rounded once, so the weight itself enters the result.
// hi x alone would scale every term of one direction class by the same factor (1/3 rounds
// up by 3e-8 relative, 1/18 and 1/36 by 7e-9), and a collision built on it would create
// mass in proportion to delta rho and momentum in proportion to rho u at every step,
// coherently across the lattice.  (The other order, fma(lo, x, hi x), rounds hi x first and
// then adds lo x to a value already rounded: a term below half an ulp of it is lost.)
struct Wt {
    float w, wl, w3, w3l;
};
__host__ __device__ constexpr double wexact(int a) {
    return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr Wt wsplit(int a) {
    return Wt{(float)wexact(a), (float)(wexact(a) - (double)(float)wexact(a)), (float)(3.0 * wexact(a)),
              (float)(3.0 * wexact(a) - (double)(float)(3.0 * wexact(a)))};
}
__device__ __forceinline__ float wmul(float hi, float lo, float x) { return fmaf(hi, x, lo * x); }

// symmetric 3x3 tensor component index in (xx, yy, zz, xy, xz, yz) order
__host__ __device__ constexpr int sidx(int i, int j) {
    return i == j ? i : ((i + j) == 1 ? 3 : ((i + j) == 2 ? 4 : 5));
}

// c_a . u_w for a wall velocity with no wall-normal component, the zero terms left out
// (0 * x is not folded under IEEE rules, and such products of a per-lane wall velocity
// would otherwise be formed for every direction)
__host__ __device__ __forceinline__ float wall_cu(int a, const float* uw) {
    const int ex = cx(a), ez = cz(a);
    if (ex != 0 && ez != 0) return float(ex) * uw[0] + float(ez) * uw[2];
    if (ex != 0) return ex > 0 ? uw[0] : -uw[0];
    if (ez != 0) return ez > 0 ? uw[2] : -uw[2];
    return 0.0f;
}

// Periodic wrap for |d| <= 1 offsets.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// Wall-normal clamp (ghost layer copies the wall-adjacent node).
__device__ __forceinline__ int clampy(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

}  // namespace lbfd

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

// symmetric 3x3 tensor component index in (xx, yy, zz, xy, xz, yz) order
__host__ __device__ constexpr int sidx(int i, int j) {
    return i == j ? i : ((i + j) == 1 ? 3 : ((i + j) == 2 ? 4 : 5));
}

// Periodic wrap for |d| <= 1 offsets.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// Wall-normal clamp (ghost layer copies the wall-adjacent node).
__device__ __forceinline__ int clampy(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

}  // namespace lbfd

// fene_chol.h -- the Cholesky-log update of the FENE-P conformation at one node, shared by
// the per-node split path and the chained step.
#pragma once
#include <hip/hip_runtime.h>

namespace lbfd {

// One step of the Cholesky scheme for the FENE-P equation (Sec. 2, paragraph on the FENE-P
// solver) at one node, in deviation form so that FP32 keeps the departures from I.
// d: C - I (xx, yy, zz, xy, xz, yz); rc: dC/dt.  With f = (L^2 - 3)/(L^2 - tr C),
// sigma = f C = I + S, S = (f - 1) I + f d, and sigma' = f rc + C f^2 tr(rc)/(L^2 - 3).  For
// sigma = L L^t (L lower triangular, l_ii = 1 + m_ii) the factor moves as L' = L Phi(A),
// A = L^-1 sigma' L^-t, Phi = strict lower part + half the diagonal, so (ln l_ii)' = A_ii/2.
// y = (ln l11, l21, ln l22, l31, l32, ln l33) takes one Adams-Bashforth-2 step (forward
// Euler when hist is false); yd returns the rate.  Since f = (L^2 - 3 + tr sigma)/L^2, the
// new C is sigma/f: SPD with tr C < L^2 by construction.  Returns false if sigma is not SPD.
__device__ __forceinline__ bool cholesky_ab2_step(float L2, float L2m3, const float d[6], const float rc[6],
                                                  const float yprev[6], bool hist, float dn[6], float yd[6]) {
    const float trd = d[0] + d[1] + d[2], trr = rc[0] + rc[1] + rc[2];
    const float inv = 1.0f / (L2m3 - trd);
    const float f = L2m3 * inv, fm1 = trd * inv;
    const float g = f * f * trr / L2m3;
    float S[6], r[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        S[k] = f * d[k] + (k < 3 ? fm1 : 0.0f);
        r[k] = f * rc[k] + g * (d[k] + (k < 3 ? 1.0f : 0.0f));
    }
    // Cholesky factor of I + S; m = l - 1 on the diagonal, formed without cancellation
    const float b11 = S[0];
    if (!(b11 > -1.0f)) return false;
    const float m11 = b11 / (1.0f + sqrtf(1.0f + b11));
    const float l11 = 1.0f + m11, i11 = 1.0f / l11;
    const float l21 = S[3] * i11, l31 = S[4] * i11;
    const float b22 = S[1] - l21 * l21;
    if (!(b22 > -1.0f)) return false;
    const float m22 = b22 / (1.0f + sqrtf(1.0f + b22));
    const float l22 = 1.0f + m22, i22 = 1.0f / l22;
    const float l32 = (S[5] - l31 * l21) * i22;
    const float b33 = S[2] - l31 * l31 - l32 * l32;
    if (!(b33 > -1.0f)) return false;
    const float m33 = b33 / (1.0f + sqrtf(1.0f + b33));
    const float l33 = 1.0f + m33, i33 = 1.0f / l33;
    // X = L^-1 R (R symmetric 3x3 from r), then A = L^-1 X^t (A symmetric)
    const float R[3][3] = {{r[0], r[3], r[4]}, {r[3], r[1], r[5]}, {r[4], r[5], r[2]}};
    float X[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        X[0][j] = R[0][j] * i11;
        X[1][j] = (R[1][j] - l21 * X[0][j]) * i22;
        X[2][j] = (R[2][j] - l31 * X[0][j] - l32 * X[1][j]) * i33;
    }
    float A[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j][0] = X[j][0] * i11;
        A[j][1] = (X[j][1] - l21 * A[j][0]) * i22;
        A[j][2] = (X[j][2] - l31 * A[j][0] - l32 * A[j][1]) * i33;
    }
    // L' = L Phi(A)
    const float p11 = 0.5f * A[0][0], p22 = 0.5f * A[1][1], p33 = 0.5f * A[2][2];
    const float p21 = A[1][0], p31 = A[2][0], p32 = A[2][1];
    yd[0] = p11;
    yd[1] = l21 * p11 + l22 * p21;
    yd[2] = p22;
    yd[3] = l31 * p11 + l32 * p21 + l33 * p31;
    yd[4] = l32 * p22 + l33 * p32;
    yd[5] = p33;
    float st[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) st[k] = hist ? 1.5f * yd[k] - 0.5f * yprev[k] : yd[k];
    // l_ii' = l_ii exp(step): m' = m + e + m e with e = exp(step) - 1
    const float e1 = expm1f(st[0]), e2 = expm1f(st[2]), e3 = expm1f(st[5]);
    const float n11 = m11 + e1 + m11 * e1, n22 = m22 + e2 + m22 * e2, n33 = m33 + e3 + m33 * e3;
    const float q11 = 1.0f + n11, q21 = l21 + st[1], q22 = 1.0f + n22;
    const float q31 = l31 + st[3], q32 = l32 + st[4];
    // S' = L' L'^t - I
    float Sn[6];
    Sn[0] = n11 * (2.0f + n11);
    Sn[1] = q21 * q21 + n22 * (2.0f + n22);
    Sn[2] = q31 * q31 + q32 * q32 + n33 * (2.0f + n33);
    Sn[3] = q21 * q11;
    Sn[4] = q31 * q11;
    Sn[5] = q31 * q21 + q32 * q22;
    // f' = 1 + tr S'/L^2;  C' - I = (S' - (tr S'/L^2) I) / f'
    const float t = (Sn[0] + Sn[1] + Sn[2]) / L2;
    const float ifn = 1.0f / (1.0f + t);
#pragma unroll
    for (int k = 0; k < 6; ++k) dn[k] = (Sn[k] - (k < 3 ? t : 0.0f)) * ifn;
    return true;
}

}  // namespace lbfd

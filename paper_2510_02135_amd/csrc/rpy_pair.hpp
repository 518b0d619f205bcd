// Pair-kernel data types and constants of the generalised RPY blocks,
// shared by the pair, adjoint and batched kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace rpy {

// ---------------------------------------------------------------------------
// Device vector types: one particle's 3-vector padded to 4 lanes.
// ---------------------------------------------------------------------------
template <typename Real> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };
template <typename Real> using vec4_t = typename V4<Real>::type;

// Pair-kernel constants, all in units of k = 1/(8 pi eta) so that the pair
// loop never multiplies by k; the epilogue does it once per output.
//   far  (r >= 2a):  A = 1/r + (2a^2/3)/r^3      B = 1/r^3 - 2a^2/r^5
//                    G = 1/r^3  D = -1/(2r^3)    E = 3/(2r^5)
//   near (r <  2a):  A = 4/(3a) - 3r/(8a^2)      B = 1/(8a^2 r)
//                    G = 1/(2a^3) - 3r/(16a^4)
//                    D = 1/a^3 - 27r/(32a^4) + 5r^3/(64a^6)
//                    E = 9/(32a^4 r) - 3r/(64a^6)
// contribution of source j to target i, d = X_i - X_j:
//   U_i += A F + B (d.F) d + G (T x d)
//   W_i += G (F x d) + D T + E (d.T) d
template <typename Real>
struct PairConst {
    Real two_a2_3;   // 2a^2/3
    Real m_two_a2;   // -2a^2
    Real four_a2;    // (2a)^2, near-branch threshold on r^2
    Real nA0, nA1;   // 4/(3a), -3/(8a^2)
    Real nB;         // 1/(8a^2)
    Real nG0, nG1;   // 1/(2a^3), -3/(16a^4)
    Real nD0, nD1, nD3;  // 1/a^3, -27/(32a^4), 5/(64a^6)
    Real nE_1, nE1;  // 9/(32a^4), -3/(64a^6)
};

template <typename Real>
inline PairConst<Real> make_pair_const(double a) {
    PairConst<Real> c;
    const double a2 = a * a, a3 = a2 * a, a4 = a2 * a2, a6 = a3 * a3;
    c.two_a2_3 = Real(2.0 * a2 / 3.0);
    c.m_two_a2 = Real(-2.0 * a2);
    c.four_a2 = Real(4.0 * a2);
    c.nA0 = Real(4.0 / (3.0 * a));
    c.nA1 = Real(-3.0 / (8.0 * a2));
    c.nB = Real(1.0 / (8.0 * a2));
    c.nG0 = Real(1.0 / (2.0 * a3));
    c.nG1 = Real(-3.0 / (16.0 * a4));
    c.nD0 = Real(1.0 / a3);
    c.nD1 = Real(-27.0 / (32.0 * a4));
    c.nD3 = Real(5.0 / (64.0 * a6));
    c.nE_1 = Real(9.0 / (32.0 * a4));
    c.nE1 = Real(-3.0 / (64.0 * a6));
    return c;
}

}  // namespace rpy

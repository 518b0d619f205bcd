// Pair term of the adjoint of the RPY mobility product, shared by the
// adjoint kernel (rpy_adjoint.hip) and the symmetric pair mode
// (rpy_sym.hip).  See rpy_adjoint.hip for the formulas.
#pragma once

#include <hip/hip_runtime.h>

#include "rpy_device.hpp"

namespace rpy {

template <typename Real>
__device__ __forceinline__ Real dot3(Real ax, Real ay, Real az, Real bx, Real by, Real bz) {
    return fma(ax, bx, fma(ay, by, az * bz));
}

// Target-side data of one lane.
template <typename Real, bool ANG>
struct Tgt {
    Real x, y, z;
    Real fx, fy, fz;
    Real gx, gy, gz;          // g_U
    Real tx, ty, tz;          // T      (ANG)
    Real hx, hy, hz;          // g_W    (ANG)
};

// Output accumulator layout: [0..2] dX, [3..5] dF (= (M g)_U), [6..8] dT.
// With BOTH, the same pair's terms for the source particle j (target k's
// records, separation -d) go to jacc as well: dX_j -= the dX_k term (the
// pair's part of L depends on X_k - X_j only), and (M g)_j gets the blocks
// at -d applied to k's cotangents.
template <typename Real, bool ANG, bool BOTH>
__device__ __forceinline__ void adj_pair(const Tgt<Real, ANG> &k, const vec4_t<Real> &sp, const vec4_t<Real> &sf,
                                         const vec4_t<Real> &sg, const vec4_t<Real> &st, const vec4_t<Real> &sh,
                                         const PairConst<Real> &c, Real *acc, Real *jacc) {
    const Real dx = k.x - sp.x, dy = k.y - sp.y, dz = k.z - sp.z;
    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    const Real ri3 = ri * ri2;
    const Real ri5 = ri3 * ri2;
    const Real ri7 = ri5 * ri2;
    // far branch; c.m_two_a2 = -2a^2, c.two_a2_3 = 2a^2/3
    Real A = fma(c.two_a2_3, ri3, ri);
    Real B = fma(c.m_two_a2, ri5, ri3);
    Real Ar = fma(c.m_two_a2, ri5, -ri3);                    // -1/r^3 - 2a^2/r^5
    Real Br = fma(Real(-5) * c.m_two_a2, ri7, Real(-3) * ri5);  // -3/r^5 + 10a^2/r^7
    Real G = ri3, Gg = ri3, Gr = Real(-3) * ri5;
    Real D = Real(-0.5) * ri3, Dr = Real(1.5) * ri5;
    Real E = Real(1.5) * ri5, Er = Real(-7.5) * ri7;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        const Real rs = r2 > Real(0) ? ri : Real(0);
        const Real r = r2 * rs;
        const Real rs3 = rs * rs * rs;
        A = fma(c.nA1, r, c.nA0);
        Ar = c.nA1 * rs;
        B = c.nB * rs;
        Br = -c.nB * rs3;
        if constexpr (ANG) {
            G = fma(c.nG1, r, c.nG0);
            Gg = r2 > Real(0) ? G : Real(0);
            Gr = c.nG1 * rs;
            D = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
            Dr = fma(c.nD1, rs, Real(3) * c.nD3 * r);
            E = fma(c.nE_1, rs, c.nE1 * r);
            Er = fma(-c.nE_1, rs3, c.nE1 * rs);
        }
    }
    // dot products shared by the terms
    const Real dFj = dot3(dx, dy, dz, sf.x, sf.y, sf.z);
    const Real dgj = dot3(dx, dy, dz, sg.x, sg.y, sg.z);
    const Real dFk = dot3(dx, dy, dz, k.fx, k.fy, k.fz);
    const Real dgk = dot3(dx, dy, dz, k.gx, k.gy, k.gz);
    const Real gkFj = dot3(k.gx, k.gy, k.gz, sf.x, sf.y, sf.z);
    const Real gjFk = dot3(sg.x, sg.y, sg.z, k.fx, k.fy, k.fz);
    Real S = fma(Ar, gkFj + gjFk, Br * fma(dgk, dFj, dgj * dFk));
    const Real b1 = B * dFj, b2 = B * dgk, b3 = B * dFk, b4 = B * dgj;
    Real ox = fma(b1, k.gx, fma(b2, sf.x, fma(b3, sg.x, b4 * k.fx)));
    Real oy = fma(b1, k.gy, fma(b2, sf.y, fma(b3, sg.y, b4 * k.fy)));
    Real oz = fma(b1, k.gz, fma(b2, sf.z, fma(b3, sg.z, b4 * k.fz)));
    // (M g)_U += A gUj + B (d.gUj) d
    acc[3] = fma(A, sg.x, fma(b4, dx, acc[3]));
    acc[4] = fma(A, sg.y, fma(b4, dy, acc[4]));
    acc[5] = fma(A, sg.z, fma(b4, dz, acc[5]));
    if constexpr (BOTH) {
        // (M g)_U,j += A gUk + B (d.gUk) d
        jacc[3] = fma(A, k.gx, fma(b2, dx, jacc[3]));
        jacc[4] = fma(A, k.gy, fma(b2, dy, jacc[4]));
        jacc[5] = fma(A, k.gz, fma(b2, dz, jacc[5]));
    }
    if constexpr (ANG) {
        // C = gUk x Tj + gWk x Fj - gUj x Tk - gWj x Fk, one fused chain per component
        const Real cx = fma(k.gy, st.z, fma(-k.gz, st.y, fma(k.hy, sf.z, fma(-k.hz, sf.y,
                        fma(-sg.y, k.tz, fma(sg.z, k.ty, fma(-sh.y, k.fz, sh.z * k.fy)))))));
        const Real cy = fma(k.gz, st.x, fma(-k.gx, st.z, fma(k.hz, sf.x, fma(-k.hx, sf.z,
                        fma(-sg.z, k.tx, fma(sg.x, k.tz, fma(-sh.z, k.fx, sh.x * k.fz)))))));
        const Real cz = fma(k.gx, st.y, fma(-k.gy, st.x, fma(k.hx, sf.y, fma(-k.hy, sf.x,
                        fma(-sg.x, k.ty, fma(sg.y, k.tx, fma(-sh.x, k.fy, sh.y * k.fx)))))));
        // gUk.(Tj x d) + gWk.(Fj x d) - gUj.(Tk x d) - gWj.(Fk x d) = d.C (cyclic triple products)
        const Real gsum = dot3(dx, dy, dz, cx, cy, cz);
        const Real dTj = dot3(dx, dy, dz, st.x, st.y, st.z);
        const Real dhj = dot3(dx, dy, dz, sh.x, sh.y, sh.z);
        const Real dTk = dot3(dx, dy, dz, k.tx, k.ty, k.tz);
        const Real dhk = dot3(dx, dy, dz, k.hx, k.hy, k.hz);
        const Real hkTj = dot3(k.hx, k.hy, k.hz, st.x, st.y, st.z);
        const Real hjTk = dot3(sh.x, sh.y, sh.z, k.tx, k.ty, k.tz);
        S = fma(Gr, gsum, fma(Dr, hkTj + hjTk, fma(Er, fma(dhk, dTj, dhj * dTk), S)));
        // G C
        const Real e1 = E * dTj, e2 = E * dhk, e3 = E * dTk, e4 = E * dhj;
        ox = fma(Gg, cx, fma(e1, k.hx, fma(e2, st.x, fma(e3, sh.x, fma(e4, k.tx, ox)))));
        oy = fma(Gg, cy, fma(e1, k.hy, fma(e2, st.y, fma(e3, sh.y, fma(e4, k.ty, oy)))));
        oz = fma(Gg, cz, fma(e1, k.hz, fma(e2, st.z, fma(e3, sh.z, fma(e4, k.tz, oz)))));
        // (M g)_U += G (gWj x d);  (M g)_W += G (gUj x d) + D gWj + E (d.gWj) d,
        // the cross products taken with e = G d
        const Real ex = G * dx, ey = G * dy, ez = G * dz;
        acc[3] = fma(sh.y, ez, fma(-sh.z, ey, acc[3]));
        acc[4] = fma(sh.z, ex, fma(-sh.x, ez, acc[4]));
        acc[5] = fma(sh.x, ey, fma(-sh.y, ex, acc[5]));
        acc[6] = fma(sg.y, ez, fma(-sg.z, ey, fma(D, sh.x, fma(e4, dx, acc[6]))));
        acc[7] = fma(sg.z, ex, fma(-sg.x, ez, fma(D, sh.y, fma(e4, dy, acc[7]))));
        acc[8] = fma(sg.x, ey, fma(-sg.y, ex, fma(D, sh.z, fma(e4, dz, acc[8]))));
        if constexpr (BOTH) {
            // (M g)_U,j -= G (gWk x d);  (M g)_W,j += -G (gUk x d) + D gWk + E (d.gWk) d
            jacc[3] = fma(-k.hy, ez, fma(k.hz, ey, jacc[3]));
            jacc[4] = fma(-k.hz, ex, fma(k.hx, ez, jacc[4]));
            jacc[5] = fma(-k.hx, ey, fma(k.hy, ex, jacc[5]));
            jacc[6] = fma(-k.gy, ez, fma(k.gz, ey, fma(D, k.hx, fma(e2, dx, jacc[6]))));
            jacc[7] = fma(-k.gz, ex, fma(k.gx, ez, fma(D, k.hy, fma(e2, dy, jacc[7]))));
            jacc[8] = fma(-k.gx, ey, fma(k.gy, ex, fma(D, k.hz, fma(e2, dz, jacc[8]))));
        }
    }
    if constexpr (BOTH) {
        const Real tx = fma(S, dx, ox), ty = fma(S, dy, oy), tz = fma(S, dz, oz);
        acc[0] += tx;
        acc[1] += ty;
        acc[2] += tz;
        jacc[0] -= tx;
        jacc[1] -= ty;
        jacc[2] -= tz;
    } else {
        acc[0] = fma(S, dx, acc[0] + ox);
        acc[1] = fma(S, dy, acc[1] + oy);
        acc[2] = fma(S, dz, acc[2] + oz);
    }
}

template <typename Real, bool ANG>
__device__ __forceinline__ void adj_interact(const Tgt<Real, ANG> &k, const vec4_t<Real> &sp, const vec4_t<Real> &sf,
                                             const vec4_t<Real> &sg, const vec4_t<Real> &st, const vec4_t<Real> &sh,
                                             const PairConst<Real> &c, Real *acc) {
    adj_pair<Real, ANG, false>(k, sp, sf, sg, st, sh, c, acc, nullptr);
}


}  // namespace rpy

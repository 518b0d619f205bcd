// Device functions of the single-wall geometry (heights, damping and the
// image part of the Swan-Brady blocks), shared by the wall pair kernel
// (rpy_wall.hip) and the preconditioner's block assembly (rpy_precond.hip).
// The formulas are listed at the top of rpy_wall.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "rpy_device.hpp"
#include "rpy_pair.hpp"

namespace rpy {

template <typename Real>
struct WallConst {
    Real wall;    // wall height
    Real a;       // radius
    Real inv_a;   // 1/a
    Real a2;      // a^2
};

// Height above the wall raised to at least a, and the damping factor.
template <typename Real>
__device__ __forceinline__ void wall_height(Real z, const WallConst<Real> &w, Real &h, Real &d) {
    const Real hr = z - w.wall;
    h = hr > w.a ? hr : w.a;
    const Real q = hr * w.inv_a;
    d = q < Real(0) ? Real(0) : (q > Real(1) ? Real(1) : q);
}

// Image part of the pair (target at height hi, source at hj, in-plane
// separation dx, dy) acting with force f (and torque t), added to u (and w).
template <typename Real, bool ANG>
__device__ __forceinline__ void wall_image(Real dx, Real dy, Real hi, Real hj, const vec4_t<Real> &f,
                                           const vec4_t<Real> &t, Real a2, Real *u, Real *w) {
    constexpr Real c23 = Real(2.0 / 3.0), c103 = Real(10.0 / 3.0), c203 = Real(20.0 / 3.0), c43 = Real(4.0 / 3.0);
    const Real R3 = hi + hj;
    const Real rho2 = fma(dx, dx, fma(dy, dy, R3 * R3));
    const Real ri = rsq(rho2);
    const Real ri2 = ri * ri;
    const Real ex = dx * ri, ey = dy * ri, ez = R3 * ri;
    const Real Hi = hi * ri, Hj = hj * ri;
    const Real s2 = a2 * ri2, s4 = s2 * s2;
    const Real ez2 = ez * ez, HH = Hi * Hj;
    const Real f1 = fma(c23 * s4, fma(Real(-5), ez2, Real(1)), fma(-c23 * s2, fma(Real(-3), ez2, Real(1)),
                                                                     fma(Real(-2), HH, Real(-1))));
    const Real f2 = fma(-c103 * s4, fma(Real(-7), ez2, Real(1)), fma(Real(2) * s2, fma(Real(-5), ez2, Real(1)),
                                                                       fma(Real(6), HH, Real(-1))));
    const Real f3 = fma(c203 * s4 * ez, fma(Real(-7), ez2, Real(2)),
                        fma(Real(-4) * s2 * ez, fma(Real(-5), ez2, Real(1)), fma(Real(-12) * ez, HH, Real(2) * Hj)));
    const Real f4 = fma(-c203 * s4, ez, Real(2) * Hj);
    const Real f5 = fma(-c43 * s4, fma(Real(-15), ez2, Real(2)), Real(-4) * fma(s2, ez2, Hj * Hj));
    const Real eF = fma(ex, f.x, fma(ey, f.y, ez * f.z));
    const Real c1 = f1 * ri;
    const Real ce = fma(f2, eF, f3 * f.z) * ri;
    const Real cz = fma(f4, eF, f5 * f.z) * ri;
    u[0] = fma(c1, f.x, fma(ce, ex, u[0]));
    u[1] = fma(c1, f.y, fma(ce, ey, u[1]));
    u[2] = fma(c1, f.z, fma(ce, ez, u[2] + cz));
    if constexpr (ANG) {
        const Real ri3 = ri2 * ri;
        // force -> rotation: e x F + c2 (z x F) + (c3 (e.F) + c4 F_z) w, w = (e_y, -e_x, 0)
        const Real s2ez = s2 * ez;
        const Real c2 = Real(2) * (s2ez - Hj);
        const Real g = fma(fma(Real(10), s2ez, Real(-6) * Hj), eF,
                           fma(Real(2), s2, fma(Real(12) * Hj, ez, Real(-20) * s2ez * ez)) * f.z);
        w[0] = fma(ri2, fma(ey, f.z, fma(-ez, f.y, fma(-c2, f.y, g * ey))), w[0]);
        w[1] = fma(ri2, fma(ez, f.x, fma(-ex, f.z, fma(c2, f.x, -g * ex))), w[1]);
        w[2] = fma(ri2, fma(ex, f.y, -ey * f.x), w[2]);
        // torque -> velocity: -(e' x T) - c2' (z x T) + (c3' e' + c4' z)(w'.T),
        // e' = (-e_x, -e_y, e_z), w' = (-e_y, e_x, 0)
        const Real c2p = Real(2) * (s2ez - Hi);
        const Real wT = fma(-ey, t.x, ex * t.y);
        const Real c3p = fma(Real(10), s2ez, Real(-6) * Hi) * wT;
        const Real c4p = fma(Real(2), s2, fma(Real(12) * Hi, ez, Real(-20) * s2ez * ez)) * wT;
        // e' x T = (-e_y T_z - e_z T_y, e_z T_x + e_x T_z, -e_x T_y + e_y T_x)
        u[0] = fma(ri2, fma(ey, t.z, fma(ez, t.y, fma(c2p, t.y, -c3p * ex))), u[0]);
        u[1] = fma(ri2, fma(-ez, t.x, fma(-ex, t.z, fma(-c2p, t.x, -c3p * ey))), u[1]);
        u[2] = fma(ri2, fma(ex, t.y, fma(-ey, t.x, fma(c3p, ez, c4p))), u[2]);
        // torque -> rotation
        const Real eT = fma(ex, t.x, fma(ey, t.y, ez * t.z));
        const Real di = fma(Real(-6), ez2, Real(3.5));
        const Real ce2 = fma(Real(-4.5), eT, Real(3) * ez * t.z);
        const Real cz2 = fma(Real(6) * ez, eT, Real(-3) * t.z);
        w[0] = fma(ri3, fma(di, t.x, ce2 * ex), w[0]);
        w[1] = fma(ri3, fma(di, t.y, ce2 * ey), w[1]);
        w[2] = fma(ri3, fma(di, t.z, fma(ce2, ez, cz2)), w[2]);
    }
}

template <typename Real>
inline WallConst<Real> make_wall_const(double wall_height, double a) {
    WallConst<Real> wc;
    wc.wall = (Real)wall_height;
    wc.a = (Real)a;
    wc.inv_a = (Real)(1.0 / a);
    wc.a2 = (Real)(a * a);
    return wc;
}

}  // namespace rpy

// Device-side helpers shared by the HIP translation units of librpy:
// pair arithmetic of the RPY blocks, compensated summation, reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "rpy_pair.hpp"

namespace rpy {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/sqrt(x) in double: hardware estimate (relative error below 5.2e-8,
// measured over x in [1e-7, 1e7] on gfx950), then one Newton step
// y <- y + y (1 - x y^2) / 2, which squares it: below 4.2e-15 relative,
// far inside the float64 path's 1e-12 bar (a second step would reach full
// precision at the cost of three more float64 instructions per pair).
__device__ __forceinline__ double rsq(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Neumaier's compensated addition of x into (s, c).
__device__ __forceinline__ void neumaier(float &s, float &c, float x) {
    const float t = s + x;
    const float lost = (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
    c += lost;
    s = t;
}

template <typename Real>
__device__ __forceinline__ Real sel_pos(Real r2, Real v) { return r2 > Real(0) ? v : Real(0); }

// One source record (position sp, force sf, torque st) acting on target
// position (xi, yi, zi): adds its contribution to u (and w).
template <typename Real, bool ANG>
__device__ __forceinline__ void interact(Real xi, Real yi, Real zi, const vec4_t<Real> &sp,
                                         const vec4_t<Real> &sf, const vec4_t<Real> &st,
                                         const PairConst<Real> &c, Real *u, Real *w) {
    const Real dx = xi - sp.x, dy = yi - sp.y, dz = zi - sp.z;
    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    const Real ri3 = ri * ri2;
    const Real ri5 = ri3 * ri2;
    Real A = fma(c.two_a2_3, ri3, ri);
    Real B = fma(c.m_two_a2, ri5, ri3);
    Real G = ri3, D = Real(-0.5) * ri3, E = Real(1.5) * ri5;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        // overlap branch; at r = 0 (self pair) it gives the Stokes drag
        const Real rs = sel_pos(r2, ri);
        const Real r = r2 * rs;
        A = fma(c.nA1, r, c.nA0);
        B = c.nB * rs;
        if constexpr (ANG) {
            G = fma(c.nG1, r, c.nG0);
            D = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
            E = fma(c.nE_1, rs, c.nE1 * r);
        }
    }
    const Real dF = fma(dx, sf.x, fma(dy, sf.y, dz * sf.z));
    const Real s = B * dF;
    u[0] = fma(A, sf.x, fma(s, dx, u[0]));
    u[1] = fma(A, sf.y, fma(s, dy, u[1]));
    u[2] = fma(A, sf.z, fma(s, dz, u[2]));
    if constexpr (ANG) {
        // U += G (T x d)
        const Real tx = st.y * dz - st.z * dy;
        const Real ty = st.z * dx - st.x * dz;
        const Real tz = st.x * dy - st.y * dx;
        u[0] = fma(G, tx, u[0]);
        u[1] = fma(G, ty, u[1]);
        u[2] = fma(G, tz, u[2]);
        // W += G (F x d) + D T + E (d.T) d
        const Real fx = sf.y * dz - sf.z * dy;
        const Real fy = sf.z * dx - sf.x * dz;
        const Real fz = sf.x * dy - sf.y * dx;
        const Real dT = fma(dx, st.x, fma(dy, st.y, dz * st.z));
        const Real e = E * dT;
        w[0] = fma(G, fx, fma(D, st.x, fma(e, dx, w[0])));
        w[1] = fma(G, fy, fma(D, st.y, fma(e, dy, w[1])));
        w[2] = fma(G, fz, fma(D, st.z, fma(e, dz, w[2])));
    }
}

// The angular pair in a form with fewer instructions.  With G = 1/r^3 the
// far-field contribution regroups as
//   U += a1 F + g [ F' + s1 d + T x d ],   W += g [ T~ + s2 d + F x d ],
//   a1 = 1/r, g = G, s1 = (1 - 2a^2/r^2)(d.F), s2 = (3/(2 r^2))(d.T),
// where F' = (2a^2/3) F and T~ = -T/2 are per-source vectors prepared once
// per LDS tile (records: p = (x, y, z, F'x), f = (F, F'y), t = (T, F'z),
// h = (T~, 0)).  The overlap branch maps its coefficients onto the same
// form (a1 = A - (2a^2/3) G, s1 = (B/G)(d.F), s2 = (E/G)(d.T), g = G, and
// W += (D + G/2) T for the part of D T that T~ does not carry); G > 0 on
// [0, 2a), and at r = 0 it reduces to the self mobility.
template <typename Real>
__device__ __forceinline__ void interact_ang(Real xi, Real yi, Real zi, const vec4_t<Real> &p,
                                             const vec4_t<Real> &f, const vec4_t<Real> &t,
                                             const vec4_t<Real> &h, const PairConst<Real> &c, Real *u,
                                             Real *w) {
    const Real dx = xi - p.x, dy = yi - p.y, dz = zi - p.z;
    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    Real g = ri * ri2;
    Real a1 = ri;
    const Real dF = fma(dx, f.x, fma(dy, f.y, dz * f.z));
    const Real dT = fma(dx, t.x, fma(dy, t.y, dz * t.z));
    Real s1 = fma(c.m_two_a2, ri2, Real(1)) * dF;
    Real s2 = (Real(1.5) * ri2) * dT;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        // overlap branch; at r = 0 (self pair) it gives the Stokes drag
        const Real rs = sel_pos(r2, ri);
        const Real r = r2 * rs;
        const Real An = fma(c.nA1, r, c.nA0);
        const Real Bn = c.nB * rs;
        const Real Gn = fma(c.nG1, r, c.nG0);
        const Real Dn = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
        const Real En = fma(c.nE_1, rs, c.nE1 * r);
        const Real inv = Real(1) / Gn;
        a1 = fma(-c.two_a2_3, Gn, An);
        s1 = (Bn * inv) * dF;
        s2 = (En * inv) * dT;
        g = Gn;
        const Real dd = fma(Real(0.5), Gn, Dn);
        w[0] = fma(dd, t.x, w[0]);
        w[1] = fma(dd, t.y, w[1]);
        w[2] = fma(dd, t.z, w[2]);
    }
    // U += a1 F + g (F' + s1 d + T x d)
    const Real vux = fma(-t.z, dy, fma(t.y, dz, fma(s1, dx, p.w)));
    const Real vuy = fma(-t.x, dz, fma(t.z, dx, fma(s1, dy, f.w)));
    const Real vuz = fma(-t.y, dx, fma(t.x, dy, fma(s1, dz, t.w)));
    u[0] = fma(a1, f.x, fma(g, vux, u[0]));
    u[1] = fma(a1, f.y, fma(g, vuy, u[1]));
    u[2] = fma(a1, f.z, fma(g, vuz, u[2]));
    // W += g (T~ + s2 d + F x d)
    const Real vwx = fma(-f.z, dy, fma(f.y, dz, fma(s2, dx, h.x)));
    const Real vwy = fma(-f.x, dz, fma(f.z, dx, fma(s2, dy, h.y)));
    const Real vwz = fma(-f.y, dx, fma(f.x, dy, fma(s2, dz, h.z)));
    w[0] = fma(g, vwx, w[0]);
    w[1] = fma(g, vwy, w[1]);
    w[2] = fma(g, vwz, w[2]);
}

// ---------------------------------------------------------------------------
// reductions (fixed order: results do not depend on scheduling)
// ---------------------------------------------------------------------------
// Sum over a workgroup through LDS (sh has one slot per thread).
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Sum over a 64-lane wavefront by butterfly shuffles (every lane gets it).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace rpy

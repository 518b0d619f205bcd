// Device-side helpers shared by the HIP translation units of librpy:
// pair arithmetic of the RPY blocks, compensated summation, reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "rpy_internal.hpp"

namespace rpy {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/sqrt(x) in double: hardware estimate, then two Newton steps
// y <- y + y (1 - x y^2) / 2 (quadratic convergence to full precision).
__device__ __forceinline__ double rsq(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
    h = x * y;
    e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
    return y;
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

// One step of a plane rotation pair (c, s) with r = hypot(f, g), without
// divisions: 1/r from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rhyp(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
    h = x * y;
    e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
    return y;
}

// ---------------------------------------------------------------------------
// Symmetric tridiagonal square root on one workgroup (Lanczos step, Sec. 3.3)
// ---------------------------------------------------------------------------
constexpr int kMaxK = 1024;        // largest tridiagonal the eigensolver takes
constexpr int kEigThreads = 256;   // threads of the eigensolver workgroup

// One implicit QL sweep (Wilkinson-type shift, the textbook tql2 scheme)
// on the tridiagonal (d, e) in LDS, run by a single thread.  Advances the
// deflation state (l, iter); stores the sweep's plane rotations in (rc, rs)
// at indices lo..m-1 and returns lo and m in sw, or sw[0] = -1 once every
// eigenvalue has converged.
__device__ __forceinline__ void ql_sweep(double *d, double *e, int kk, int &l, int &iter, double *rc, double *rs,
                                         int *sw) {
    int m = l;
    while (l < kk) {
        for (m = l; m < kk - 1; ++m) {
            const double dd = fabs(d[m]) + fabs(d[m + 1]);
            if (fabs(e[m]) <= 2.220446049250313e-16 * dd) break;
        }
        if (m != l && iter < 60) break;
        // eigenvalue l converged (or gave up after 60 sweeps)
        ++l;
        iter = 0;
    }
    if (l >= kk) {
        sw[0] = -1;
        return;
    }
    ++iter;
    double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
    double r = sqrt(fma(g, g, 1.0));
    g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
    double sn = 1.0, cs = 1.0, p = 0.0;
    int i;
    bool underflow = false;
    double ei = e[m - 1], di = d[m - 1], dip1 = d[m];
    for (i = m - 1; i >= l; --i) {
        // prefetch the next step's (unmodified) entries
        const double e_nx = i > l ? e[i - 1] : 0.0;
        const double d_nx = i > l ? d[i - 1] : 0.0;
        const double f = sn * ei;
        const double b = cs * ei;
        const double r2 = fma(f, f, g * g);
        if (r2 == 0.0) {
            d[i + 1] = dip1 - p;
            e[m] = 0.0;
            underflow = true;
            break;
        }
        const double ri = rhyp(r2);
        e[i + 1] = r2 * ri;
        sn = f * ri;
        cs = g * ri;
        g = dip1 - p;
        r = (di - g) * sn + 2.0 * cs * b;
        p = sn * r;
        d[i + 1] = g + p;
        g = cs * r - b;
        rc[i] = cs;
        rs[i] = sn;
        dip1 = di;
        di = d_nx;
        ei = e_nx;
    }
    const int lo = underflow ? i + 1 : l;
    if (!underflow) {
        d[l] = dip1 - p;
        e[l] = g;
        e[m] = 0.0;
    }
    sw[0] = lo;
    sw[1] = m;
}

// Eigen-decomposition of the kk x kk symmetric tridiagonal T (diagonal
// alpha[0..kk), off-diagonal beta[0..kk-1)) by implicit QL, then
// s_out = Q diag(sqrt(max(lambda, 0))) Q^T e_1.  Q (kk x kk, column-major,
// column j = eigenvector j) lives in global memory.  The scalar QL
// recurrences are inherently sequential; they run on thread 0 and are
// pipelined against the eigenvector updates: while thread 0 computes sweep
// p+1 into one LDS rotation buffer, waves 1..3 apply sweep p from the other
// buffer to the rows of Q, each thread carrying the running column of its
// row in a register so the loads of a sweep do not wait on its stores.
// When spd_flag is given it receives 1 if an eigenvalue is below
// -1e-10 lambda_max (not positive definite), else 0.  Must be called by all
// threads of a workgroup of kEigThreads threads.
__device__ __noinline__ void tridiag_sqrt_block(const double *__restrict__ alpha, const double *__restrict__ beta,
                                                int kk, double *__restrict__ s_out, double *__restrict__ Q,
                                                double *spd_flag) {
    __shared__ double d[kMaxK], e[kMaxK];
    __shared__ double rc[2][kMaxK], rs[2][kMaxK];
    __shared__ int sw[2][2];
    const int tid = threadIdx.x;
    for (int i = tid; i < kk; i += blockDim.x) {
        d[i] = alpha[i];
        e[i] = (i + 1 < kk) ? beta[i] : 0.0;
    }
    for (int64_t idx = tid; idx < (int64_t)kk * kk; idx += blockDim.x)
        Q[idx] = (idx / kk == idx % kk) ? 1.0 : 0.0;
    __syncthreads();

    int l = 0, iter = 0;                      // QL state, meaningful on thread 0 only
    if (tid == 0) ql_sweep(d, e, kk, l, iter, rc[0], rs[0], sw[0]);
    __syncthreads();
    for (int p = 0;; p ^= 1) {
        if (sw[p][0] < 0) break;               // uniform: read after the barrier
        if (tid == 0) {
            ql_sweep(d, e, kk, l, iter, rc[p ^ 1], rs[p ^ 1], sw[p ^ 1]);
        } else if (tid >= 64) {
            const int lo = sw[p][0], m = sw[p][1];
            const double *c = rc[p], *sn = rs[p];
            for (int row = tid - 64; row < kk; row += (int)blockDim.x - 64) {
                double carry = Q[(size_t)m * kk + row];
                int i = m - 1;
                for (; i - 3 >= lo; i -= 4) {
                    const double q0 = Q[(size_t)i * kk + row];
                    const double q1 = Q[(size_t)(i - 1) * kk + row];
                    const double q2 = Q[(size_t)(i - 2) * kk + row];
                    const double q3 = Q[(size_t)(i - 3) * kk + row];
                    double nv;
                    nv = fma(sn[i], q0, c[i] * carry);
                    carry = fma(c[i], q0, -sn[i] * carry);
                    Q[(size_t)(i + 1) * kk + row] = nv;
                    nv = fma(sn[i - 1], q1, c[i - 1] * carry);
                    carry = fma(c[i - 1], q1, -sn[i - 1] * carry);
                    Q[(size_t)i * kk + row] = nv;
                    nv = fma(sn[i - 2], q2, c[i - 2] * carry);
                    carry = fma(c[i - 2], q2, -sn[i - 2] * carry);
                    Q[(size_t)(i - 1) * kk + row] = nv;
                    nv = fma(sn[i - 3], q3, c[i - 3] * carry);
                    carry = fma(c[i - 3], q3, -sn[i - 3] * carry);
                    Q[(size_t)(i - 2) * kk + row] = nv;
                }
                for (; i >= lo; --i) {
                    const double q0 = Q[(size_t)i * kk + row];
                    Q[(size_t)(i + 1) * kk + row] = fma(sn[i], q0, c[i] * carry);
                    carry = fma(c[i], q0, -sn[i] * carry);
                }
                Q[(size_t)lo * kk + row] = carry;
            }
        }
        __syncthreads();
    }

    // spectrum check and the square root applied to e_1
    if (spd_flag && tid == 0) {
        double lmax = -1e308, lmin = 1e308;
        for (int j = 0; j < kk; ++j) {
            lmax = fmax(lmax, d[j]);
            lmin = fmin(lmin, d[j]);
        }
        *spd_flag = (lmin < -1e-10 * fmax(lmax, 0.0)) ? 1.0 : 0.0;
    }
    // u_j = sqrt(max(lambda_j, 0)) * Q[0][j]  (row 0 of column j)
    double *u = rc[0];
    for (int j = tid; j < kk; j += blockDim.x) u[j] = sqrt(fmax(d[j], 0.0)) * Q[(size_t)j * kk];
    __syncthreads();
    for (int row = tid; row < kk; row += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < kk; ++j) acc = fma(Q[(size_t)j * kk + row], u[j], acc);
        s_out[row] = acc;
    }
}

}  // namespace rpy

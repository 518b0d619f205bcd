// Device-side pieces of the Lanczos square root (Sec. 3.3) shared by the
// single-system and batched solvers: the workgroup eigensolver of the
// tridiagonal T_k and the quadrature estimate of T_k^{1/2} e_1.
#pragma once

#include <hip/hip_runtime.h>

#include "rpy_device.hpp"

namespace rpy {

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


// ---------------------------------------------------------------------------
// quadrature estimate of the Lanczos square-root iterate
// ---------------------------------------------------------------------------
// Estimate of s = T^{1/2} e_1 for the leading kk x kk block of the Lanczos
// tridiagonal T_k = (alpha, beta), kk in {k-1, k}, without an
// eigendecomposition, used to decide when the exact increment test is worth
// running.  With x^{-1/2} = (1/pi) int exp(u/2) / (x + exp(u)) du over the
// real line (the substitution t^2 = e^u in the standard integral
// (2/pi) int_0^inf dt / (x + t^2)), the trapezoid rule with step h gives
//   T^{1/2} e_1 = T T^{-1/2} e_1 ~ T sum_l w_l (T + c_l I)^{-1} e_1,
//   c_l = exp(u_l), w_l = (h/pi) exp(u_l/2).
// The integrand is analytic in the strip |Im u| < pi, so the rule's error
// falls like exp(-2 pi^2 / h) (about 1e-17 at h = 0.5).  The nodes span
// [log(1e-10 g) - 20, log(g) + 20] for the Gershgorin bound g of T_k, the
// same nodes for kk = k-1 and kk = k.  Beyond the last node the integrand
// is e^{-u/2} (1 + O(x e^{-u})), below the first e^{u/2} / x (1 + O(e^u / x)),
// so the trapezoid sums over the missing nodes are geometric series:
// C_up e_1 and C_lo T^{-1} e_1 with C = (h/pi) e^{-(m + h)/2} / (1 - e^{-h/2})
// at distance m from the node range's edge, i.e. C_up T e_1 + C_lo e_1 in
// s; both are added back, and the terms left out are below exp(-30)
// relative for eigenvalues in [1e-10 g, g].
//
// Thread l < kMonNodes solves (T + c_l I) y = e_1 by elimination from the
// bottom row up (pivots g_i, ratios r_i = -beta_i / g_{i+1}; y_0 = 1 / g_0,
// y_{i+1} = r_i y_i), which is stable for these SPD systems.  Meanwhile one
// lane of the extra wavefront factors T - 1e-10 g I = L D L^T: a
// non-positive pivot means T has an eigenvalue below the quadrature's range
// (or a negative one) and the estimate is returned as NaN, which sends the
// caller to the exact test.  Called by all kMonThreads threads of a
// workgroup; `scratch` holds kk * kMonNodes doubles.
constexpr int kMonNodes = 128;
constexpr int kMonThreads = kMonNodes + 64;
constexpr int kMonChunk = 16;  // scratch rows fetched together in the forward pass
constexpr int kMonRows = 8;    // rows of the node sums per wavefront at a time

// 1/x from the hardware estimate and two Newton steps y <- y + y (1 - x y)
// (within an ulp or two; the serial recurrences below run on its latency).
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

__device__ __noinline__ void monitor_block(const double *__restrict__ alpha, const double *__restrict__ beta, int k,
                                           int kk, double *__restrict__ scratch, double *__restrict__ est) {
    constexpr int kWaves = kMonThreads / 64;
    __shared__ double a[kMaxK], b[kMaxK], q[kMaxK];
    __shared__ double wmax[kWaves];
    __shared__ int indefinite;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // T_k into LDS (the kk-block uses the first kk rows, b_i for i < kk - 1)
    // and its Gershgorin bound
    double g = 0.0;
    for (int i = tid; i < k; i += blockDim.x) {
        const double ai = alpha[i], bl = i > 0 ? beta[i - 1] : 0.0, br = i + 1 < k ? beta[i] : 0.0;
        a[i] = ai;
        b[i] = br;
        g = fmax(g, fabs(ai) + fabs(bl) + fabs(br));
    }
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o));
    if (lane == 0) wmax[wv] = g;
    if (tid == 0) indefinite = 0;
    __syncthreads();
    double bound = wmax[0];
    for (int w = 1; w < kWaves; ++w) bound = fmax(bound, wmax[w]);
    if (!(bound > 0.0)) bound = 1.0;
    if (tid >= kMonNodes) {
        if (tid == kMonNodes) {
            // only the pivots' signs matter: reciprocal instead of division
            const double shift = 1e-10 * bound;
            double piv = a[0] - shift;
            bool pd = piv > 0.0;
            double bn = kk > 1 ? b[0] : 0.0, an = kk > 1 ? a[1] : 0.0;
            for (int i = 1; i < kk && pd; ++i) {
                const double bi = bn, ai = an;
                if (i + 1 < kk) {   // next row's operands, loaded ahead of the chain
                    bn = b[i];
                    an = a[i + 1];
                }
                piv = (ai - shift) - bi * (bi * recip(piv));
                pd = piv > 0.0;
            }
            if (!pd) indefinite = 1;
        }
    } else {
        const int l = tid;
        const double u_hi = log(bound) + 20.0, u_lo = log(bound) + log(1e-10) - 20.0;
        const double h = (u_hi - u_lo) / (double)(kMonNodes - 1);
        const double ul = u_lo + h * l;
        const double c = exp(ul), wl = h / M_PI * exp(0.5 * ul);
        double gp = a[kk - 1] + c;
        double bn = kk > 1 ? b[kk - 2] : 0.0, an = kk > 1 ? a[kk - 2] : 0.0;
        for (int i = kk - 2; i >= 0; --i) {
            const double bi = bn, ai = an;
            if (i > 0) {   // next row's operands, loaded ahead of the chain
                bn = b[i - 1];
                an = a[i - 1];
            }
            const double r = -bi * recip(gp);
            scratch[(size_t)i * kMonNodes + l] = r;
            gp = fma(bi, r, ai + c);
        }
        double y = recip(gp);
        // w_l y_i replaces r_i; the ratios of kMonChunk rows are fetched
        // together so that the product chain waits once per chunk
        int i = 0;
        for (; i + kMonChunk < kk; i += kMonChunk) {
            double rr[kMonChunk];
#pragma unroll
            for (int u = 0; u < kMonChunk; ++u) rr[u] = scratch[(size_t)(i + u) * kMonNodes + l];
#pragma unroll
            for (int u = 0; u < kMonChunk; ++u) {
                scratch[(size_t)(i + u) * kMonNodes + l] = wl * y;
                y *= rr[u];
            }
        }
        for (; i + 1 < kk; ++i) {
            const double r = scratch[(size_t)i * kMonNodes + l];
            scratch[(size_t)i * kMonNodes + l] = wl * y;
            y *= r;
        }
        scratch[(size_t)(kk - 1) * kMonNodes + l] = wl * y;
    }
    __syncthreads();
    // q_i = sum_l w_l y_{l,i}: each wavefront takes kMonRows rows at a time,
    // all their loads issued together (coalesced along l), then one
    // butterfly per row
    static_assert(kMonNodes == 128, "two nodes per lane");
    for (int i0 = kMonRows * wv; i0 < kk; i0 += kMonRows * kWaves) {
        double sr[kMonRows];
#pragma unroll
        for (int u = 0; u < kMonRows; ++u) {
            const double *row = scratch + (size_t)(i0 + u) * kMonNodes;
            sr[u] = i0 + u < kk ? row[lane] + row[lane + 64] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kMonRows; ++u) sr[u] = wave_sum(sr[u]);
        if (lane < kMonRows && i0 + lane < kk) {
            double mine = sr[0];
#pragma unroll
            for (int u = 1; u < kMonRows; ++u) mine = lane == u ? sr[u] : mine;
            q[i0 + lane] = mine;
        }
    }
    __syncthreads();
    // est = T q + C_up T e_1 + C_lo e_1 (tails of the trapezoid sum)
    const double u_hi = log(bound) + 20.0, u_lo = log(bound) + log(1e-10) - 20.0;
    const double h = (u_hi - u_lo) / (double)(kMonNodes - 1);
    const double geo = h / M_PI / (1.0 - exp(-0.5 * h));
    const double c_up = geo * exp(-0.5 * (u_hi + h)), c_lo = geo * exp(0.5 * (u_lo - h));
    const double poison = indefinite ? NAN : 0.0;
    for (int i = tid; i < kk; i += blockDim.x) {
        double v = a[i] * q[i];
        if (i > 0) v = fma(b[i - 1], q[i - 1], v);
        if (i + 1 < kk) v = fma(b[i], q[i + 1], v);
        if (i == 0) v += fma(c_up, a[0], c_lo);
        if (i == 1) v = fma(c_up, b[0], v);
        est[i] = v + poison;
    }
    __syncthreads();
}

}  // namespace rpy

// M^{1/2} W by Lanczos on the device (Sec. 3.3: Krylov square root of Ando,
// Chow, Saad & Skolnick for solvers that only apply M).
//
// Every vector operation is float64 and runs on the device; the products
// M v_k use the solver's pair precision (float32 pairs for float32
// solvers).  Per iteration k (v_k = column k-1 of the basis V):
//   w = M v_k;  w -= beta_{k-1} v_{k-1};  alpha_k = v_k . w;  w -= alpha_k v_k
//   classical Gram-Schmidt against V_k (w -= V_k (V_k^T w)), a second pass
//     when the first removed more than half of |w|^2
//   beta_k = |w|
//   T_k = tridiag(beta, alpha, beta) = Q diag(lambda) Q^T on one workgroup
//     (implicit-shift QL), s_k = Q diag(sqrt(lambda)) Q^T e_1, and the
//     relative increment |s_k - [s_{k-1}; 0]| / |s_k|, which equals
//     |y_k - y_{k-1}| / |y_k| for y_k = beta_0 V_k s_k because V_k is
//     orthonormal;
//   v_{k+1} = w / beta_k.
// The host reads a small status block after each iteration, written by the
// device to pinned host memory, to decide whether to stop (first k >= 2
// with increment < tol; a clearly negative Ritz value; beta_k ~ 0 meaning
// the Krylov space is invariant); with one recurrence the next basis vector
// and, while far from tol, its product are already enqueued meanwhile.  s_{k-1}
// and s_k come from a quadrature estimate of T^{1/2} e_1 that is exact to
// rounding for safely positive definite T_k; the eigensolver runs only where
// that estimate cannot decide.  The final y = prefactor * beta_0 V_k s_k is
// formed on the device and written in the caller's dtype.
//
// Reductions are two-stage with a fixed block count and fixed order, so the
// result does not depend on scheduling.  A reduction's workgroup sums are
// added, in a fixed order, by the launch that needs the result (every one of
// its workgroups forms the same value), so an iteration's vector work takes
// eight launches (three of them return at once when the second
// Gram-Schmidt pass is not needed), with no grid-wide synchronisation.
#include "rpy_device.hpp"
#include "rpy_krylov.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace rpy {
namespace {

constexpr int kRedBlocks = 256;    // blocks of the first reduction stage
constexpr int kRedThreads = 256;

// status block (double): beta0, relative increment, flags, running
// max(|alpha|, beta), first breakdown iteration (0 = none), estimated
// relative increment (monitor), |w|^2 before Gram-Schmidt, skip flag of the
// second pass, bytes of skipped passes
enum { ST_BETA0 = 0, ST_INCR = 1, ST_FLAGS = 2, ST_TSCALE = 3, ST_BREAK = 4, ST_EST = 5, ST_NW = 6, ST_SKIP = 7,
       ST_SKIPPED = 8, ST_SIZE = 10 };
enum { FLAG_NOT_SPD = 1, FLAG_NONFINITE = 2 };
// Workgroup sums of one iteration's reductions, per recurrence: v_k . w,
// |w|^2 after the recurrence, |w|^2 at the end of the iteration.
constexpr int kMaxUpdateBlocks = 2048;   // grid of the Gram-Schmidt update
constexpr int kDotBlocks = 1024;         // grid of the recurrence's dot products (16 wavefronts per CU)
enum { PS_ALPHA = 0, PS_NW = kDotBlocks, PS_BETA = 2 * kDotBlocks, PS_SIZE = 2 * kDotBlocks + kMaxUpdateBlocks };

// Sum over the threads of a workgroup of whole wavefronts: each wavefront's
// butterfly, then the wavefronts' sums in order (every thread gets it).
__device__ __forceinline__ double group_sum(double v, double *sh) {
    v = wave_sum(v);
    const int nw = (int)blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
    for (int q = 1; q < nw; ++q) t += sh[q];
    return t;
}

// Arrival of a workgroup at the end of its share of a one-launch reduction
// over a few workgroups: its results are stored, made visible to the other
// workgroups, and counted; true in the workgroup that arrives last (counter
// reset), after which its loads see every other workgroup's stores.  Called
// by all threads.
__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned total) {
    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        last = atomicAdd(counter, 1u) == total - 1;
        if (last) *counter = 0u;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    return true;
}

// Breakdown bookkeeping after beta_k: running max(|alpha|, beta) and the
// first k with beta_k <= 1e-14 of it.
__device__ __forceinline__ void finish_iter(const double *__restrict__ alpha, const double *__restrict__ beta, int k,
                                            double *__restrict__ status) {
    const double a = fabs(alpha[k - 1]), b = beta[k - 1];
    const double sc = fmax(status[ST_TSCALE], fmax(a, b));
    status[ST_TSCALE] = sc;
    if (status[ST_BREAK] == 0.0 && !(b > 1e-14 * sc)) status[ST_BREAK] = (double)k;
}

// w -= c x (no update when x is NULL), and this thread's share of y . w
// (w . w when y is NULL): its strided entries in index order, four loads
// per operand issued together.
__device__ __forceinline__ double axpy_dot_thread(double *w, const double *__restrict__ x, double c,
                                                  const double *y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        double wv[4], xv[4], yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            wv[u] = w[i + u * stride];
            xv[u] = x ? x[i + u * stride] : 0.0;
            yv[u] = y ? y[i + u * stride] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (x) {
                wv[u] = fma(c, xv[u], wv[u]);
                w[i + u * stride] = wv[u];
            }
            acc = fma(y ? yv[u] : wv[u], wv[u], acc);
        }
    }
    for (; i < n; i += stride) {
        double wv = w[i];
        if (x) {
            wv = fma(c, x[i], wv);
            w[i] = wv;
        }
        acc = fma(y ? y[i] : wv, wv, acc);
    }
    return acc;
}

// Recurrence, first half: w -= beta_{k-1} v_{k-1} (k > 1; x = v_{k-1},
// coef = &beta_{k-1}, both NULL at k = 1), and the workgroup sums of
// v_k . w into pa.
__global__ void __launch_bounds__(kRedThreads)
recur_beta(double *w, const double *__restrict__ x, const double *coef, const double *__restrict__ vk, int64_t n,
           double *__restrict__ pa) {
    __shared__ double sh[kRedThreads];
    const double acc = axpy_dot_thread(w, x, x ? -(*coef) : 0.0, vk, n);
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) pa[blockIdx.x] = r;
}

// The kDotBlocks workgroup sums of a recurrence dot product, added in the
// same order by every workgroup of a launch of kRedThreads threads.
__device__ __forceinline__ double dot_from_sums(const double *__restrict__ p, double *sh) {
    static_assert(kDotBlocks % kRedThreads == 0, "whole sums per thread");
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < kDotBlocks / kRedThreads; ++m) t += p[threadIdx.x + kRedThreads * m];
    return block_sum(t, sh);
}

// Recurrence, second half: alpha_k = the sum of pa (dot_from_sums;
// workgroup 0 stores it), then w -= alpha_k v_k and the workgroup sums of
// |w|^2 into pn.
__global__ void __launch_bounds__(kRedThreads)
recur_alpha(double *w, const double *__restrict__ vk, const double *__restrict__ pa, double *alpha_out, int64_t n,
            double *__restrict__ pn) {
    __shared__ double sh[kRedThreads];
    const double a = dot_from_sums(pa, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = a;
    const double acc = axpy_dot_thread(w, vk, -a, nullptr, n);
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) pn[blockIdx.x] = r;
}

// out = sum(partial) (or its square root); optional second copy
__global__ void reduce_scalar(const double *__restrict__ partial, int nb, double *out, int take_sqrt) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partial[i];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = take_sqrt ? sqrt(r) : r;
}

// v1 = W / beta0, W in the caller's dtype
template <typename Tin>
__global__ void init_basis(double *__restrict__ v, const Tin *__restrict__ w, const double *beta0, int64_t n) {
    const double inv = 1.0 / (*beta0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (double)w[i] * inv;
}

template <typename Tin>
__global__ void sumsq_partial(const Tin *__restrict__ w, int64_t n, double *__restrict__ partial) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)w[i];
        acc = fma(x, x, acc);
    }
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// partial[b * k + j] = sum over row chunk b of V[j][i] w[i], j < k.
// Grid (row chunks of kGtRows * 256 rows) x (groups of kGtCols columns):
// each thread issues all kGtRows * kGtCols coalesced loads of its tile (and
// its kGtRows entries of w) before the first multiply-add, which keeps
// enough loads in flight per wavefront to stream V near the HBM rate; each
// column's sums are then added by a butterfly over the wavefront and the
// four wavefronts' values in order (deterministic).  The second pass
// (skip != NULL) does nothing when *skip is set (see gemv_n_pass).
constexpr int kGtRows = 4;
constexpr int kGtCols = 8;
constexpr int kGtChunk = kGtRows * kRedThreads;   // rows per chunk
__global__ void __launch_bounds__(kRedThreads)
gemv_t_partial(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ w, int64_t n,
               double *__restrict__ partial, const double *skip) {
    if (skip && *skip != 0.0) return;
    __shared__ double sh[kRedThreads / 64][kGtCols];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kGtChunk + tid;
    const int j0 = (int)blockIdx.y * kGtCols;
    double x[kGtCols][kGtRows], wr[kGtRows];
    if ((int64_t)blockIdx.x * kGtChunk + kGtChunk <= n && j0 + kGtCols <= k) {
#pragma unroll
        for (int q = 0; q < kGtRows; ++q) wr[q] = w[base + (int64_t)q * kRedThreads];
#pragma unroll
        for (int c = 0; c < kGtCols; ++c)
#pragma unroll
            for (int q = 0; q < kGtRows; ++q) x[c][q] = V[(size_t)(j0 + c) * ld + base + (int64_t)q * kRedThreads];
    } else {
#pragma unroll
        for (int q = 0; q < kGtRows; ++q) {
            const int64_t i = base + (int64_t)q * kRedThreads;
            wr[q] = i < n ? w[i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kGtCols; ++c)
#pragma unroll
            for (int q = 0; q < kGtRows; ++q) {
                const int64_t i = base + (int64_t)q * kRedThreads;
                x[c][q] = (j0 + c < k && i < n) ? V[(size_t)(j0 + c) * ld + i] : 0.0;
            }
    }
    double acc[kGtCols];
#pragma unroll
    for (int c = 0; c < kGtCols; ++c) {
        acc[c] = 0.0;
#pragma unroll
        for (int q = 0; q < kGtRows; ++q) acc[c] = fma(x[c][q], wr[q], acc[c]);
        acc[c] = wave_sum(acc[c]);
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < kGtCols; ++c) sh[wv][c] = acc[c];
    }
    __syncthreads();
    if (tid < kGtCols && j0 + tid < k) {
        double v = sh[0][tid];
#pragma unroll
        for (int q = 1; q < kRedThreads / 64; ++q) v += sh[q][tid];
        partial[(size_t)blockIdx.x * k + j0 + tid] = v;
    }
}

// h[j] = sum_b partial[b * k + j]   (one block per j)
__global__ void gemv_t_final(const double *__restrict__ partial, int nb, int k, double *__restrict__ h,
                             const double *skip) {
    __shared__ double sh[kRedThreads];
    if (skip && *skip != 0.0) return;
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[(size_t)b * k + j];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) h[j] = r;
}

// w[i] -= sum_j V[j][i] h[j] for Gram-Schmidt pass `pass` (0 or 1).
// Pass 0 first decides whether pass 1 is needed, in every workgroup alike
// from h and the workgroup sums pn of |w|^2 (workgroup 0 records the
// decision): the part the pass removes has squared norm |h|^2 (V
// orthonormal), so pass 1 is needed only when |h|^2 > |w|^2 / 2, i.e. when
// pass 0 cuts |w| below 1/sqrt(2) of itself (Kahan and Parlett's "twice is
// enough" test, as in Daniel, Gragg, Kaufman and Stewart's
// reorthogonalisation); otherwise w is already orthogonal to V to working
// precision, the skip flag is set and the skipped pass's bytes are counted
// (NaN never skips).  Pass 1 does nothing when skipped.  The pass that ends
// the iteration stores its workgroup sums of the new |w|^2 to pb.
__global__ void __launch_bounds__(256)
gemv_n_pass(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ h, double *__restrict__ w,
            int64_t n, int pass, const double *__restrict__ pn, double *status, double pass_bytes,
            double *__restrict__ pb) {
    static_assert(kRedThreads == 256, "launched with 256 threads");
    __shared__ double hs[kMaxK];
    __shared__ double red[4];
    __shared__ double sh[kRedThreads];
    if (pass == 1 && status[ST_SKIP] != 0.0) return;
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
    bool last_pass = true;
    if (pass == 0) {
        double a = 0.0;
        for (int j = threadIdx.x; j < k; j += blockDim.x) a = fma(hs[j], hs[j], a);
        const double hh = group_sum(a, red);
        const double nw = dot_from_sums(pn, sh);
        last_pass = hh <= 0.5 * nw;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            status[ST_NW] = nw;
            status[ST_SKIP] = last_pass ? 1.0 : 0.0;
            if (last_pass) status[ST_SKIPPED] += pass_bytes;
        }
    }
    double sq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(V[(size_t)j * ld + i], hs[j], acc);
        const double wn = w[i] - acc;
        w[i] = wn;
        sq = fma(wn, wn, sq);
    }
    if (!last_pass) return;
    const double r = group_sum(sq, red);
    if (threadIdx.x == 0) pb[blockIdx.x] = r;
}

// beta_k = sqrt of the nb workgroup sums pb, added by one wavefront in a
// fixed order, then the breakdown bookkeeping.  Called by wavefront 0 of a
// workgroup.
__device__ __forceinline__ void beta_from_sums(const double *__restrict__ pb, int nb, const double *alpha,
                                               double *beta, int k, double *status) {
    static_assert(kMaxUpdateBlocks <= 32 * 64, "at most 32 sums per lane");
    const int lane = threadIdx.x & 63;
    double v[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) v[m] = lane + 64 * m < nb ? pb[lane + 64 * m] : 0.0;   // loads issued together
    double t = 0.0;
#pragma unroll
    for (int m = 0; m < 32; ++m) t += v[m];
    t = wave_sum(t);
    if (lane == 0) {
        beta[k - 1] = sqrt(t);
        finish_iter(alpha, beta, k, status);
    }
}

// beta_k for an iteration without the quadrature monitor (one wavefront).
__global__ void __launch_bounds__(64)
beta_kernel(const double *__restrict__ pb, int nb, const double *alpha, double *beta, int k, double *status) {
    beta_from_sums(pb, nb, alpha, beta, k, status);
}

// out = scale * sum_j V[j][i] s[j] (or out + that, with `accumulate`),
// written as n_lin linear entries to lin and the rest to ang (caller's
// dtype; the sum is formed in float64 and rounded once).
template <typename Tout>
__global__ void combine_out(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ s,
                            const double *__restrict__ status, double prefactor, int64_t n, int64_t n_lin,
                            int accumulate, Tout *__restrict__ lin, Tout *__restrict__ ang) {
    __shared__ double hs[kMaxK];
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = s[j];
    __syncthreads();
    const double scale = prefactor * status[ST_BETA0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(V[(size_t)j * ld + i], hs[j], acc);
        Tout *dst = i < n_lin ? lin + i : ang + (i - n_lin);
        const double base = accumulate ? (double)*dst : 0.0;
        *dst = (Tout)(base + scale * acc);
    }
}

// s_{k-1} (workgroup 0) and s_k (workgroup 1) of the tridiagonal T_k in one
// launch; workgroup 1 also records whether T_k is positive definite.
__global__ void __launch_bounds__(kEigThreads)
tridiag_sqrt_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int k,
                    double *__restrict__ s_out0, double *__restrict__ s_out1, double *__restrict__ Qbuf,
                    int64_t qstride, double *__restrict__ status) {
    const int kk = k - 1 + (int)blockIdx.x;
    if (kk <= 0) return;
    tridiag_sqrt_block(alpha, beta, kk, blockIdx.x == 0 ? s_out0 : s_out1, Qbuf + (size_t)blockIdx.x * qstride,
                       blockIdx.x == 1 ? status + ST_FLAGS : nullptr);
}

// Quadrature estimates of s_{k-1} (workgroup 0) and s_k (workgroup 1)
// (see monitor_block; T_k does not involve beta_k, which wavefront 0 of
// workgroup 0 forms first from the sums pb, as beta_kernel does); the
// workgroup that finishes second then writes the estimated relative
// increment |s_k - [s_{k-1}; 0]| / |s_k| to status[ST_EST] and copies the
// status block to `mirror` (pinned host memory, read by the host after the
// stream synchronises: no copy launch).  Up to
// k = kMonLdsRows the node scratch is the launch's dynamic LDS (k rows of
// kMonNodes doubles per workgroup), beyond it `scratch` in device memory.
constexpr int kMonLdsRows = 128;
__global__ void __launch_bounds__(kMonThreads)
lanczos_monitor_kernel(const double *__restrict__ alpha, double *__restrict__ beta, int k,
                       double *__restrict__ scratch, int64_t sstride, double *__restrict__ est0,
                       double *__restrict__ est1, unsigned *__restrict__ cnt, double *__restrict__ status,
                       const double *__restrict__ pb, int nb, double *__restrict__ mirror) {
    if (blockIdx.x == 0 && threadIdx.x < 64) beta_from_sums(pb, nb, alpha, beta, k, status);
    extern __shared__ double mon_lds[];
    const int kk = k - 1 + (int)blockIdx.x;
    double *scr = k <= kMonLdsRows ? mon_lds : scratch + (size_t)blockIdx.x * sstride;
    if (kk > 0) monitor_block(alpha, beta, k, kk, scr, blockIdx.x == 0 ? est0 : est1);
    if (!arrive_last(cnt, gridDim.x)) return;
    __shared__ double red[kMonThreads / 64];
    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double prev = (i < k - 1) ? est0[i] : 0.0;
        const double dlt = est1[i] - prev;
        num = fma(dlt, dlt, num);
        den = fma(est1[i], est1[i], den);
    }
    num = group_sum(num, red);
    den = group_sum(den, red);
    if (threadIdx.x == 0) status[ST_EST] = (k >= 2 && den > 0.0) ? sqrt(num / den) : INFINITY;
    __syncthreads();
    if (threadIdx.x < ST_SIZE) mirror[threadIdx.x] = status[threadIdx.x];
}

// status[ST_INCR] = |s1 - [s0; 0]| / |s1| for s0 of length k-1, s1 of length k.
__global__ void increment_kernel(const double *__restrict__ s0, const double *__restrict__ s1, int k,
                                 double *__restrict__ status, int slot) {
    __shared__ double red[kRedThreads];
    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double prev = (i < k - 1) ? s0[i] : 0.0;
        const double dlt = s1[i] - prev;
        num = fma(dlt, dlt, num);
        den = fma(s1[i], s1[i], den);
    }
    num = block_sum(num, red);
    den = block_sum(den, red);
    if (threadIdx.x == 0) status[slot] = (k >= 2 && den > 0.0) ? sqrt(num / den) : INFINITY;
}

// After beta_k: track max(|alpha|, beta) and record the first breakdown
// beta_k <= 1e-14 max(|alpha|, beta) (the Krylov space is invariant).
// v_{k+1} = w / beta_k, or zeros once a breakdown has been recorded.
__global__ void next_basis_kernel(double *__restrict__ dst, const double *__restrict__ src,
                                  const double *__restrict__ beta, const double *__restrict__ status, int64_t n) {
    const bool broken = status[ST_BREAK] != 0.0;
    const double inv = broken ? 0.0 : 1.0 / (*beta);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = broken ? 0.0 : src[i] * inv;
}

// next_basis_kernel for one recurrence whose next product is a single-vector
// one: thread (part, p) also writes particle p's three entries of that part,
// rounded to Real, as the staged vec4 record of the product (linear part to
// f4, angular part to t4 when n = 6 np), so the product needs no staging
// launch.
template <typename Real>
__global__ void next_basis_staged(double *__restrict__ dst, const double *__restrict__ src,
                                  const double *__restrict__ beta, const double *__restrict__ status, int np,
                                  int64_t n, vec4_t<Real> *__restrict__ f4, vec4_t<Real> *__restrict__ t4) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n / 3) return;
    const int part = (int)(gid / np), p = (int)(gid - (int64_t)part * np);
    const bool broken = status[ST_BREAK] != 0.0;
    const double inv = broken ? 0.0 : 1.0 / (*beta);
    const size_t i = (size_t)part * 3 * np + 3 * (size_t)p;
    double v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = broken ? 0.0 : src[i + c] * inv;
        dst[i + c] = v[c];
    }
    vec4_t<Real> r;
    r.x = (Real)v[0];
    r.y = (Real)v[1];
    r.z = (Real)v[2];
    r.w = Real(0);
    (part == 0 ? f4 : t4)[p] = r;
}

// Device state of one recurrence inside the shared workspace, and the
// host's view of its progress.
struct LzRec {
    double *V = nullptr;   // basis, cap + 1 columns of ld doubles
    double *status = nullptr, *alpha = nullptr, *beta = nullptr, *h = nullptr;
    double *s = nullptr, *s_prev = nullptr, *est0 = nullptr, *est1 = nullptr;
    int kf = 0;
    double incr = INFINITY;
    const double *s_final = nullptr;   // exact s_k unless the estimate decided
    double *ps = nullptr;              // workgroup sums of the iteration's reductions (PS_*)
    bool done = false, converged = false, not_spd = false, exact = false;
};

int grid_for(int64_t n) { return (int)std::min<int64_t>(kMaxUpdateBlocks, std::max<int64_t>(1, (n + 255) / 256)); }

// w (slots of ld doubles, linear then angular rows) = M v for the basis
// column `col` of every listed recurrence: one single-vector product, or
// one multi-vector product for several.
template <typename Real>
rpy_status lanczos_products(rpy_solver *s, const std::vector<LzRec *> &act, int64_t ld, int col, double *W,
                            hipStream_t st, bool pre = false, bool staged = false) {
    const int64_t np = s->n;
    const bool am = s->angular;
    if (pre) {
        // preconditioned operator L^{-1} M L^{-T} applied to the basis column
        double *t = s->pc_tmp.as<double>();
        rpy_status r = precond_solve_lt(s, act[0]->V + (size_t)col * ld, t, st);
        if (r != RPY_OK) return r;
        const size_t elt = sizeof(vec4_t<Real>);
        HIP_TRY(s, s->f.ensure(elt * (size_t)np));
        if (am) HIP_TRY(s, s->t.ensure(elt * (size_t)np));
        HIP_TRY(s, (launch_stage_vec<double, Real>(t, np, s->f.as<vec4_t<Real>>(), st)));
        if (am) HIP_TRY(s, (launch_stage_vec<double, Real>(t + 3 * np, np, s->t.as<vec4_t<Real>>(), st)));
        r = apply_staged<Real, double>(s, am, W, am ? W + 3 * np : nullptr, st);
        if (r != RPY_OK) return r;
        return precond_solve_l(s, W, st);
    }
    const int m = (int)act.size();
    const size_t elt = sizeof(vec4_t<Real>);
    HIP_TRY(s, s->f.ensure(elt * (size_t)m * np));
    if (am) HIP_TRY(s, s->t.ensure(elt * (size_t)m * np));
    for (int j = 0; j < (staged ? 0 : m); ++j) {   // staged: by next_basis_staged (m = 1)
        const double *v = act[j]->V + (size_t)col * ld;
        HIP_TRY(s, (launch_stage_vec<double, Real>(v, np, s->f.as<vec4_t<Real>>() + (size_t)j * np, st)));
        if (am) HIP_TRY(s, (launch_stage_vec<double, Real>(v + 3 * np, np, s->t.as<vec4_t<Real>>() + (size_t)j * np, st)));
    }
    if (m == 1) return apply_staged<Real, double>(s, am, W, am ? W + 3 * np : nullptr, st);
    return apply_staged_multi<Real, double>(s, am, m, W, am ? W + 3 * np : nullptr, ld, st);
}

}  // namespace

// nrhs Lanczos recurrences for prefactor * M^{1/2} W_r with one geometry,
// advanced in lockstep: each iteration applies M to the current basis
// vector of every recurrence still running (one multi-vector product), then
// runs each recurrence's vector operations and stopping test exactly as for
// a single vector.  Translational products are bit-identical to single ones,
// so each recurrence then reproduces its single call exactly; angular
// products agree to rounding.
// W_r at w_in + r * wstride; outputs at lin / ang + r * ostride.
template <typename Tio>
rpy_status lanczos_run_multi(rpy_solver *s, const Tio *w_in, int nrhs, int64_t wstride, double prefactor,
                             double tol, int max_iter, Tio *lin, Tio *ang, int64_t ostride, int *iters_out,
                             double *incr_out, hipStream_t st, bool accumulate, bool pre) {
    if (pre && nrhs != 1) return fail(s, RPY_ERR_INVALID_ARG, "the preconditioned iteration takes one noise vector");
    const bool ang_mode = s->angular;
    const int64_t np = s->n;
    const int64_t n = (ang_mode ? 6 : 3) * np;
    if (max_iter > kMaxK)
        return fail(s, RPY_ERR_INVALID_ARG, "max_iter exceeds the largest supported Krylov dimension (1024)");
    const int kmax = (int)std::min<int64_t>({(int64_t)max_iter, (int64_t)kMaxK, n});

    // workspace: per recurrence a basis of kmax+1 columns, a product slot and
    // scalar arrays; shared partial sums, eigensolver and monitor scratch
    const int64_t ld = (n + 63) / 64 * 64;
    const size_t per_rec = 8 * (size_t)(kMaxK + 1);   // alpha, beta, h, s, s_prev, est0, est1 (+1 spare)
    HIP_TRY(s, s->lz_basis.ensure((size_t)nrhs * (kmax + 1) * ld * sizeof(double)));
    HIP_TRY(s, s->lz_w.ensure((size_t)nrhs * ld * sizeof(double)));
    HIP_TRY(s, s->lz_scal.ensure(sizeof(double) * (size_t)nrhs * (ST_SIZE + per_rec)));
    const size_t red_rows = std::max<size_t>(kRedBlocks, (size_t)((n + kGtChunk - 1) / kGtChunk));
    HIP_TRY(s, s->lz_red.ensure(sizeof(double) * red_rows * (kMaxK + 1)));
    HIP_TRY(s, s->lz_q.ensure(sizeof(double) * 2 * (size_t)kmax * kmax));
    const int64_t mon_stride = (int64_t)kmax * kMonNodes;
    // monitor scratch, the recurrences' workgroup sums, then the monitor's
    // completion counter
    HIP_TRY(s, s->lz_mon.ensure(sizeof(double) * (2 * (size_t)mon_stride + (size_t)nrhs * PS_SIZE) + sizeof(double)));
    double *const psum = s->lz_mon.as<double>() + 2 * (size_t)mon_stride;
    unsigned *const cnt = reinterpret_cast<unsigned *>(psum + (size_t)nrhs * PS_SIZE);
    HIP_TRY(s, launch_fill_zero<unsigned>(cnt, 1, st));
    if (s->host_stat_cap < (size_t)nrhs * ST_SIZE) {
        if (s->host_stat) (void)hipHostFree(s->host_stat);
        s->host_stat = nullptr;
        s->host_stat_cap = 0;
        HIP_TRY(s, hipHostMalloc((void **)&s->host_stat, sizeof(double) * (size_t)nrhs * ST_SIZE,
                                 hipHostMallocDefault));
        s->host_stat_cap = (size_t)nrhs * ST_SIZE;
    }
    double *const hstat = s->host_stat;
    double *hstat_dev = nullptr;   // the same pinned block as the device addresses it
    HIP_TRY(s, hipHostGetDevicePointer(reinterpret_cast<void **>(&hstat_dev), hstat, 0));
    double *const status_all = s->lz_scal.as<double>();   // [nrhs][ST_SIZE], contiguous for one copy
    double *const W = s->lz_w.as<double>();
    double *const red = s->lz_red.as<double>();
    double *const Q = s->lz_q.as<double>();
    double *const mon = s->lz_mon.as<double>();
    std::vector<LzRec> rec(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        LzRec &R = rec[r];
        R.V = s->lz_basis.as<double>() + (size_t)r * (kmax + 1) * ld;
        R.status = status_all + (size_t)r * ST_SIZE;
        R.alpha = status_all + (size_t)nrhs * ST_SIZE + (size_t)r * per_rec;
        R.beta = R.alpha + (kMaxK + 1);
        R.h = R.beta + (kMaxK + 1);
        R.s = R.h + (kMaxK + 1);
        R.s_prev = R.s + (kMaxK + 1);
        R.est0 = R.s_prev + (kMaxK + 1);
        R.est1 = R.est0 + (kMaxK + 1);
        R.s_final = R.s;
        R.ps = psum + (size_t)r * PS_SIZE;
    }
    const bool fp32 = s->dtype == RPY_F32;
    static const hipError_t lds_attr =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&lanczos_monitor_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * kMonLdsRows * kMonNodes));
    HIP_TRY(s, lds_attr);
    rpy_status r = ensure_vec_buffers(s, ang_mode);
    if (r != RPY_OK) return r;
    auto copy_status = [&]() -> rpy_status {
        HIP_TRY(s, hipMemcpyAsync(hstat, status_all, sizeof(double) * (size_t)nrhs * ST_SIZE, hipMemcpyDeviceToHost,
                                  st));
        HIP_TRY(s, hipStreamSynchronize(st));
        return RPY_OK;
    };

    // beta0 = |W_r|, v1 = W_r / beta0; status blocks start cleared
    HIP_TRY(s, launch_fill_zero<double>(status_all, (int64_t)nrhs * ST_SIZE, st));
    for (int q = 0; q < nrhs; ++q) {
        hipLaunchKernelGGL((sumsq_partial<Tio>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, w_in + q * wstride, n,
                           red);
        hipLaunchKernelGGL(reduce_scalar, dim3(1), dim3(kRedThreads), 0, st, red, kRedBlocks,
                           rec[q].status + ST_BETA0, 1);
    }
    HIP_TRY(s, hipGetLastError());
    if ((r = copy_status()) != RPY_OK) return r;
    for (int q = 0; q < nrhs; ++q) {
        if (iters_out) iters_out[q] = 0;
        if (incr_out) incr_out[q] = 0.0;
        const double beta0 = hstat[(size_t)q * ST_SIZE + ST_BETA0];
        if (!std::isfinite(beta0))
            return fail(s, RPY_ERR_NONFINITE,
                        nrhs == 1 ? std::string("the noise vector W is not finite")
                                  : "noise vector " + std::to_string(q) + " is not finite");
    }
    const int g = grid_for(n);
    for (int q = 0; q < nrhs; ++q) {
        if (hstat[(size_t)q * ST_SIZE + ST_BETA0] == 0.0) {
            // zero W: zero result, nothing to iterate
            rec[q].done = rec[q].converged = true;
            rec[q].incr = 0.0;
            if (!accumulate) {
                HIP_TRY(s, launch_fill_zero<Tio>(lin + q * ostride, 3 * np, st));
                if (ang) HIP_TRY(s, launch_fill_zero<Tio>(ang + q * ostride, 3 * np, st));
            }
            continue;
        }
        hipLaunchKernelGGL((init_basis<Tio>), dim3(g), dim3(256), 0, st, rec[q].V, w_in + q * wstride,
                           rec[q].status + ST_BETA0, n);
    }
    HIP_TRY(s, hipGetLastError());

    // The increment test needs s_{k-1} and s_k.  Each iteration k >= 2
    // computes both by the quadrature monitor, accurate to rounding while
    // T_k's spectrum lies in [1e-10 g, g] (checked by an LDL^T factorisation;
    // otherwise the estimate is NaN).  The eigensolver (exact test, and the
    // exact s_k for the result) runs only when the estimate cannot decide:
    // within 0.1 % of tol, NaN, after a breakdown, or at max_iter.  The loop
    // therefore stops at the same first k as the exact test at every
    // iteration.  RPY_LANCZOS_CHECK=every runs the exact test at every
    // iteration and never uses the estimate.
    const char *check_env = std::getenv("RPY_LANCZOS_CHECK");
    const bool check_every = check_env && std::string(check_env) == "every";
    // RPY_LANCZOS_PROGRESS=m prints each running recurrence's iteration and
    // stopping estimate to stderr every m iterations (long solves)
    const char *progress_env = std::getenv("RPY_LANCZOS_PROGRESS");
    const int progress_every = progress_env ? std::max(0, std::atoi(progress_env)) : 0;
    const int gt_blocks = (int)((n + kGtChunk - 1) / kGtChunk);
    // one plain recurrence: v_{k+1} is staged for its product as it is formed
    const bool stage_next = nrhs == 1 && !pre;
    // One recurrence looks ahead: with the stopping estimate of iteration
    // k - 1 still above kAheadFactor * tol, v_{k+1} and its product are
    // enqueued before the host reads iteration k's stopping test (it waits
    // on an event after the monitor instead of the stream), so the device
    // does not idle through the host's round trip.  Should iteration k stop
    // after all, that product is discarded (its result is never read).
    // RPY_LANCZOS_AHEAD=always enqueues the next product at every monitored
    // iteration from k = 3 on (=never: at none), for testing that a discarded
    // product changes nothing
    constexpr double kAheadFactor = 10.0;
    const char *ahead_env = std::getenv("RPY_LANCZOS_AHEAD");
    const int ahead_mode = !ahead_env ? 0 : std::string(ahead_env) == "always" ? 1 : std::string(ahead_env) == "never" ? 2 : 0;
    const bool lookahead = nrhs == 1 && !check_every;
    hipEvent_t mon_done = nullptr;
    if (lookahead) {
        if (!s->lz_event) HIP_TRY(s, hipEventCreateWithFlags(&s->lz_event, hipEventDisableTiming));
        mon_done = s->lz_event;
    }
    auto enqueue_next_basis = [&](LzRec &R, int j, int k) {
        if (stage_next && fp32)
            hipLaunchKernelGGL(next_basis_staged<float>, dim3((unsigned)((n / 3 + 255) / 256)), dim3(256), 0, st,
                               R.V + (size_t)k * ld, W + j * ld, R.beta + (k - 1), R.status, (int)np, n,
                               s->f.as<float4>(), ang_mode ? s->t.as<float4>() : nullptr);
        else if (stage_next)
            hipLaunchKernelGGL(next_basis_staged<double>, dim3((unsigned)((n / 3 + 255) / 256)), dim3(256), 0, st,
                               R.V + (size_t)k * ld, W + j * ld, R.beta + (k - 1), R.status, (int)np, n,
                               s->f.as<double4>(), ang_mode ? s->t.as<double4>() : nullptr);
        else
            hipLaunchKernelGGL(next_basis_kernel, dim3(g), dim3(256), 0, st, R.V + (size_t)k * ld, W + j * ld,
                               R.beta + (k - 1), R.status, n);
    };
    bool product_ahead = false;   // the product of iteration k was enqueued during iteration k - 1
    std::vector<LzRec *> act;
    for (int k = 1; k <= kmax; ++k) {
        act.clear();
        for (auto &R : rec)
            if (!R.done) act.push_back(&R);
        if (act.empty()) break;
        // w_j = M v_k for every running recurrence (slot j)
        const bool staged = k > 1 && stage_next;
        if (!product_ahead) {
            r = fp32 ? lanczos_products<float>(s, act, ld, k - 1, W, st, pre, staged)
                     : lanczos_products<double>(s, act, ld, k - 1, W, st, pre, staged);
            if (r != RPY_OK) return r;
        }
        product_ahead = false;
        bool basis_ahead = false;   // v_{k+1} enqueued before the stopping test
        for (size_t j = 0; j < act.size(); ++j) {
            LzRec &R = *act[j];
            double *w = W + j * ld;
            const double *vk = R.V + (size_t)(k - 1) * ld;
            // three-term recurrence: w -= beta_{k-1} v_{k-1}, alpha_k = v_k . w,
            // w -= alpha_k v_k and |w|^2 (the second pass's test)
            hipLaunchKernelGGL(recur_beta, dim3(kDotBlocks), dim3(kRedThreads), 0, st, w,
                               k > 1 ? R.V + (size_t)(k - 2) * ld : nullptr, k > 1 ? R.beta + (k - 2) : nullptr, vk,
                               n, R.ps + PS_ALPHA);
            hipLaunchKernelGGL(recur_alpha, dim3(kDotBlocks), dim3(kRedThreads), 0, st, w, vk, R.ps + PS_ALPHA,
                               R.alpha + (k - 1), n, R.ps + PS_NW);
            // classical Gram-Schmidt against V_k, the second pass only when
            // the first removed a sizeable part of w (gemv_n_pass); the
            // workgroup sums of the final |w|^2 for beta_k
            const double pass_bytes = (2.0 * k + 3.0) * (double)n * 8.0;
            hipEvent_t cgs0 = timing_begin(s, RPY_KERNEL_LANCZOS_CGS, 2.0 * pass_bytes);
            if (cgs0) HIP_TRY(s, hipEventRecord(cgs0, st));
            for (int pass = 0; pass < 2; ++pass) {
                const double *skip = pass == 0 ? nullptr : R.status + ST_SKIP;
                hipLaunchKernelGGL(gemv_t_partial, dim3(gt_blocks, (k + kGtCols - 1) / kGtCols), dim3(kRedThreads), 0,
                                   st, R.V, ld, k, w, n, red, skip);
                hipLaunchKernelGGL(gemv_t_final, dim3(k), dim3(kRedThreads), 0, st, red, gt_blocks, k, R.h, skip);
                hipLaunchKernelGGL(gemv_n_pass, dim3(g), dim3(256), 0, st, R.V, ld, k, R.h, w, n, pass, R.ps + PS_NW,
                                   R.status, pass_bytes, R.ps + PS_BETA);
            }
            if (hipEvent_t cgs1 = timing_end(s, RPY_KERNEL_LANCZOS_CGS)) HIP_TRY(s, hipEventRecord(cgs1, st));
            HIP_TRY(s, hipGetLastError());
            R.exact = (k == kmax) || check_every;
        }
        // stopping test by the quadrature estimate, all running recurrences at
        // once; beta_k (and the breakdown bookkeeping) in the monitor's launch
        const bool monitor = !check_every && k >= 2 && k < kmax;
        if (!monitor) {
            for (LzRec *R : act)
                hipLaunchKernelGGL(beta_kernel, dim3(1), dim3(64), 0, st, R->ps + PS_BETA, g, R->alpha, R->beta, k,
                                   R->status);
            HIP_TRY(s, hipGetLastError());
        }
        if (monitor) {
            // iteration k - 1's estimate, read before this iteration's monitor
            // rewrites the pinned mirror (the host waited for that monitor)
            const double prev_est = lookahead ? hstat[(act[0]->status - status_all) + ST_EST] : 0.0;
            for (LzRec *R : act) {
                const unsigned lds = k <= kMonLdsRows ? (unsigned)(sizeof(double) * k * kMonNodes) : 0u;
                hipLaunchKernelGGL(lanczos_monitor_kernel, dim3(2), dim3(kMonThreads), lds, st, R->alpha, R->beta, k,
                                   mon, mon_stride, R->est0, R->est1, cnt, R->status, R->ps + PS_BETA, g,
                                   hstat_dev + (R->status - status_all));
            }
            HIP_TRY(s, hipGetLastError());
            if (lookahead) {
                // the previous estimate (k >= 3) decides whether the product goes ahead too
                LzRec &R = *act[0];
                HIP_TRY(s, hipEventRecord(mon_done, st));
                enqueue_next_basis(R, 0, k);
                basis_ahead = true;
                const bool ahead = ahead_mode == 1 || (ahead_mode == 0 && prev_est > kAheadFactor * tol);
                if (k >= 3 && k < kmax && ahead) {
                    r = fp32 ? lanczos_products<float>(s, act, ld, k, W, st, pre, stage_next)
                             : lanczos_products<double>(s, act, ld, k, W, st, pre, stage_next);
                    if (r != RPY_OK) return r;
                    product_ahead = true;
                }
                HIP_TRY(s, hipGetLastError());
                HIP_TRY(s, hipEventSynchronize(mon_done));   // the monitor wrote the status block to hstat
            } else {
                HIP_TRY(s, hipStreamSynchronize(st));   // the monitors wrote the status blocks to hstat
            }
            if (progress_every > 0 && k % progress_every == 0) {
                for (LzRec *R : act)
                    std::fprintf(stderr, "rpy lanczos: recurrence %d, k = %d, estimate %.3e\n",
                                 (int)(R - rec.data()), k, hstat[(R->status - status_all) + ST_EST]);
                std::fflush(stderr);
            }
            for (LzRec *R : act) {
                const double *hs = hstat + (R->status - status_all);
                const double est = hs[ST_EST];
                // the exact test only where the estimate cannot decide: a
                // breakdown, an eigenvalue outside the quadrature's range
                // (NaN), or an estimate within 0.1 % of tol
                R->exact = hs[ST_BREAK] > 0.0 || !std::isfinite(est) || std::fabs(est - tol) <= 1e-3 * tol;
                if (!R->exact && est < tol) {
                    // converged: the quadrature s_k is T_k^{1/2} e_1 to rounding
                    R->incr = est;
                    R->kf = k;
                    R->s_final = R->est1;
                    R->converged = R->done = true;
                }
            }
        }
        bool any_exact = false;
        for (LzRec *R : act) {
            if (R->done || !R->exact) continue;
            any_exact = true;
            hipLaunchKernelGGL(tridiag_sqrt_kernel, dim3(2), dim3(kEigThreads), 0, st, R->alpha, R->beta, k, R->s_prev,
                               R->s, Q, (int64_t)kmax * kmax, R->status);
            hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(kRedThreads), 0, st, R->s_prev, R->s, k, R->status,
                               (int)ST_INCR);
        }
        if (any_exact) {
            HIP_TRY(s, hipGetLastError());
            if ((r = copy_status()) != RPY_OK) return r;
            for (LzRec *R : act) {
                if (R->done || !R->exact) continue;
                const double *hs = hstat + (R->status - status_all);
                R->incr = hs[ST_INCR];
                const int kb = (int)hs[ST_BREAK];
                R->kf = k;
                if (kb > 0) {
                    // invariant Krylov space at kb: T_k = diag(T_kb, 0), so s_k = [s_kb; 0]
                    R->kf = kb;
                    R->converged = R->done = true;
                } else if (((int)hs[ST_FLAGS]) & FLAG_NOT_SPD) {
                    R->not_spd = R->done = true;
                } else if (k >= 2 && R->incr < tol) {
                    R->converged = R->done = true;
                } else if (k == kmax) {
                    R->done = true;
                }
            }
        }
        // v_{k+1} = w / beta_k for the recurrences that go on
        for (size_t j = 0; j < act.size(); ++j) {
            LzRec &R = *act[j];
            if (R.done || basis_ahead) continue;
            enqueue_next_basis(R, (int)j, k);
        }
        HIP_TRY(s, hipGetLastError());
    }
    bool any_not_spd = false, any_not_conv = false;
    for (int q = 0; q < nrhs; ++q) {
        LzRec &R = rec[q];
        if (R.kf > 0 && pre) {
            // z = beta0 V s, then y = prefactor L z
            double *z = s->pc_tmp.as<double>();
            hipLaunchKernelGGL((combine_out<double>), dim3(g), dim3(256), 0, st, R.V, ld, R.kf, R.s_final, R.status,
                               1.0, n, 3 * np, 0, z, z + 3 * np);
            HIP_TRY(s, hipGetLastError());
            r = precond_mul_l<Tio>(s, z, prefactor, accumulate, lin, ang, st);
            if (r != RPY_OK) return r;
        } else if (R.kf > 0) {
            hipLaunchKernelGGL((combine_out<Tio>), dim3(g), dim3(256), 0, st, R.V, ld, R.kf, R.s_final, R.status,
                               prefactor, n, 3 * np, accumulate ? 1 : 0, lin + q * ostride,
                               ang ? ang + q * ostride : nullptr);
        }
        if (iters_out) iters_out[q] = R.kf;
        if (incr_out) incr_out[q] = R.incr;
        any_not_spd |= R.not_spd;
        any_not_conv |= !R.converged && !R.not_spd;
    }
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipStreamSynchronize(st));
    if (s->timing) {
        // the Gram-Schmidt timing counted two passes per iteration; take off
        // the bytes of the second passes that were skipped
        if ((r = copy_status()) != RPY_OK) return r;
        for (int q = 0; q < nrhs; ++q) s->ev_pairs[RPY_KERNEL_LANCZOS_CGS] -= hstat[(size_t)q * ST_SIZE + ST_SKIPPED];
    }
    if (any_not_spd)
        return fail(s, RPY_ERR_NOT_SPD, "the mobility matrix is not positive definite (negative Ritz value)");
    if (any_not_conv)
        return fail(s, RPY_ERR_NOT_CONVERGED, "Lanczos did not reach the tolerance within max_iter iterations");
    return RPY_OK;
}

template <typename Tio>
rpy_status lanczos_run(rpy_solver *s, const Tio *w_in, double prefactor, double tol, int max_iter, Tio *lin,
                       Tio *ang, int *iters_out, double *incr_out, hipStream_t st, bool accumulate) {
    return lanczos_run_multi<Tio>(s, w_in, 1, 0, prefactor, tol, max_iter, lin, ang, 0, iters_out, incr_out, st,
                                  accumulate, false);
}

template rpy_status lanczos_run<float>(rpy_solver *, const float *, double, double, int, float *, float *, int *,
                                       double *, hipStream_t, bool);
template rpy_status lanczos_run<double>(rpy_solver *, const double *, double, double, int, double *, double *, int *,
                                        double *, hipStream_t, bool);
template rpy_status lanczos_run_multi<float>(rpy_solver *, const float *, int, int64_t, double, double, int, float *,
                                             float *, int64_t, int *, double *, hipStream_t, bool, bool);
template rpy_status lanczos_run_multi<double>(rpy_solver *, const double *, int, int64_t, double, double, int,
                                              double *, double *, int64_t, int *, double *, hipStream_t, bool, bool);

}  // namespace rpy

extern "C" rpy_status rpy_sqrt_mdot_w(rpy_solver *s, const void *w, double prefactor, double tol, int max_iter,
                                      void *lin_out, void *ang_out, int *iters_out, double *incr_out,
                                      void *hip_stream) {
    using namespace rpy;
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!w || !lin_out) return fail(s, RPY_ERR_INVALID_ARG, "W and the linear output must not be NULL");
    if (s->angular && !ang_out) return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!s->angular && ang_out) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    if (!(tol > 0.0 && tol < 1.0)) return fail(s, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(s, RPY_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!std::isfinite(prefactor)) return fail(s, RPY_ERR_INVALID_ARG, "prefactor must be finite");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return lanczos_run<double>(s, static_cast<const double *>(w), prefactor, tol, max_iter,
                                   static_cast<double *>(lin_out), static_cast<double *>(ang_out), iters_out,
                                   incr_out, st, false);
    return lanczos_run<float>(s, static_cast<const float *>(w), prefactor, tol, max_iter, static_cast<float *>(lin_out),
                              static_cast<float *>(ang_out), iters_out, incr_out, st, false);
}

extern "C" rpy_status rpy_sqrt_mdot_w_multi(rpy_solver *s, const void *w, int nrhs, double prefactor, double tol,
                                            int max_iter, void *lin_out, void *ang_out, int *iters_out,
                                            double *incr_out, void *hip_stream) {
    using namespace rpy;
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(s, RPY_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    if (!w || !lin_out) return fail(s, RPY_ERR_INVALID_ARG, "W and the linear output must not be NULL");
    if (s->angular && !ang_out) return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!s->angular && ang_out) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    if (!(tol > 0.0 && tol < 1.0)) return fail(s, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(s, RPY_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!std::isfinite(prefactor)) return fail(s, RPY_ERR_INVALID_ARG, "prefactor must be finite");
    if ((int64_t)nrhs * s->n > (int64_t)INT32_MAX)
        return fail(s, RPY_ERR_INVALID_ARG, "nrhs * n must stay below 2^31");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t wstride = (s->angular ? 6 : 3) * s->n, ostride = 3 * s->n;
    if (s->dtype == RPY_F64)
        return lanczos_run_multi<double>(s, static_cast<const double *>(w), nrhs, wstride, prefactor, tol, max_iter,
                                         static_cast<double *>(lin_out), static_cast<double *>(ang_out), ostride,
                                         iters_out, incr_out, st, false);
    return lanczos_run_multi<float>(s, static_cast<const float *>(w), nrhs, wstride, prefactor, tol, max_iter,
                                    static_cast<float *>(lin_out), static_cast<float *>(ang_out), ostride, iters_out,
                                    incr_out, st, false);
}

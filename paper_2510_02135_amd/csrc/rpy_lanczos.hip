// M^{1/2} W by Lanczos on the device (Sec. 3.3: Krylov square root of Ando,
// Chow, Saad & Skolnick for solvers that only apply M).
//
// Every vector operation is float64 and runs on the device; the products
// M v_k use the solver's pair precision (float32 pairs for float32
// solvers).  Per iteration k (v_k = column k-1 of the basis V):
//   w = M v_k;  w -= beta_{k-1} v_{k-1};  alpha_k = v_k . w;  w -= alpha_k v_k
//   two passes of classical Gram-Schmidt against V_k (w -= V_k (V_k^T w))
//   beta_k = |w|
//   T_k = tridiag(beta, alpha, beta) = Q diag(lambda) Q^T on one workgroup
//     (implicit-shift QL), s_k = Q diag(sqrt(lambda)) Q^T e_1, and the
//     relative increment |s_k - [s_{k-1}; 0]| / |s_k|, which equals
//     |y_k - y_{k-1}| / |y_k| for y_k = beta_0 V_k s_k because V_k is
//     orthonormal;
//   v_{k+1} = w / beta_k.
// The host reads a small status block after each iteration to decide
// whether to stop (first k >= 2 with increment < tol; a clearly negative
// Ritz value; beta_k ~ 0 meaning the Krylov space is invariant).  s_{k-1}
// and s_k come from a quadrature estimate of T^{1/2} e_1 that is exact to
// rounding for safely positive definite T_k; the eigensolver runs only where
// that estimate cannot decide.  The final y = prefactor * beta_0 V_k s_k is
// formed on the device and written in the caller's dtype.
//
// Reductions are two-stage with a fixed block count and fixed order, so the
// result does not depend on scheduling.
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

// status block (double): [0] beta0, [1] relative increment, [2] flags,
// [3] running max(|alpha|, beta), [4] first breakdown iteration (0 = none),
// [5] estimated relative increment (monitor)
// status block: beta0, increment, flags, scale of T, breakdown step, stopping
// estimate, |w|^2 before Gram-Schmidt, skip flag of the second pass, bytes
// of skipped passes
enum { ST_BETA0 = 0, ST_INCR = 1, ST_FLAGS = 2, ST_TSCALE = 3, ST_BREAK = 4, ST_EST = 5, ST_NW = 6, ST_SKIP = 7,
       ST_SKIPPED = 8, ST_SIZE = 10 };
enum { FLAG_NOT_SPD = 1, FLAG_NONFINITE = 2 };

// partial[b] = sum over the b-th strided slice of a[i] * b[i]
__global__ void dot_partial(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                            double *__restrict__ partial) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc = fma(a[i], b[i], acc);
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
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

// *out = a . b (or its square root) in one launch: every block stores its
// partial sum, and the block that finishes last (a counter, reset by it)
// adds the partials in the fixed order of reduce_scalar, so the result is
// that of dot_partial + reduce_scalar bit for bit.  With `status` the last
// block then runs the breakdown bookkeeping of iteration k.
__global__ void __launch_bounds__(kRedThreads)
dot_reduce(const double *__restrict__ a, const double *__restrict__ b, int64_t n, double *__restrict__ partial,
           unsigned *__restrict__ counter, double *out, int take_sqrt, const double *alpha, const double *beta,
           int k, double *status) {
    __shared__ double sh[kRedThreads];
    __shared__ bool last;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc = fma(a[i], b[i], acc);
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = r;
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double t = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) t += partial[i];
    const double tot = block_sum(t, sh);
    if (threadIdx.x == 0) {
        *out = take_sqrt ? sqrt(tot) : tot;
        *counter = 0u;
        if (status) finish_iter(alpha, beta, k, status);
    }
}

// out = sum(partial) (or its square root); optional second copy
__global__ void reduce_scalar(const double *__restrict__ partial, int nb, double *out, int take_sqrt) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partial[i];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = take_sqrt ? sqrt(r) : r;
}

// y += sign * (*coef) * x
__global__ void axpy_dev(double *__restrict__ y, const double *__restrict__ x, const double *coef, double sign,
                         int64_t n) {
    const double c = sign * (*coef);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = fma(c, x[i], y[i]);
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
// each thread keeps its kGtRows entries of w in registers and issues all
// kGtRows * kGtCols coalesced loads of its tile at once (unguarded in the
// interior), then the block reduces the tile's columns through LDS.  Every
// sum has a fixed order (deterministic).
constexpr int kGtRows = 4;
constexpr int kGtCols = 16;
constexpr int kGtChunk = kGtRows * kRedThreads;   // rows per chunk
template <bool GUARD>
__device__ __forceinline__ void gemv_t_tile(const double *__restrict__ V, int64_t ld, int j0, int k,
                                            const double *__restrict__ w, int64_t n, int64_t base,
                                            double (&acc)[kGtCols]) {
    double wr[kGtRows];
#pragma unroll
    for (int q = 0; q < kGtRows; ++q) {
        const int64_t i = base + (int64_t)q * kRedThreads;
        wr[q] = (!GUARD || i < n) ? w[i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kGtCols; ++c) {
        acc[c] = 0.0;
        if (!GUARD || j0 + c < k) {
            const double *col = V + (size_t)(j0 + c) * ld;
#pragma unroll
            for (int q = 0; q < kGtRows; ++q) {
                const int64_t i = base + (int64_t)q * kRedThreads;
                if (!GUARD || i < n) acc[c] = fma(col[i], wr[q], acc[c]);
            }
        }
    }
}

// The kernels of a Gram-Schmidt pass take `skip` (NULL for the first pass):
// the second pass does nothing when *skip is set (see cgs_decide).
__global__ void __launch_bounds__(kRedThreads)
gemv_t_partial(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ w, int64_t n,
               double *__restrict__ partial, const double *skip) {
    static_assert(kRedThreads == 256 && kGtCols * 16 == kRedThreads, "tile reduction layout");
    if (skip && *skip != 0.0) return;
    __shared__ double sh[kGtCols][kRedThreads];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kGtChunk + tid;
    const int j0 = (int)blockIdx.y * kGtCols;
    double acc[kGtCols];
    if ((int64_t)blockIdx.x * kGtChunk + kGtChunk <= n && j0 + kGtCols <= k)
        gemv_t_tile<false>(V, ld, j0, k, w, n, base, acc);
    else
        gemv_t_tile<true>(V, ld, j0, k, w, n, base, acc);
#pragma unroll
    for (int c = 0; c < kGtCols; ++c) sh[c][tid] = acc[c];
    __syncthreads();
    // column gc = tid / 16 of the tile: 16 threads sum its 256 partials
    const int gc = tid >> 4, gl = tid & 15;
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < kRedThreads / 16; ++m) v += sh[gc][gl + 16 * m];
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
    if (gl == 0 && j0 + gc < k) partial[(size_t)blockIdx.x * k + j0 + gc] = v;
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

// w[i] -= sum_j V[j][i] h[j]
__global__ void gemv_n_sub(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ h,
                           double *__restrict__ w, int64_t n, const double *skip) {
    __shared__ double hs[kMaxK];
    if (skip && *skip != 0.0) return;
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(V[(size_t)j * ld + i], hs[j], acc);
        w[i] -= acc;
    }
}

// After the first Gram-Schmidt pass, with h its coefficients: the removed
// part has squared norm |h|^2 (V orthonormal), so the second pass is needed
// only when |h|^2 > |w|^2 / 2, i.e. when the first pass cut |w| below
// 1/sqrt(2) of itself (Kahan and Parlett's "twice is enough" test, as in
// Daniel, Gragg, Kaufman and Stewart's reorthogonalisation).  Otherwise w is
// already orthogonal to V to working precision; the skip flag is set and the
// skipped pass's bytes are counted.  NaN never skips.
__global__ void cgs_decide(const double *__restrict__ h, int k, double *__restrict__ status, double pass_bytes) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    for (int j = threadIdx.x; j < k; j += blockDim.x) acc = fma(h[j], h[j], acc);
    const double hh = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        const bool skip = hh <= 0.5 * status[ST_NW];
        status[ST_SKIP] = skip ? 1.0 : 0.0;
        if (skip) status[ST_SKIPPED] += pass_bytes;
    }
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

// Quadrature estimates of s_{k-1} (workgroup 0) and s_k (workgroup 1);
// see monitor_block.
__global__ void __launch_bounds__(kMonThreads)
lanczos_monitor_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int k,
                       double *__restrict__ scratch, int64_t sstride, double *__restrict__ est0,
                       double *__restrict__ est1) {
    const int kk = k - 1 + (int)blockIdx.x;
    if (kk <= 0) return;
    monitor_block(alpha, beta, k, kk, scratch + (size_t)blockIdx.x * sstride, blockIdx.x == 0 ? est0 : est1);
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

// Device state of one recurrence inside the shared workspace, and the
// host's view of its progress.
struct LzRec {
    double *V = nullptr;   // basis, cap + 1 columns of ld doubles
    double *status = nullptr, *alpha = nullptr, *beta = nullptr, *h = nullptr;
    double *s = nullptr, *s_prev = nullptr, *est0 = nullptr, *est1 = nullptr;
    int kf = 0;
    double incr = INFINITY;
    const double *s_final = nullptr;   // exact s_k unless the estimate decided
    bool done = false, converged = false, not_spd = false, exact = false;
};

int grid_for(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + 255) / 256)); }

// w (slots of ld doubles, linear then angular rows) = M v for the basis
// column `col` of every listed recurrence: one single-vector product, or
// one multi-vector product for several.
template <typename Real>
rpy_status lanczos_products(rpy_solver *s, const std::vector<LzRec *> &act, int64_t ld, int col, double *W,
                            hipStream_t st, bool pre = false) {
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
    for (int j = 0; j < m; ++j) {
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
    // monitor scratch, then one word for the counter of dot_reduce
    HIP_TRY(s, s->lz_mon.ensure(sizeof(double) * (2 * (size_t)mon_stride + 1)));
    unsigned *const cnt = reinterpret_cast<unsigned *>(s->lz_mon.as<double>() + 2 * (size_t)mon_stride);
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
    }
    const bool fp32 = s->dtype == RPY_F32;
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
    std::vector<LzRec *> act;
    for (int k = 1; k <= kmax; ++k) {
        act.clear();
        for (auto &R : rec)
            if (!R.done) act.push_back(&R);
        if (act.empty()) break;
        // w_j = M v_k for every running recurrence (slot j)
        r = fp32 ? lanczos_products<float>(s, act, ld, k - 1, W, st, pre)
                 : lanczos_products<double>(s, act, ld, k - 1, W, st, pre);
        if (r != RPY_OK) return r;
        for (size_t j = 0; j < act.size(); ++j) {
            LzRec &R = *act[j];
            double *w = W + j * ld;
            const double *vk = R.V + (size_t)(k - 1) * ld;
            // three-term recurrence
            if (k > 1)
                hipLaunchKernelGGL(axpy_dev, dim3(g), dim3(256), 0, st, w, R.V + (size_t)(k - 2) * ld, R.beta + (k - 2),
                                   -1.0, n);
            hipLaunchKernelGGL(dot_reduce, dim3(kRedBlocks), dim3(kRedThreads), 0, st, vk, w, n, red, cnt,
                               R.alpha + (k - 1), 0, nullptr, nullptr, 0, nullptr);
            hipLaunchKernelGGL(axpy_dev, dim3(g), dim3(256), 0, st, w, vk, R.alpha + (k - 1), -1.0, n);
            // classical Gram-Schmidt against V_k, the second pass only when
            // the first removed a sizeable part of w (cgs_decide)
            const double pass_bytes = (2.0 * k + 3.0) * (double)n * 8.0;
            hipLaunchKernelGGL(dot_reduce, dim3(kRedBlocks), dim3(kRedThreads), 0, st, w, w, n, red, cnt,
                               R.status + ST_NW, 0, nullptr, nullptr, 0, nullptr);
            hipEvent_t cgs0 = timing_begin(s, RPY_KERNEL_LANCZOS_CGS, 2.0 * pass_bytes);
            if (cgs0) HIP_TRY(s, hipEventRecord(cgs0, st));
            for (int pass = 0; pass < 2; ++pass) {
                const double *skip = pass == 0 ? nullptr : R.status + ST_SKIP;
                hipLaunchKernelGGL(gemv_t_partial, dim3(gt_blocks, (k + kGtCols - 1) / kGtCols), dim3(kRedThreads), 0,
                                   st, R.V, ld, k, w, n, red, skip);
                hipLaunchKernelGGL(gemv_t_final, dim3(k), dim3(kRedThreads), 0, st, red, gt_blocks, k, R.h, skip);
                if (pass == 0)
                    hipLaunchKernelGGL(cgs_decide, dim3(1), dim3(kRedThreads), 0, st, R.h, k, R.status, pass_bytes);
                hipLaunchKernelGGL(gemv_n_sub, dim3(g), dim3(256), 0, st, R.V, ld, k, R.h, w, n, skip);
            }
            if (hipEvent_t cgs1 = timing_end(s, RPY_KERNEL_LANCZOS_CGS)) HIP_TRY(s, hipEventRecord(cgs1, st));
            // beta_k = |w|, breakdown bookkeeping
            hipLaunchKernelGGL(dot_reduce, dim3(kRedBlocks), dim3(kRedThreads), 0, st, w, w, n, red, cnt,
                               R.beta + (k - 1), 1, R.alpha, R.beta, k, R.status);
            HIP_TRY(s, hipGetLastError());
            R.exact = (k == kmax) || check_every;
        }
        // stopping test by the quadrature estimate, all running recurrences at once
        if (!check_every && k >= 2 && k < kmax) {
            for (LzRec *R : act) {
                hipLaunchKernelGGL(lanczos_monitor_kernel, dim3(2), dim3(kMonThreads), 0, st, R->alpha, R->beta, k,
                                   mon, mon_stride, R->est0, R->est1);
                hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(kRedThreads), 0, st, R->est0, R->est1, k,
                                   R->status, (int)ST_EST);
            }
            HIP_TRY(s, hipGetLastError());
            if ((r = copy_status()) != RPY_OK) return r;
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
            if (R.done) continue;
            hipLaunchKernelGGL(next_basis_kernel, dim3(g), dim3(256), 0, st, R.V + (size_t)k * ld, W + j * ld,
                               R.beta + (k - 1), R.status, n);
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

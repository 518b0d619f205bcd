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
enum { ST_BETA0 = 0, ST_INCR = 1, ST_FLAGS = 2, ST_TSCALE = 3, ST_BREAK = 4, ST_EST = 5, ST_SIZE = 8 };
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

__global__ void __launch_bounds__(kRedThreads)
gemv_t_partial(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ w, int64_t n,
               double *__restrict__ partial) {
    static_assert(kRedThreads == 256 && kGtCols * 16 == kRedThreads, "tile reduction layout");
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
__global__ void gemv_t_final(const double *__restrict__ partial, int nb, int k, double *__restrict__ h) {
    __shared__ double sh[kRedThreads];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[(size_t)b * k + j];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) h[j] = r;
}

// w[i] -= sum_j V[j][i] h[j]
__global__ void gemv_n_sub(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ h,
                           double *__restrict__ w, int64_t n) {
    __shared__ double hs[kMaxK];
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(V[(size_t)j * ld + i], hs[j], acc);
        w[i] -= acc;
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
__global__ void finish_iter_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int k,
                                   double *__restrict__ status) {
    if (threadIdx.x != 0) return;
    const double a = fabs(alpha[k - 1]), b = beta[k - 1];
    const double sc = fmax(status[ST_TSCALE], fmax(a, b));
    status[ST_TSCALE] = sc;
    if (status[ST_BREAK] == 0.0 && !(b > 1e-14 * sc)) status[ST_BREAK] = (double)k;
}

// v_{k+1} = w / beta_k, or zeros once a breakdown has been recorded.
__global__ void next_basis_kernel(double *__restrict__ dst, const double *__restrict__ src,
                                  const double *__restrict__ beta, const double *__restrict__ status, int64_t n) {
    const bool broken = status[ST_BREAK] != 0.0;
    const double inv = broken ? 0.0 : 1.0 / (*beta);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = broken ? 0.0 : src[i] * inv;
}

struct LanczosWork {
    double *V = nullptr;
    int64_t ld = 0;
    int cap = 0;
    double *w = nullptr, *alpha = nullptr, *beta = nullptr, *h = nullptr, *red = nullptr;
    double *s = nullptr, *s_prev = nullptr, *Q = nullptr, *status = nullptr;
    double *est0 = nullptr, *est1 = nullptr, *mon = nullptr;
    int64_t mon_stride = 0;
};

int grid_for(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

template <typename Tio>
rpy_status lanczos_run(rpy_solver *s, const Tio *w_in, double prefactor, double tol, int max_iter, Tio *lin,
                       Tio *ang, int *iters_out, double *incr_out, hipStream_t st, bool accumulate) {
    const bool ang_mode = s->angular;
    const int64_t np = s->n;
    const int64_t n = (ang_mode ? 6 : 3) * np;
    const int kmax = (int)std::min<int64_t>({(int64_t)max_iter, (int64_t)kMaxK, n});
    if (max_iter > kMaxK)
        return fail(s, RPY_ERR_INVALID_ARG, "max_iter exceeds the largest supported Krylov dimension (1024)");

    // workspace: basis of kmax+1 columns, scalars, Q (kmax x kmax)
    const int64_t ld = (n + 63) / 64 * 64;
    const size_t basis_bytes = (size_t)(kmax + 1) * ld * sizeof(double);
    HIP_TRY(s, s->lz_basis.ensure(basis_bytes));
    HIP_TRY(s, s->lz_w.ensure((size_t)ld * sizeof(double)));
    HIP_TRY(s, s->lz_scal.ensure(sizeof(double) * (ST_SIZE + 8 * (size_t)(kMaxK + 1))));
    // partial sums: the Gram-Schmidt projection keeps one per (row chunk, column)
    const size_t red_rows = std::max<size_t>(kRedBlocks, (size_t)((n + kGtChunk - 1) / kGtChunk));
    HIP_TRY(s, s->lz_red.ensure(sizeof(double) * red_rows * (kMaxK + 1)));
    HIP_TRY(s, s->lz_q.ensure(sizeof(double) * 2 * (size_t)kmax * kmax));
    // monitor scratch: per workgroup, one vector of kMonNodes systems
    const int64_t mon_stride = (int64_t)kmax * kMonNodes;
    HIP_TRY(s, s->lz_mon.ensure(sizeof(double) * 2 * (size_t)mon_stride));
    if (!s->host_scal) HIP_TRY(s, hipHostMalloc((void **)&s->host_scal, sizeof(double) * 8, hipHostMallocDefault));
    LanczosWork L;
    L.V = s->lz_basis.as<double>();
    L.ld = ld;
    L.cap = kmax;
    L.w = s->lz_w.as<double>();
    L.status = s->lz_scal.as<double>();
    L.alpha = L.status + ST_SIZE;
    L.beta = L.alpha + (kMaxK + 1);
    L.h = L.beta + (kMaxK + 1);
    L.s = L.h + (kMaxK + 1);
    L.s_prev = L.s + (kMaxK + 1);
    L.est0 = L.s_prev + (kMaxK + 1);
    L.est1 = L.est0 + (kMaxK + 1);
    L.mon = s->lz_mon.as<double>();
    L.mon_stride = mon_stride;
    L.red = s->lz_red.as<double>();
    L.Q = s->lz_q.as<double>();

    const bool fp32 = s->dtype == RPY_F32;
    rpy_status r = ensure_vec_buffers(s, ang_mode);
    if (r != RPY_OK) return r;

    // beta0 = |W|, v1 = W / beta0; the status block starts cleared
    HIP_TRY(s, launch_fill_zero<double>(L.status, ST_SIZE, st));
    hipLaunchKernelGGL((sumsq_partial<Tio>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, w_in, n, L.red);
    hipLaunchKernelGGL(reduce_scalar, dim3(1), dim3(kRedThreads), 0, st, L.red, kRedBlocks, L.status + ST_BETA0, 1);
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipMemcpyAsync(s->host_scal, L.status, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(s, hipStreamSynchronize(st));
    const double beta0 = s->host_scal[0];
    if (!std::isfinite(beta0)) return fail(s, RPY_ERR_NONFINITE, "the noise vector W is not finite");
    if (iters_out) *iters_out = 0;
    if (incr_out) *incr_out = 0.0;
    if (beta0 == 0.0) {
        if (!accumulate) {
            HIP_TRY(s, launch_fill_zero<Tio>(lin, 3 * np, st));
            if (ang) HIP_TRY(s, launch_fill_zero<Tio>(ang, 3 * np, st));
        }
        return RPY_OK;
    }
    hipLaunchKernelGGL((init_basis<Tio>), dim3(grid_for(n)), dim3(256), 0, st, L.V, w_in, L.status + ST_BETA0, n);
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
    const int g = grid_for(n);
    const int gt_blocks = (int)((n + kGtChunk - 1) / kGtChunk);
    int k = 0, kf = 0;
    double incr = INFINITY;
    const double *s_final = L.s;   // exact s_k unless the estimate decided
    bool converged = false, not_spd = false;
    for (k = 1; k <= kmax; ++k) {
        const double *vk = L.V + (size_t)(k - 1) * ld;
        // w = M v_k
        if (fp32) {
            HIP_TRY(s, (launch_stage_vec<double, float>(vk, np, s->f.as<float4>(), st)));
            if (ang_mode) HIP_TRY(s, (launch_stage_vec<double, float>(vk + 3 * np, np, s->t.as<float4>(), st)));
            r = apply_staged<float, double>(s, ang_mode, L.w, ang_mode ? L.w + 3 * np : nullptr, st);
        } else {
            HIP_TRY(s, (launch_stage_vec<double, double>(vk, np, s->f.as<double4>(), st)));
            if (ang_mode) HIP_TRY(s, (launch_stage_vec<double, double>(vk + 3 * np, np, s->t.as<double4>(), st)));
            r = apply_staged<double, double>(s, ang_mode, L.w, ang_mode ? L.w + 3 * np : nullptr, st);
        }
        if (r != RPY_OK) return r;
        // three-term recurrence
        if (k > 1)
            hipLaunchKernelGGL(axpy_dev, dim3(g), dim3(256), 0, st, L.w, L.V + (size_t)(k - 2) * ld, L.beta + (k - 2),
                               -1.0, n);
        hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, vk, L.w, n, L.red);
        hipLaunchKernelGGL(reduce_scalar, dim3(1), dim3(kRedThreads), 0, st, L.red, kRedBlocks, L.alpha + (k - 1), 0);
        hipLaunchKernelGGL(axpy_dev, dim3(g), dim3(256), 0, st, L.w, vk, L.alpha + (k - 1), -1.0, n);
        // classical Gram-Schmidt against V_k, twice
        hipEvent_t cgs0 = timing_begin(s, RPY_KERNEL_LANCZOS_CGS, 2.0 * (2.0 * k + 3.0) * (double)n * 8.0);
        if (cgs0) HIP_TRY(s, hipEventRecord(cgs0, st));
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(gemv_t_partial, dim3(gt_blocks, (k + kGtCols - 1) / kGtCols), dim3(kRedThreads), 0, st,
                               L.V, ld, k, L.w, n, L.red);
            hipLaunchKernelGGL(gemv_t_final, dim3(k), dim3(kRedThreads), 0, st, L.red, gt_blocks, k, L.h);
            hipLaunchKernelGGL(gemv_n_sub, dim3(g), dim3(256), 0, st, L.V, ld, k, L.h, L.w, n);
        }
        if (hipEvent_t cgs1 = timing_end(s, RPY_KERNEL_LANCZOS_CGS)) HIP_TRY(s, hipEventRecord(cgs1, st));
        // beta_k = |w|, breakdown bookkeeping, v_{k+1}
        hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, L.w, L.w, n, L.red);
        hipLaunchKernelGGL(reduce_scalar, dim3(1), dim3(kRedThreads), 0, st, L.red, kRedBlocks, L.beta + (k - 1), 1);
        hipLaunchKernelGGL(finish_iter_kernel, dim3(1), dim3(64), 0, st, L.alpha, L.beta, k, L.status);
        HIP_TRY(s, hipGetLastError());
        const bool last = (k == kmax);
        bool exact = last || check_every;
        if (!exact && k >= 2) {
            hipLaunchKernelGGL(lanczos_monitor_kernel, dim3(2), dim3(kMonThreads), 0, st, L.alpha, L.beta, k, L.mon,
                               L.mon_stride, L.est0, L.est1);
            hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(kRedThreads), 0, st, L.est0, L.est1, k, L.status,
                               (int)ST_EST);
            HIP_TRY(s, hipGetLastError());
            HIP_TRY(s, hipMemcpyAsync(s->host_scal, L.status, sizeof(double) * ST_SIZE, hipMemcpyDeviceToHost, st));
            HIP_TRY(s, hipStreamSynchronize(st));
            const double est = s->host_scal[ST_EST];
            // the exact test only where the estimate cannot decide: a breakdown,
            // an eigenvalue outside the quadrature's range (NaN), or an
            // estimate within 0.1 % of tol
            exact = s->host_scal[ST_BREAK] > 0.0 || !std::isfinite(est) || std::fabs(est - tol) <= 1e-3 * tol;
            if (!exact && est < tol) {
                // converged: the quadrature s_k is T_k^{1/2} e_1 to rounding
                incr = est;
                kf = k;
                s_final = L.est1;
                converged = true;
                break;
            }
        }
        if (exact) {
            hipLaunchKernelGGL(tridiag_sqrt_kernel, dim3(2), dim3(kEigThreads), 0, st, L.alpha, L.beta, k, L.s_prev,
                               L.s, L.Q, (int64_t)kmax * kmax, L.status);
            hipLaunchKernelGGL(increment_kernel, dim3(1), dim3(kRedThreads), 0, st, L.s_prev, L.s, k, L.status,
                               (int)ST_INCR);
            HIP_TRY(s, hipGetLastError());
            HIP_TRY(s, hipMemcpyAsync(s->host_scal, L.status, sizeof(double) * ST_SIZE, hipMemcpyDeviceToHost, st));
            HIP_TRY(s, hipStreamSynchronize(st));
            incr = s->host_scal[ST_INCR];
            const int kb = (int)s->host_scal[ST_BREAK];
            kf = k;
            if (kb > 0) {
                // invariant Krylov space at kb: T_k = diag(T_kb, 0), so s_k = [s_kb; 0]
                kf = kb;
                converged = true;
                break;
            }
            if (((int)s->host_scal[ST_FLAGS]) & FLAG_NOT_SPD) {
                not_spd = true;
                break;
            }
            if (k >= 2 && incr < tol) {
                converged = true;
                break;
            }
            if (last) break;
        }
        hipLaunchKernelGGL(next_basis_kernel, dim3(g), dim3(256), 0, st, L.V + (size_t)k * ld, L.w, L.beta + (k - 1),
                           L.status, n);
    }
    hipLaunchKernelGGL((combine_out<Tio>), dim3(g), dim3(256), 0, st, L.V, ld, kf, s_final, L.status, prefactor, n,
                       3 * np, accumulate ? 1 : 0, lin, ang);
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipStreamSynchronize(st));
    if (iters_out) *iters_out = kf;
    if (incr_out) *incr_out = incr;
    if (not_spd) return fail(s, RPY_ERR_NOT_SPD, "the mobility matrix is not positive definite (negative Ritz value)");
    if (!converged)
        return fail(s, RPY_ERR_NOT_CONVERGED, "Lanczos did not reach the tolerance within max_iter iterations");
    return RPY_OK;
}

template rpy_status lanczos_run<float>(rpy_solver *, const float *, double, double, int, float *, float *, int *,
                                       double *, hipStream_t, bool);
template rpy_status lanczos_run<double>(rpy_solver *, const double *, double, double, int, double *, double *, int *,
                                        double *, hipStream_t, bool);

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

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
// The host reads a 4-double status block after each iteration to decide
// whether to stop (first k >= 2 with increment < tol; a clearly negative
// Ritz value; beta_k ~ 0 meaning the Krylov space is invariant).  The
// final y = prefactor * beta_0 V_k s_k is formed on the device and written
// in the caller's dtype.
//
// Reductions are two-stage with a fixed block count and fixed order, so the
// result does not depend on scheduling.
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace rpy {
namespace {

constexpr int kRedBlocks = 256;    // blocks of the first reduction stage
constexpr int kRedThreads = 256;
constexpr int kMaxK = 1024;        // largest tridiagonal the eigensolver takes
constexpr int kEigThreads = 256;

// status block (double): [0] beta0, [1] increment, [2] flags; the host
// copy also receives [3] beta_k and [4] alpha_k
enum { ST_BETA0 = 0, ST_INCR = 1, ST_FLAGS = 2, ST_BETAK = 3, ST_ALPHAK = 4, ST_SIZE = 4 };
enum { FLAG_NOT_SPD = 1, FLAG_NONFINITE = 2 };

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

// dst = src / (*beta)
__global__ void scale_div(double *__restrict__ dst, const double *__restrict__ src, const double *beta, int64_t n) {
    const double inv = 1.0 / (*beta);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] * inv;
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

// partial[b * k + j] = sum over block b's rows of V[j][i] w[i], j < k.
// Block b owns one contiguous slab of rows; its slice of w stays in L1/L2
// while the k basis columns stream past.
__global__ void gemv_t_partial(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ w,
                               int64_t n, double *__restrict__ partial) {
    __shared__ double sh[kRedThreads];
    int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    chunk = (chunk + blockDim.x - 1) / blockDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = std::min<int64_t>(n, i0 + chunk);
    for (int j = 0; j < k; ++j) {
        const double *col = V + (size_t)j * ld;
        double acc = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) acc = fma(col[i], w[i], acc);
        const double r = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * k + j] = r;
    }
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

// out = scale * sum_j V[j][i] s[j], written as n_lin linear entries to lin and
// the rest to ang (caller's dtype).
template <typename Tout>
__global__ void combine_out(const double *__restrict__ V, int64_t ld, int k, const double *__restrict__ s,
                            const double *__restrict__ status, double prefactor, int64_t n, int64_t n_lin,
                            Tout *__restrict__ lin, Tout *__restrict__ ang) {
    __shared__ double hs[kMaxK];
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = s[j];
    __syncthreads();
    const double scale = prefactor * status[ST_BETA0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(V[(size_t)j * ld + i], hs[j], acc);
        const Tout v = (Tout)(scale * acc);
        if (i < n_lin)
            lin[i] = v;
        else
            ang[i - n_lin] = v;
    }
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

// Eigen-decomposition of the k x k symmetric tridiagonal T (diagonal alpha,
// off-diagonal beta) by implicit QL with Wilkinson-type shifts (the
// textbook tql2 scheme), Q accumulated in global memory (row-major k x k,
// thread r owning row r).  Then s = Q sqrt(lambda) Q^T e_1 and the
// relative increment against s_prev (length k-1).  One workgroup.
__global__ void __launch_bounds__(kEigThreads)
tridiag_sqrt_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int k,
                    const double *__restrict__ s_prev, double *__restrict__ s_out, double *__restrict__ Q,
                    double *__restrict__ status) {
    __shared__ double d[kMaxK], e[kMaxK];
    __shared__ double rc[kMaxK], rs[kMaxK];
    __shared__ int sweep[3];   // l, m (rotations m-1 .. l), done flag
    __shared__ double red[kEigThreads];
    const int tid = threadIdx.x;
    for (int i = tid; i < k; i += blockDim.x) {
        d[i] = alpha[i];
        e[i] = (i + 1 < k) ? beta[i] : 0.0;
        for (int j = 0; j < k; ++j) Q[(size_t)i * k + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();

    // Thread 0 runs the scalar QL recurrences; the rotations of each sweep
    // are then applied to the rows of Q by all threads.
    int l = 0;
    int iter = 0;
    while (true) {
        if (tid == 0) {
            int m = l;
            int done = 0;
            while (l < k) {
                for (m = l; m < k - 1; ++m) {
                    const double dd = fabs(d[m]) + fabs(d[m + 1]);
                    if (fabs(e[m]) <= 2.220446049250313e-16 * dd) break;
                }
                if (m != l && iter < 60) break;
                // eigenvalue l converged (or gave up after 60 sweeps)
                ++l;
                iter = 0;
            }
            if (l >= k) {
                done = 1;
            } else {
                ++iter;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = sqrt(fma(g, g, 1.0));
                g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
                double s = 1.0, c = 1.0, p = 0.0;
                int i;
                bool underflow = false;
                for (i = m - 1; i >= l; --i) {
                    const double f = s * e[i];
                    const double b = c * e[i];
                    const double r2 = fma(f, f, g * g);
                    if (r2 == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        underflow = true;
                        break;
                    }
                    const double ri = rhyp(r2);
                    r = r2 * ri;
                    e[i + 1] = r;
                    s = f * ri;
                    c = g * ri;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    rc[i] = c;
                    rs[i] = s;
                }
                const int lo = underflow ? i + 1 : l;
                if (!underflow) {
                    d[l] -= p;
                    e[l] = g;
                    e[m] = 0.0;
                }
                sweep[0] = lo;
                sweep[1] = m;
            }
            sweep[2] = done;
        }
        __syncthreads();
        if (sweep[2]) break;
        const int lo = sweep[0], m = sweep[1];
        for (int row = tid; row < k; row += blockDim.x) {
            double *q = Q + (size_t)row * k;
            for (int i = m - 1; i >= lo; --i) {
                const double f = q[i + 1];
                q[i + 1] = rs[i] * q[i] + rc[i] * f;
                q[i] = rc[i] * q[i] - rs[i] * f;
            }
        }
        __syncthreads();
    }

    // spectrum check and square roots (eigenvalues d[j], eigenvectors = columns of Q)
    double lmax = -1e308, lmin = 1e308;
    for (int j = 0; j < k; ++j) {
        lmax = fmax(lmax, d[j]);
        lmin = fmin(lmin, d[j]);
    }
    // u_j = sqrt(max(lambda_j, 0)) * Q[0][j]
    for (int j = tid; j < k; j += blockDim.x) rc[j] = sqrt(fmax(d[j], 0.0)) * Q[j];
    __syncthreads();
    double num = 0.0, den = 0.0;
    for (int row = tid; row < k; row += blockDim.x) {
        const double *q = Q + (size_t)row * k;
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(q[j], rc[j], acc);
        s_out[row] = acc;
        const double prev = (row < k - 1) ? s_prev[row] : 0.0;
        num = fma(acc - prev, acc - prev, num);
        den = fma(acc, acc, den);
    }
    num = block_sum(num, red);
    den = block_sum(den, red);
    if (tid == 0) {
        status[ST_INCR] = (k >= 2 && den > 0.0) ? sqrt(num / den) : INFINITY;
        double flags = 0.0;
        if (lmin < -1e-10 * fmax(lmax, 0.0)) flags += FLAG_NOT_SPD;
        status[ST_FLAGS] = flags;
    }
}

struct LanczosWork {
    double *V = nullptr;
    int64_t ld = 0;
    int cap = 0;
    double *w = nullptr, *alpha = nullptr, *beta = nullptr, *h = nullptr, *red = nullptr;
    double *s = nullptr, *s_prev = nullptr, *Q = nullptr, *status = nullptr;
};

int grid_for(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

template <typename Tio>
rpy_status lanczos_run(rpy_solver *s, const Tio *w_in, double prefactor, double tol, int max_iter, Tio *lin,
                       Tio *ang, int *iters_out, double *incr_out, hipStream_t st) {
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
    HIP_TRY(s, s->lz_scal.ensure(sizeof(double) * (ST_SIZE + 6 * (size_t)(kMaxK + 1))));
    HIP_TRY(s, s->lz_red.ensure(sizeof(double) * (size_t)kRedBlocks * (kMaxK + 1)));
    HIP_TRY(s, s->lz_q.ensure(sizeof(double) * (size_t)kmax * kmax));
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
    L.red = s->lz_red.as<double>();
    L.Q = s->lz_q.as<double>();

    const bool fp32 = s->dtype == RPY_F32;
    rpy_status r = ensure_vec_buffers(s, ang_mode);
    if (r != RPY_OK) return r;

    // beta0 = |W|, v1 = W / beta0
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
        HIP_TRY(s, launch_fill_zero<Tio>(lin, 3 * np, st));
        if (ang) HIP_TRY(s, launch_fill_zero<Tio>(ang, 3 * np, st));
        return RPY_OK;
    }
    hipLaunchKernelGGL((init_basis<Tio>), dim3(grid_for(n)), dim3(256), 0, st, L.V, w_in, L.status + ST_BETA0, n);
    HIP_TRY(s, hipGetLastError());

    const int g = grid_for(n);
    int k = 0;
    double incr = INFINITY, tscale = 0.0;
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
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(gemv_t_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, L.V, ld, k, L.w, n, L.red);
            hipLaunchKernelGGL(gemv_t_final, dim3(k), dim3(kRedThreads), 0, st, L.red, kRedBlocks, k, L.h);
            hipLaunchKernelGGL(gemv_n_sub, dim3(g), dim3(256), 0, st, L.V, ld, k, L.h, L.w, n);
        }
        // beta_k = |w|
        hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, L.w, L.w, n, L.red);
        hipLaunchKernelGGL(reduce_scalar, dim3(1), dim3(kRedThreads), 0, st, L.red, kRedBlocks, L.beta + (k - 1), 1);
        // T_k eigensolve, s_k, increment
        hipLaunchKernelGGL(tridiag_sqrt_kernel, dim3(1), dim3(kEigThreads), 0, st, L.alpha, L.beta, k, L.s_prev, L.s,
                           L.Q, L.status);
        HIP_TRY(s, hipGetLastError());
        HIP_TRY(s, hipMemcpyAsync(s->host_scal, L.status, sizeof(double) * ST_SIZE, hipMemcpyDeviceToHost, st));
        HIP_TRY(s, hipMemcpyAsync(s->host_scal + ST_BETAK, L.beta + (k - 1), sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(s, hipMemcpyAsync(s->host_scal + ST_ALPHAK, L.alpha + (k - 1), sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(s, hipStreamSynchronize(st));
        incr = s->host_scal[ST_INCR];
        const double flags = s->host_scal[ST_FLAGS];
        const double betak = s->host_scal[ST_BETAK];
        tscale = std::max({tscale, std::fabs(s->host_scal[ST_ALPHAK]), betak});
        if (((int)flags) & FLAG_NOT_SPD) {
            not_spd = true;
            break;
        }
        if (k >= 2 && incr < tol) {
            converged = true;
            break;
        }
        // breakdown: the Krylov space is (numerically) invariant, y_k is exact
        if (!(betak > 1e-14 * tscale) || k == n) {
            converged = true;
            break;
        }
        if (k == kmax) break;
        // scale for the next basis vector; remember s_k
        hipLaunchKernelGGL(scale_div, dim3(g), dim3(256), 0, st, L.V + (size_t)k * ld, L.w, L.beta + (k - 1), n);
        HIP_TRY(s, hipMemcpyAsync(L.s_prev, L.s, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
    }
    const int kf = std::min(k, kmax);
    hipLaunchKernelGGL((combine_out<Tio>), dim3(g), dim3(256), 0, st, L.V, ld, kf, L.s, L.status, prefactor, n,
                       3 * np, lin, ang);
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
                                       double *, hipStream_t);
template rpy_status lanczos_run<double>(rpy_solver *, const double *, double, double, int, double *, double *, int *,
                                        double *, hipStream_t);

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
                                   incr_out, st);
    return lanczos_run<float>(s, static_cast<const float *>(w), prefactor, tol, max_iter, static_cast<float *>(lin_out),
                              static_cast<float *>(ang_out), iters_out, incr_out, st);
}

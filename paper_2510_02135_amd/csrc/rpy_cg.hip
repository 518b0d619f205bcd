// Conjugate gradients on the mobility matrix: a Krylov consumer of the
// product (Sec. 3.3 builds its square root from products alone; the same
// products drive a linear solve).  For nrhs right-hand sides [U_r; Omega_r]
// it finds [F_r; T_r] with M [F_r; T_r] = [U_r; Omega_r], i.e. the forces
// (and torques) that produce prescribed velocities.  M is symmetric positive
// definite, so plain CG applies (GMRES would too, at more memory).
//
// Every vector operation is float64 on the device; the products use the
// solver's pair precision (one multi-vector product for all unconverged
// right-hand sides per iteration).  Per iteration and right-hand side:
//   q = M p;  alpha = (r.r) / (p.q);  x += alpha p;  r -= alpha q;
//   beta = (r.r)_new / (r.r);  p = r + beta p,
// stopping at the first iteration with |r| / |b| < tol (the recursive
// residual).  Reductions are two-stage with a fixed block count (the result
// does not depend on scheduling).
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace rpy {
namespace {

constexpr int kCgBlocks = 256;
constexpr int kCgThreads = 256;

// scalar block per right-hand side: r.r, p.q, b.b, r.r after the update
enum { CG_RR = 0, CG_PQ = 1, CG_BB = 2, CG_RRN = 3, CG_SIZE = 4 };

// x = 0, r = p = b; partial sums of b.b.  b: linear entries from ul (3N),
// then angular ones from ua.
template <typename Tin>
__global__ void __launch_bounds__(kCgThreads)
cg_init(const Tin *__restrict__ ul, const Tin *__restrict__ ua, int64_t n3, int64_t n, double *__restrict__ x,
        double *__restrict__ r, double *__restrict__ p, double *__restrict__ partial) {
    __shared__ double sh[kCgThreads];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double v = e < n3 ? (double)ul[e] : (double)ua[e - n3];
        x[e] = 0.0;
        r[e] = v;
        p[e] = v;
        acc = fma(v, v, acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// partial sums of a.b
__global__ void __launch_bounds__(kCgThreads)
cg_dot(const double *__restrict__ a, const double *__restrict__ b, int64_t n, double *__restrict__ partial) {
    __shared__ double sh[kCgThreads];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        acc = fma(a[e], b[e], acc);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// scal[dst] = sum of the partials (also scal[dst2] when dst2 >= 0); with
// `shift`, scal[CG_RR] = scal[CG_RRN] first (the previous iteration's new
// r.r becomes the current one; p was already updated with both).
__global__ void __launch_bounds__(kCgThreads)
cg_reduce(const double *__restrict__ partial, int nb, double *__restrict__ scal, int dst, int dst2, int shift) {
    __shared__ double sh[kCgThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        if (shift) scal[CG_RR] = scal[CG_RRN];
        scal[dst] = s;
        if (dst2 >= 0) scal[dst2] = s;
    }
}

// alpha = r.r / p.q (0 when p.q is not positive: the host then reports an
// indefinite matrix and leaves x as it was); x += alpha p; r -= alpha q;
// partial sums of the new r.r
__global__ void __launch_bounds__(kCgThreads)
cg_update(const double *__restrict__ scal, const double *__restrict__ p, const double *__restrict__ q, int64_t n,
          double *__restrict__ x, double *__restrict__ r, double *__restrict__ partial) {
    __shared__ double sh[kCgThreads];
    const double pq = scal[CG_PQ];
    const double alpha = pq > 0.0 ? scal[CG_RR] / pq : 0.0;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        x[e] = fma(alpha, p[e], x[e]);
        const double re = fma(-alpha, q[e], r[e]);
        r[e] = re;
        acc = fma(re, re, acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// p = r + beta p with beta = (r.r)_new / (r.r)
__global__ void __launch_bounds__(kCgThreads)
cg_direction(const double *__restrict__ scal, const double *__restrict__ r, int64_t n, double *__restrict__ p) {
    const double beta = scal[CG_RRN] / scal[CG_RR];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = fma(beta, p[e], r[e]);
}

// x (float64, linear then angular entries) to the caller's arrays
template <typename Tout>
__global__ void cg_store(const double *__restrict__ x, int64_t n3, int64_t n, Tout *__restrict__ fl,
                         Tout *__restrict__ fa) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < n3)
            fl[e] = (Tout)x[e];
        else
            fa[e - n3] = (Tout)x[e];
    }
}

int cg_grid(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + 255) / 256)); }

struct CgRhs {
    double *x, *r, *p, *scal;
    int iters = 0;
    double resid = 0.0;
    bool done = false, converged = false, not_spd = false;
};

// q_j = M p for the listed right-hand sides (slot j of Q, stride ld)
template <typename Real>
rpy_status cg_products(rpy_solver *s, const std::vector<CgRhs *> &act, int64_t ld, double *Q, hipStream_t st) {
    const int64_t np = s->n;
    const bool am = s->angular;
    const int m = (int)act.size();
    const size_t elt = sizeof(vec4_t<Real>);
    HIP_TRY(s, s->f.ensure(elt * (size_t)m * np));
    if (am) HIP_TRY(s, s->t.ensure(elt * (size_t)m * np));
    for (int j = 0; j < m; ++j) {
        const double *v = act[j]->p;
        HIP_TRY(s, (launch_stage_vec<double, Real>(v, np, s->f.as<vec4_t<Real>>() + (size_t)j * np, st)));
        if (am) HIP_TRY(s, (launch_stage_vec<double, Real>(v + 3 * np, np, s->t.as<vec4_t<Real>>() + (size_t)j * np, st)));
    }
    if (m == 1) return apply_staged<Real, double>(s, am, Q, am ? Q + 3 * np : nullptr, st);
    return apply_staged_multi<Real, double>(s, am, m, Q, am ? Q + 3 * np : nullptr, ld, st);
}

template <typename Tio>
rpy_status cg_run(rpy_solver *s, const Tio *ul, const Tio *ua, int nrhs, double tol, int max_iter, Tio *fl, Tio *fa,
                  int *iters_out, double *resid_out, hipStream_t st) {
    const bool am = s->angular;
    const int64_t np = s->n, n3 = 3 * np;
    const int64_t n = (am ? 6 : 3) * np;
    const int64_t ld = (n + 63) / 64 * 64;
    // workspace: x, r, p per right-hand side, one product slot each, scalars
    HIP_TRY(s, s->cg_vec.ensure(sizeof(double) * (size_t)nrhs * 4 * ld));
    HIP_TRY(s, s->cg_scal.ensure(sizeof(double) * ((size_t)nrhs * CG_SIZE + kCgBlocks)));
    if (s->host_stat_cap < (size_t)nrhs * CG_SIZE) {
        if (s->host_stat) (void)hipHostFree(s->host_stat);
        s->host_stat = nullptr;
        s->host_stat_cap = 0;
        HIP_TRY(s, hipHostMalloc((void **)&s->host_stat, sizeof(double) * (size_t)nrhs * CG_SIZE,
                                 hipHostMallocDefault));
        s->host_stat_cap = (size_t)nrhs * CG_SIZE;
    }
    rpy_status rs = ensure_vec_buffers(s, am);
    if (rs != RPY_OK) return rs;
    double *const V = s->cg_vec.as<double>();
    double *const Q = V + (size_t)nrhs * 3 * ld;
    double *const scal_all = s->cg_scal.as<double>();
    double *const partial = scal_all + (size_t)nrhs * CG_SIZE;
    double *const hs = s->host_stat;
    std::vector<CgRhs> rhs(nrhs);
    const int g = cg_grid(n);
    for (int q = 0; q < nrhs; ++q) {
        CgRhs &R = rhs[q];
        R.x = V + (size_t)(3 * q) * ld;
        R.r = R.x + ld;
        R.p = R.r + ld;
        R.scal = scal_all + (size_t)q * CG_SIZE;
        hipLaunchKernelGGL((cg_init<Tio>), dim3(kCgBlocks), dim3(kCgThreads), 0, st, ul + q * n3,
                           ua ? ua + q * n3 : nullptr, n3, n, R.x, R.r, R.p, partial);
        hipLaunchKernelGGL(cg_reduce, dim3(1), dim3(kCgThreads), 0, st, partial, kCgBlocks, R.scal, (int)CG_BB,
                           (int)CG_RR, 0);
    }
    HIP_TRY(s, hipGetLastError());
    auto copy_scal = [&]() -> rpy_status {
        HIP_TRY(s, hipMemcpyAsync(hs, scal_all, sizeof(double) * (size_t)nrhs * CG_SIZE, hipMemcpyDeviceToHost, st));
        HIP_TRY(s, hipStreamSynchronize(st));
        return RPY_OK;
    };
    if ((rs = copy_scal()) != RPY_OK) return rs;
    for (int q = 0; q < nrhs; ++q) {
        const double bb = hs[(size_t)q * CG_SIZE + CG_BB];
        if (!std::isfinite(bb))
            return fail(s, RPY_ERR_NONFINITE, "right-hand side " + std::to_string(q) + " is not finite");
        if (bb == 0.0) rhs[q].done = rhs[q].converged = true;   // x = 0
    }
    const bool fp32 = s->dtype == RPY_F32;
    std::vector<CgRhs *> act;
    for (int k = 1; k <= max_iter; ++k) {
        act.clear();
        for (auto &R : rhs)
            if (!R.done) act.push_back(&R);
        if (act.empty()) break;
        rs = fp32 ? cg_products<float>(s, act, ld, Q, st) : cg_products<double>(s, act, ld, Q, st);
        if (rs != RPY_OK) return rs;
        for (size_t j = 0; j < act.size(); ++j) {
            CgRhs &R = *act[j];
            const double *q = Q + j * ld;
            hipLaunchKernelGGL(cg_dot, dim3(kCgBlocks), dim3(kCgThreads), 0, st, R.p, q, n, partial);
            hipLaunchKernelGGL(cg_reduce, dim3(1), dim3(kCgThreads), 0, st, partial, kCgBlocks, R.scal, (int)CG_PQ,
                               -1, k > 1 ? 1 : 0);
            hipLaunchKernelGGL(cg_update, dim3(kCgBlocks), dim3(kCgThreads), 0, st, R.scal, R.p, q, n, R.x, R.r,
                               partial);
            hipLaunchKernelGGL(cg_reduce, dim3(1), dim3(kCgThreads), 0, st, partial, kCgBlocks, R.scal, (int)CG_RRN,
                               -1, 0);
        }
        HIP_TRY(s, hipGetLastError());
        if ((rs = copy_scal()) != RPY_OK) return rs;
        for (CgRhs *R : act) {
            const double *h = hs + (R->scal - scal_all);
            R->iters = k;
            if (!(h[CG_PQ] > 0.0)) {   // p^T M p <= 0 (or NaN): M is not positive definite
                R->not_spd = R->done = true;
                R->resid = std::sqrt(h[CG_RR] / h[CG_BB]);
                continue;
            }
            R->resid = std::sqrt(h[CG_RRN] / h[CG_BB]);
            if (R->resid < tol) R->converged = R->done = true;
            else if (k == max_iter) R->done = true;
        }
        for (CgRhs *R : act)
            if (!R->done)
                hipLaunchKernelGGL(cg_direction, dim3(g), dim3(256), 0, st, R->scal, R->r, n, R->p);
        HIP_TRY(s, hipGetLastError());
    }
    bool any_not_spd = false, any_not_conv = false;
    for (int q = 0; q < nrhs; ++q) {
        const CgRhs &R = rhs[q];
        hipLaunchKernelGGL((cg_store<Tio>), dim3(g), dim3(256), 0, st, R.x, n3, n, fl + q * n3,
                           fa ? fa + q * n3 : nullptr);
        if (iters_out) iters_out[q] = R.iters;
        if (resid_out) resid_out[q] = R.resid;
        any_not_spd |= R.not_spd;
        any_not_conv |= !R.converged && !R.not_spd;
    }
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipStreamSynchronize(st));
    if (any_not_spd) return fail(s, RPY_ERR_NOT_SPD, "conjugate gradients met p^T M p <= 0 (M not positive definite)");
    if (any_not_conv)
        return fail(s, RPY_ERR_NOT_CONVERGED, "conjugate gradients did not reach the tolerance within max_iter");
    return RPY_OK;
}

}  // namespace
}  // namespace rpy

using namespace rpy;

extern "C" rpy_status rpy_mobility_solve(rpy_solver *s, const void *u_lin, const void *u_ang, int nrhs, double tol,
                                         int max_iter, void *f_out, void *t_out, int *iters_out, double *resid_out,
                                         void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(s, RPY_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    if (!u_lin || !f_out) return fail(s, RPY_ERR_INVALID_ARG, "the linear velocities and forces must not be NULL");
    if (s->angular && (!u_ang || !t_out))
        return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs angular velocities and the torque output");
    if (!s->angular && (u_ang || t_out))
        return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular velocities / torques need include_angular");
    if (!(tol > 0.0 && tol < 1.0)) return fail(s, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(s, RPY_ERR_INVALID_ARG, "max_iter must be >= 1");
    if ((int64_t)nrhs * s->n > (int64_t)INT32_MAX)
        return fail(s, RPY_ERR_INVALID_ARG, "nrhs * n must stay below 2^31");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return cg_run<double>(s, static_cast<const double *>(u_lin), static_cast<const double *>(u_ang), nrhs, tol,
                              max_iter, static_cast<double *>(f_out), static_cast<double *>(t_out), iters_out,
                              resid_out, st);
    return cg_run<float>(s, static_cast<const float *>(u_lin), static_cast<const float *>(u_ang), nrhs, tol, max_iter,
                         static_cast<float *>(f_out), static_cast<float *>(t_out), iters_out, resid_out, st);
}

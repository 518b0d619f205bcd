// Time stepping of eq. (bdhi) on top of the solver's products.
//
// rpy_langevin_velocities (Sec. 3.2, LangevinVelocities): the Euler-Maruyama
// velocities
//   [U; Omega] = M [F; T] + sqrt(2 kBT / dt) M^{1/2} W + kBT d_X . M,
// i.e. X^{n+1} = X^n + dt U is one Euler-Maruyama step of eq. (bdhi).
//
// rpy_ab2_step (the stochastic Adams-Bashforth scheme of Sec. 5.1):
//   X^{n+1} = X^n + dt [ 3/2 u^n - 1/2 u^{n-1} ] + sqrt(2 kBT dt) (M^n)^{1/2} W^n,
//   u^n = M^n [F^n; T^n] + kBT (d_X . M)^n,
// with the angular rows giving the rotation increment.  The caller keeps
// u^{n-1} in a history buffer that the step overwrites with u^n; the first
// step (no history) takes the Euler-Maruyama step (coefficients 1 and 0).
//
// In open space d_X . M = 0, so u = M [F; T].  The noise goes through the
// Lanczos solver (written straight into the outputs), the deterministic part
// is reduced into float64, and one elementwise kernel forms the update and
// rounds once to the solver's dtype.
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <cmath>

namespace rpy {
namespace {

// out_lin[e] = x[e] + dt (c1 u[e] - c0 h[e]) + noise[e]   (e < 3N; noise in out_lin)
// out_ang[e] = dt (c1 u[3N+e] - c0 h[3N+e]) + noise[e]     (noise in out_ang)
// h[e] = u[e]                                               (all entries)
template <typename Real>
__global__ void ab2_update_kernel(const vec4_t<Real> *__restrict__ pos, const double *__restrict__ u,
                                  Real *__restrict__ hist, int64_t n3, int nv_mult, double dt, double c1, double c0,
                                  int have_noise, Real *__restrict__ out_lin, Real *__restrict__ out_ang) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3 * nv_mult) return;
    const double ue = u[e];
    const double he = c0 != 0.0 ? (double)hist[e] : 0.0;
    const double det = dt * (c1 * ue - c0 * he);
    if (e < n3) {
        const vec4_t<Real> x = pos[e / 3];
        const int c = (int)(e % 3);
        const double xe = (double)(c == 0 ? x.x : (c == 1 ? x.y : x.z));
        const double nz = have_noise ? (double)out_lin[e] : 0.0;
        out_lin[e] = (Real)(xe + det + nz);
    } else {
        const double nz = have_noise ? (double)out_ang[e - n3] : 0.0;
        out_ang[e - n3] = (Real)(det + nz);
    }
    hist[e] = (Real)ue;
}

template <typename Real>
rpy_status stage_forces(rpy_solver *s, const Real *F, const Real *T, bool am, hipStream_t st) {
    rpy_status r = ensure_vec_buffers(s, am);
    if (r != RPY_OK) return r;
    HIP_TRY(s, (launch_stage_vec<Real, Real>(F, s->n, s->f.as<vec4_t<Real>>(), st)));
    if (am) HIP_TRY(s, (launch_stage_vec<Real, Real>(T, s->n, s->t.as<vec4_t<Real>>(), st)));
    return RPY_OK;
}

template <typename Real>
rpy_status langevin_typed(rpy_solver *s, const Real *F, const Real *T, const Real *w, double dt, double kbt,
                          double tol, int max_iter, Real *lin, Real *ang, int *iters_out, hipStream_t st) {
    const bool am = s->angular;
    if (iters_out) *iters_out = 0;
    // deterministic part (zero without forces and torques)
    if (F || T) {
        rpy_status r = stage_forces<Real>(s, F, T, am, st);
        if (r != RPY_OK) return r;
        r = apply_staged<Real, Real>(s, am, lin, ang, st);
        if (r != RPY_OK) return r;
    } else {
        HIP_TRY(s, launch_fill_zero<Real>(lin, 3 * s->n, st));
        if (ang) HIP_TRY(s, launch_fill_zero<Real>(ang, 3 * s->n, st));
    }
    // + kBT d_X . M: zero in open space
    // + sqrt(2 kBT / dt) M^{1/2} W
    if (kbt > 0.0)
        return lanczos_run<Real>(s, w, std::sqrt(2.0 * kbt / dt), tol, max_iter, lin, ang, iters_out, nullptr, st,
                                 true);
    return RPY_OK;
}

template <typename Real>
rpy_status ab2_typed(rpy_solver *s, const Real *F, const Real *T, const Real *w, double dt, double kbt, double tol,
                     int max_iter, Real *hist, bool have_hist, Real *pos_out, Real *ang_out, int *iters_out,
                     hipStream_t st) {
    const bool am = s->angular;
    const int64_t n3 = 3 * s->n;
    const int mult = am ? 2 : 1;
    if (iters_out) *iters_out = 0;
    // noise sqrt(2 kBT dt) M^{1/2} W, written into the outputs
    rpy_status r = RPY_OK;
    if (kbt > 0.0) {
        r = lanczos_run<Real>(s, w, std::sqrt(2.0 * kbt * dt), tol, max_iter, pos_out, ang_out, iters_out, nullptr,
                              st, false);
        if (r != RPY_OK && r != RPY_ERR_NOT_CONVERGED) return r;
    }
    const rpy_status noise_status = r;
    // u^n = M [F; T] in float64 (the drift term is zero in open space)
    HIP_TRY(s, s->drift.ensure(sizeof(double) * (size_t)n3 * mult));
    double *u = s->drift.as<double>();
    if (F || T) {
        r = stage_forces<Real>(s, F, T, am, st);
        if (r != RPY_OK) return r;
        r = apply_staged<Real, double>(s, am, u, am ? u + n3 : nullptr, st);
        if (r != RPY_OK) return r;
    } else {
        HIP_TRY(s, launch_fill_zero<double>(u, n3 * mult, st));
    }
    const double c1 = have_hist ? 1.5 : 1.0, c0 = have_hist ? 0.5 : 0.0;
    hipLaunchKernelGGL((ab2_update_kernel<Real>), dim3((unsigned)((n3 * mult + 255) / 256)), dim3(256), 0, st,
                       s->pos.as<vec4_t<Real>>(), u, hist, n3, mult, dt, c1, c0, kbt > 0.0 ? 1 : 0, pos_out,
                       ang_out);
    HIP_TRY(s, hipGetLastError());
    return noise_status;
}

rpy_status check_step_args(rpy_solver *s, const void *w, double dt, double kbt, double tol, int max_iter) {
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(s, RPY_ERR_INVALID_ARG, "dt must be positive and finite");
    if (!(kbt >= 0.0) || !std::isfinite(kbt)) return fail(s, RPY_ERR_INVALID_ARG, "kbt must be >= 0 and finite");
    if (kbt > 0.0) {
        if (s->wall)
            return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY,
                        "kbt > 0 above a wall needs the thermal drift, which this step does not include");
        if (!w) return fail(s, RPY_ERR_INVALID_ARG, "kbt > 0 needs the noise vector W");
        if (!(tol > 0.0 && tol < 1.0)) return fail(s, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
        if (max_iter < 1) return fail(s, RPY_ERR_INVALID_ARG, "max_iter must be >= 1");
    }
    return RPY_OK;
}

}  // namespace
}  // namespace rpy

using namespace rpy;

extern "C" {

rpy_status rpy_langevin_velocities(rpy_solver *s, const void *forces, const void *torques, const void *w, double dt,
                                   double kbt, double tol, int max_iter, void *lin_out, void *ang_out, int *iters_out,
                                   void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!lin_out) return fail(s, RPY_ERR_INVALID_ARG, "linear output pointer is NULL");
    if (torques && !s->angular) return fail(s, RPY_ERR_ANGULAR_DISABLED, "torques need include_angular");
    if (s->angular && !ang_out) return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!s->angular && ang_out) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    r = check_step_args(s, w, dt, kbt, tol, max_iter);
    if (r != RPY_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return langevin_typed<double>(s, static_cast<const double *>(forces), static_cast<const double *>(torques),
                                      static_cast<const double *>(w), dt, kbt, tol, max_iter,
                                      static_cast<double *>(lin_out), static_cast<double *>(ang_out), iters_out, st);
    return langevin_typed<float>(s, static_cast<const float *>(forces), static_cast<const float *>(torques),
                                 static_cast<const float *>(w), dt, kbt, tol, max_iter, static_cast<float *>(lin_out),
                                 static_cast<float *>(ang_out), iters_out, st);
}

rpy_status rpy_ab2_step(rpy_solver *s, const void *forces, const void *torques, const void *w, double dt, double kbt,
                        double tol, int max_iter, void *history, int have_history, void *pos_out, void *ang_out,
                        int *iters_out, void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!pos_out || !history) return fail(s, RPY_ERR_INVALID_ARG, "pos_out and history must not be NULL");
    if (torques && !s->angular) return fail(s, RPY_ERR_ANGULAR_DISABLED, "torques need include_angular");
    if (s->angular && !ang_out) return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!s->angular && ang_out) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    r = check_step_args(s, w, dt, kbt, tol, max_iter);
    if (r != RPY_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return ab2_typed<double>(s, static_cast<const double *>(forces), static_cast<const double *>(torques),
                                 static_cast<const double *>(w), dt, kbt, tol, max_iter, static_cast<double *>(history),
                                 have_history != 0, static_cast<double *>(pos_out), static_cast<double *>(ang_out),
                                 iters_out, st);
    return ab2_typed<float>(s, static_cast<const float *>(forces), static_cast<const float *>(torques),
                            static_cast<const float *>(w), dt, kbt, tol, max_iter, static_cast<float *>(history),
                            have_history != 0, static_cast<float *>(pos_out), static_cast<float *>(ang_out), iters_out,
                            st);
}

}  // extern "C"

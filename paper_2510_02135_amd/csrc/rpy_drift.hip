// Thermal drift by random finite differences (eq. (rfd), Sec. 3.4).
//
// One sample is
//   (1/delta) [ M(X + delta/2 W_X) W - M(X - delta/2 W_X) W ]
// for a caller-supplied W (3N entries, or 6N with the angular blocks, linear
// first, as for sqrtMdotW).  Only the positional part W_X displaces the
// particles: orientation does not enter M for spheres, so d_theta . M = 0.
// The average over W ~ N(0, I) is d_X . M up to O(delta^2); in open space
// that is zero, which makes the routine a check of the solver rather than a
// correction, and the building block for geometries where it is not.
//
// Both products run through the ordinary pair kernel on displaced copies of
// the stored positions; they are reduced into float64 so that the
// difference and the division by delta lose nothing beyond the products'
// own rounding, and rounded once to the caller's dtype.
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <cmath>

namespace rpy {
namespace {

// plus/minus = X +- (delta/2) W_X, formed in float64 as written (no fused
// multiply-add, so the rounding is that of the two separate operations) and
// rounded once to the solver's precision.
template <typename Real>
__global__ void rfd_displace_kernel(const vec4_t<Real> *__restrict__ pos, const Real *__restrict__ w, int n,
                                    double half_delta, vec4_t<Real> *__restrict__ plus,
                                    vec4_t<Real> *__restrict__ minus) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const vec4_t<Real> x = pos[i];
    const double sx = half_delta * (double)w[3 * (size_t)i];
    const double sy = half_delta * (double)w[3 * (size_t)i + 1];
    const double sz = half_delta * (double)w[3 * (size_t)i + 2];
    vec4_t<Real> p, m;
    p.x = (Real)((double)x.x + sx);
    p.y = (Real)((double)x.y + sy);
    p.z = (Real)((double)x.z + sz);
    m.x = (Real)((double)x.x - sx);
    m.y = (Real)((double)x.y - sy);
    m.z = (Real)((double)x.z - sz);
    p.w = m.w = Real(0);
    plus[i] = p;
    minus[i] = m;
}

// out[i] = (Tout)((up[i] - um[i]) / delta) for the n_lin linear entries and
// the angular ones after them
template <typename Tout>
__global__ void rfd_combine_kernel(const double *__restrict__ up, const double *__restrict__ um, int64_t n,
                                   int64_t n_lin, double delta, Tout *__restrict__ lin, Tout *__restrict__ ang) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = (up[i] - um[i]) / delta;
    if (i < n_lin)
        lin[i] = (Tout)v;
    else
        ang[i - n_lin] = (Tout)v;
}

template <typename Real>
rpy_status rfd_typed(rpy_solver *s, const Real *w, double delta, Real *lin, Real *ang, hipStream_t st) {
    const bool am = s->angular;
    const int64_t n = s->n;
    const int64_t nv = (am ? 6 : 3) * n;
    rpy_status r = ensure_vec_buffers(s, am);
    if (r != RPY_OK) return r;
    // displaced positions and the two float64 products
    const size_t pos_bytes = sizeof(vec4_t<Real>) * (size_t)n;
    HIP_TRY(s, s->drift.ensure(2 * pos_bytes + 2 * sizeof(double) * (size_t)nv));
    auto *plus = s->drift.as<vec4_t<Real>>();
    auto *minus = plus + n;
    double *up = reinterpret_cast<double *>(s->drift.as<char>() + 2 * pos_bytes);
    double *um = up + nv;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((rfd_displace_kernel<Real>), dim3(grid), dim3(256), 0, st, s->pos.as<vec4_t<Real>>(), w,
                       (int)n, 0.5 * delta, plus, minus);
    HIP_TRY(s, hipGetLastError());
    // W as the source vector: forces = W_X, torques = W_theta
    HIP_TRY(s, (launch_stage_vec<Real, Real>(w, n, s->f.as<vec4_t<Real>>(), st)));
    if (am) HIP_TRY(s, (launch_stage_vec<Real, Real>(w + 3 * n, n, s->t.as<vec4_t<Real>>(), st)));
    r = apply_staged<Real, double>(s, am, up, am ? up + 3 * n : nullptr, st, plus);
    if (r != RPY_OK) return r;
    r = apply_staged<Real, double>(s, am, um, am ? um + 3 * n : nullptr, st, minus);
    if (r != RPY_OK) return r;
    hipLaunchKernelGGL((rfd_combine_kernel<Real>), dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, up, um, nv,
                       3 * n, delta, lin, ang);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

}  // namespace
}  // namespace rpy

using namespace rpy;

extern "C" rpy_status rpy_div_m_rfd(rpy_solver *s, const void *w, double delta, void *lin_out, void *ang_out,
                                    void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!w || !lin_out) return fail(s, RPY_ERR_INVALID_ARG, "W and the linear output must not be NULL");
    if (s->angular && !ang_out) return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!s->angular && ang_out) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(s, RPY_ERR_INVALID_ARG, "delta must be positive and finite");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return rfd_typed<double>(s, static_cast<const double *>(w), delta, static_cast<double *>(lin_out),
                                 static_cast<double *>(ang_out), st);
    return rfd_typed<float>(s, static_cast<const float *>(w), delta, static_cast<float *>(lin_out),
                            static_cast<float *>(ang_out), st);
}

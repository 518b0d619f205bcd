// Host-side helpers shared by the C interface translation units.
#pragma once

#include <string>

#include "rpy_internal.hpp"

namespace rpy {

rpy_status fail(rpy_solver *s, rpy_status code, const std::string &msg);
rpy_status hip_fail(rpy_solver *s, hipError_t e, const char *what);
rpy_status check_ready(rpy_solver *s);
rpy_status ensure_vec_buffers(rpy_solver *s, bool ang);
double k_factor(const rpy_solver *s);
int splits_for(const rpy_solver *s, bool ang);

// Launch timing: returns the event to record before (after) a launch of
// kernel class `kind`, or nullptr when timing is off.
hipEvent_t timing_begin(rpy_solver *s, int kind, double pairs);
hipEvent_t timing_end(rpy_solver *s, int kind);

// M [F; T] with F (and T) already staged in s->f (s->t); Real is the pair
// precision, Tout the output element type.  ang_out may be NULL.  `pos`
// replaces the stored positions when not NULL (vec4_t<Real>, N entries).
template <typename Real, typename Tout>
rpy_status apply_staged(rpy_solver *s, bool ang, Tout *lin, Tout *ang_out, hipStream_t st,
                        const void *pos = nullptr);

// M [F; T] by the fused small-N kernel (tile mode 3, rpy_fused.hip): forces
// f and torques t (either may be NULL) with `stride` Reals per particle (3
// for the caller's N x 3 arrays, 4 for staged vec4 records); outputs as
// apply_staged (ang_out may be NULL).
template <typename Real, typename Tout>
rpy_status apply_fused(rpy_solver *s, bool ang, const Real *f, const Real *t, int stride, Tout *lin, Tout *ang_out,
                       hipStream_t st, const void *pos = nullptr);

// M [F; T] above the wall of a single_wall solver (rpy_wall.hip), with the
// staged vectors f (and t) given explicitly; otherwise as apply_staged.
template <typename Real, typename Tout>
rpy_status apply_wall(rpy_solver *s, bool ang, const vec4_t<Real> *f, const vec4_t<Real> *t, Tout *lin,
                      Tout *ang_out, hipStream_t st, const void *pos = nullptr);
int wall_targets_per_lane(const rpy_solver *s, bool ang);

// M F for the triply periodic geometry (rpy_pse.hip): F staged as vec4 at
// f, lin (n x 3) overwritten; positions `pos` (vec4) or the stored ones.
// While PseState::real_only is set, the real-space part alone.
template <typename Real, typename Tout>
rpy_status apply_pse(rpy_solver *s, const vec4_t<Real> *f, Tout *lin, hipStream_t st, const void *pos = nullptr);
rpy_status pse_create(rpy_solver *s);
void pse_release(rpy_solver *s);
rpy_status pse_set_parameter(rpy_solver *s, const char *key, double value);

// M [F; T] by the symmetric pair kernel (each unordered pair once), with
// F, T staged as for apply_staged; `span` source blocks per task (0 =
// automatic).  Large N runs in slabs of target blocks whose partials fit a
// fixed workspace.  sym_max_n() is the largest N for which the autotuner
// times the mode.  Defined in rpy_sym.hip.
template <typename Real, typename Tout>
rpy_status apply_sym(rpy_solver *s, bool ang, int span, Tout *lin, Tout *ang_out, hipStream_t st,
                     const void *pos = nullptr);
int64_t sym_max_n();
// The adjoint by the symmetric mode (rpy_sym.hip): staged vec4 F, g_U (,
// T, g_W); outputs as rpy_mdot_backward's (each may be NULL).
template <typename Real>
rpy_status adjoint_sym(rpy_solver *s, bool ang, const vec4_t<Real> *f, const vec4_t<Real> *g, const vec4_t<Real> *t,
                       const vec4_t<Real> *h, Real *gp, Real *gf, Real *gt, hipStream_t st);

// nrhs products M [F_r; T_r] with the vectors staged in s->f (s->t) as
// [vector][n] vec4 arrays (stage_multi); vector r's outputs are the n x 3
// arrays at lin + r * ostride and ang_out + r * ostride.  Defined in
// rpy_multi.hip.
template <typename Real, typename Tout>
rpy_status apply_staged_multi(rpy_solver *s, bool ang, int nrhs, Tout *lin, Tout *ang_out, int64_t ostride,
                              hipStream_t st);
template <typename Real>
rpy_status stage_multi(rpy_solver *s, const Real *F, const Real *T, int nrhs, bool ang, hipStream_t st);

// prefactor * M^{1/2} W by Lanczos for the stored positions (W and the
// outputs in the solver's dtype Tio); with `accumulate` the result is added
// to lin/ang instead of overwriting them.  Synchronises `st`.
template <typename Tio>
rpy_status lanczos_run(rpy_solver *s, const Tio *w_in, double prefactor, double tol, int max_iter, Tio *lin,
                       Tio *ang, int *iters_out, double *incr_out, hipStream_t st, bool accumulate);

// nrhs recurrences of lanczos_run with one geometry, in lockstep: W_r at
// w_in + r * wstride, outputs at lin / ang + r * ostride, iters_out and
// incr_out (host, nrhs entries, may be NULL).  Every recurrence stops and
// ends as it would alone.
// With `pre` (nrhs = 1) the iteration runs on the preconditioned operator
// L^{-1} M L^{-T} of precond_setup and the result is prefactor * L z.
template <typename Tio>
rpy_status lanczos_run_multi(rpy_solver *s, const Tio *w_in, int nrhs, int64_t wstride, double prefactor,
                             double tol, int max_iter, Tio *lin, Tio *ang, int64_t ostride, int *iters_out,
                             double *incr_out, hipStream_t st, bool accumulate, bool pre = false);

// Block-diagonal Lanczos preconditioner (rpy_precond.hip): setup for groups
// of `group` consecutive particles at the stored positions (cached until
// they change), out = L^{-T} v, w = L^{-1} w, and outputs = prefactor L z
// (+ outputs when accumulating); vectors of 3N (6N) float64 entries.
rpy_status precond_setup(rpy_solver *s, int64_t group, hipStream_t st);
rpy_status precond_solve_lt(rpy_solver *s, const double *v, double *out, hipStream_t st);
rpy_status precond_solve_l(rpy_solver *s, double *w, hipStream_t st);
template <typename Tout>
rpy_status precond_mul_l(rpy_solver *s, const double *z, double prefactor, bool accumulate, Tout *lin, Tout *ang,
                         hipStream_t st);
void precond_release(rpy_solver *s);

}  // namespace rpy

#define HIP_TRY(s, expr)                                                   \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) return ::rpy::hip_fail((s), e_, #expr);      \
    } while (0)

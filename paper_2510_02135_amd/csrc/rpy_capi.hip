// C interface of librpy: argument checking, buffer management and launch
// sequencing around the kernels.  See include/rpy.h for the contract.
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

using namespace rpy;

namespace rpy {

rpy_status fail(rpy_solver *s, rpy_status code, const std::string &msg) {
    if (s) s->err = msg;
    return code;
}

rpy_status hip_fail(rpy_solver *s, hipError_t e, const char *what) {
    std::string m = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
    if (s) s->err = m;
    return e == hipErrorOutOfMemory ? RPY_ERR_OUT_OF_MEMORY : RPY_ERR_HIP;
}

double k_factor(const rpy_solver *s) { return 1.0 / (8.0 * M_PI * s->eta); }

int splits_for(const rpy_solver *s, bool ang) {
    const TileConfig &c = s->cfg[ang ? 1 : 0];
    // in the symmetric and fused modes n_split is not a split count; other
    // kernels that share the split layout (multi-vector products) then choose
    // their own
    if (c.tm == 0 || c.tm == 3) return choose_splits(s->n, 2, s->dtype == RPY_F64, ang);
    if (c.n_split > 0) return std::min(c.n_split, max_splits(s->n));
    return choose_splits(s->n, c.tm, s->dtype == RPY_F64, ang);
}

// M [F; T] for the stored positions with F, T already staged in s->f / s->t.
// Output type Tout: the caller's dtype, or double for Lanczos products.
template <typename Real, typename Tout>
rpy_status apply_staged(rpy_solver *s, bool ang, Tout *lin, Tout *angout, hipStream_t st, const void *pos_in) {
    if (s->pse) return apply_pse<Real, Tout>(s, s->f.as<vec4_t<Real>>(), lin, st, pos_in);
    if (s->wall)
        return apply_wall<Real, Tout>(s, ang, s->f.as<vec4_t<Real>>(), s->t.as<vec4_t<Real>>(), lin, angout, st,
                                      pos_in);
    const TileConfig &cf = s->cfg[ang ? 1 : 0];
    if (cf.tm == 0 || (cf.automatic && s->n >= kAutoSymN))
        return apply_sym<Real, Tout>(s, ang, cf.tm == 0 ? cf.n_split : 0, lin, angout, st, pos_in);
    if (s->cfg[ang ? 1 : 0].tm == 3)
        return apply_fused<Real, Tout>(s, ang, s->f.as<Real>(), ang ? s->t.as<Real>() : nullptr, 4, lin, angout, st,
                                       pos_in);
    const int64_t n = s->n;
    const int splits = splits_for(s, ang);
    const int nc = (ang ? 6 : 3) * (std::is_same<Real, float>::value ? 2 : 1);
    HIP_TRY(s, s->part.ensure((size_t)splits * nc * n * sizeof(Real)));
    const PairConst<Real> pc = make_pair_const<Real>(s->radius);
    const auto *pos = pos_in ? static_cast<const vec4_t<Real> *>(pos_in) : s->pos.as<vec4_t<Real>>();
    const auto *f = s->f.as<vec4_t<Real>>();
    const auto *t = s->t.as<vec4_t<Real>>();
    hipEvent_t e0 = timing_begin(s, RPY_KERNEL_PAIR, (double)n * (double)n);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    if (ang)
        HIP_TRY(s, (launch_pair<Real, true>(pos, f, t, n, pc, s->cfg[1], splits, s->part.as<Real>(), st)));
    else
        HIP_TRY(s, (launch_pair<Real, false>(pos, f, nullptr, n, pc, s->cfg[0], splits, s->part.as<Real>(), st)));
    if (hipEvent_t e1 = timing_end(s, RPY_KERNEL_PAIR)) HIP_TRY(s, hipEventRecord(e1, st));
    if (ang)
        HIP_TRY(s, (launch_reduce<Real, Tout, true>(s->part.as<Real>(), splits, n, k_factor(s), lin, angout, st)));
    else
        HIP_TRY(s, (launch_reduce<Real, Tout, false>(s->part.as<Real>(), splits, n, k_factor(s), lin, angout, st)));
    return RPY_OK;
}

hipEvent_t timing_begin(rpy_solver *s, int kind, double pairs) {
    if (!s->timing) return nullptr;
    auto &v = s->ev[kind];
    if (s->ev_used[kind] == v.size()) {
        // timing only: no system-scope cache writeback and invalidation at
        // each record, which would stall the work that follows it
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
            (void)hipEventDestroy(a);
            return nullptr;
        }
        v.emplace_back(a, b);
    }
    s->ev_pairs[kind] += pairs;
    return v[s->ev_used[kind]].first;
}

hipEvent_t timing_end(rpy_solver *s, int kind) {
    if (!s->timing || s->ev_used[kind] >= s->ev[kind].size()) return nullptr;
    return s->ev[kind][s->ev_used[kind]++].second;
}

template rpy_status apply_staged<float, float>(rpy_solver *, bool, float *, float *, hipStream_t, const void *);
template rpy_status apply_staged<float, double>(rpy_solver *, bool, double *, double *, hipStream_t, const void *);
template rpy_status apply_staged<double, double>(rpy_solver *, bool, double *, double *, hipStream_t,
                                                 const void *);

rpy_status ensure_vec_buffers(rpy_solver *s, bool ang) {
    const size_t elt = s->dtype == RPY_F64 ? sizeof(double4) : sizeof(float4);
    HIP_TRY(s, s->f.ensure(elt * s->n));
    if (ang) HIP_TRY(s, s->t.ensure(elt * s->n));
    return RPY_OK;
}

rpy_status check_ready(rpy_solver *s) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if (!s->initialized) return fail(s, RPY_ERR_NOT_INITIALIZED, "rpy_initialize has not been called");
    if (!s->have_pos) return fail(s, RPY_ERR_NO_POSITIONS, "rpy_set_positions has not been called");
    return RPY_OK;
}

}  // namespace rpy

namespace {

template <typename Real>
rpy_status mdot_typed(rpy_solver *s, const Real *F, const Real *T, Real *lin, Real *ang, hipStream_t st) {
    const bool angmode = (T != nullptr) || (ang != nullptr);
    if (s->cfg[angmode ? 1 : 0].tm == 3 && !s->wall && !s->pse)   // one launch, no staging
        return apply_fused<Real, Real>(s, angmode, F, T, 3, lin, ang, st);
    rpy_status r = ensure_vec_buffers(s, angmode);
    if (r != RPY_OK) return r;
    HIP_TRY(s, (launch_stage_vec<Real, Real>(F, s->n, s->f.as<vec4_t<Real>>(), st)));
    if (angmode) HIP_TRY(s, (launch_stage_vec<Real, Real>(T, s->n, s->t.as<vec4_t<Real>>(), st)));
    return apply_staged<Real, Real>(s, angmode, lin, ang, st);
}

}  // namespace

extern "C" {

rpy_status rpy_create(rpy_periodicity x, rpy_periodicity y, rpy_periodicity z, rpy_solver **out) {
    if (!out) return RPY_ERR_INVALID_ARG;
    *out = nullptr;
    for (rpy_periodicity p : {x, y, z})
        if ((int)p < (int)RPY_PERIODIC || (int)p > (int)RPY_TWO_WALLS) return RPY_ERR_INVALID_ARG;
    const bool periodic = x == RPY_PERIODIC && y == RPY_PERIODIC && z == RPY_PERIODIC;
    if (!periodic && (x != RPY_OPEN || y != RPY_OPEN || (z != RPY_OPEN && z != RPY_SINGLE_WALL)))
        return RPY_ERR_UNSUPPORTED_GEOMETRY;
    rpy_solver *s = new (std::nothrow) rpy_solver();
    if (!s) return RPY_ERR_OUT_OF_MEMORY;
    if (periodic && pse_create(s) != RPY_OK) {
        delete s;
        return RPY_ERR_OUT_OF_MEMORY;
    }
    s->per[0] = x;
    s->per[1] = y;
    s->per[2] = z;
    s->wall = z == RPY_SINGLE_WALL;
    *out = s;
    return RPY_OK;
}

rpy_status rpy_set_parameter(rpy_solver *s, const char *key, double value) {
    if (!s || !key) return RPY_ERR_INVALID_ARG;
    if (s->pse) return pse_set_parameter(s, key, value);
    if (s->wall && std::strcmp(key, "wallHeight") == 0) {
        if (!std::isfinite(value)) return fail(s, RPY_ERR_INVALID_ARG, "wallHeight must be finite");
        s->wall_height = value;
        s->err.clear();
        return RPY_OK;
    }
    if (s->wall)
        return fail(s, RPY_ERR_INVALID_ARG,
                    std::string("the single-wall geometry takes only 'wallHeight' (got '") + key + "')");
    return fail(s, RPY_ERR_INVALID_ARG,
                std::string("open boundaries take no domain parameters (got '") + key + "')");
}

rpy_status rpy_initialize(rpy_solver *s, double viscosity, double hydrodynamic_radius, int include_angular) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if (!(viscosity > 0.0) || !std::isfinite(viscosity))
        return fail(s, RPY_ERR_INVALID_ARG, "viscosity must be positive and finite");
    if (!(hydrodynamic_radius > 0.0) || !std::isfinite(hydrodynamic_radius))
        return fail(s, RPY_ERR_INVALID_ARG, "hydrodynamic radius must be positive and finite");
    if (s->pse && include_angular)
        return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY, "the periodic (PSE) solver takes forces only");
    s->eta = viscosity;
    s->radius = hydrodynamic_radius;
    s->angular = include_angular != 0;
    s->initialized = true;
    s->err.clear();
    return RPY_OK;
}

rpy_status rpy_set_positions(rpy_solver *s, const void *pos, int64_t n, rpy_dtype dtype, void *hip_stream) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if (!s->initialized) return fail(s, RPY_ERR_NOT_INITIALIZED, "rpy_initialize has not been called");
    if (!pos) return fail(s, RPY_ERR_INVALID_ARG, "positions pointer is NULL");
    if (n <= 0 || n > (int64_t)(1 << 30)) return fail(s, RPY_ERR_INVALID_ARG, "particle count must be in [1, 2^30]");
    if (dtype != RPY_F32 && dtype != RPY_F64) return fail(s, RPY_ERR_DTYPE_MISMATCH, "dtype must be RPY_F32 or RPY_F64");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const size_t elt = dtype == RPY_F64 ? sizeof(double4) : sizeof(float4);
    s->have_pos = false;
    HIP_TRY(s, s->pos.ensure(elt * n));
    HIP_TRY(s, s->flag.ensure(sizeof(unsigned)));
    if (!s->host_flag) HIP_TRY(s, hipHostMalloc((void **)&s->host_flag, sizeof(unsigned) * 4, hipHostMallocDefault));
    HIP_TRY(s, launch_fill_zero<unsigned>(s->flag.as<unsigned>(), 1, st));
    if (dtype == RPY_F64)
        HIP_TRY(s, (launch_stage_positions<double, double>(static_cast<const double *>(pos), n,
                                                           s->pos.as<double4>(), s->flag.as<unsigned>(), st)));
    else
        HIP_TRY(s, (launch_stage_positions<float, float>(static_cast<const float *>(pos), n,
                                                         s->pos.as<float4>(), s->flag.as<unsigned>(), st)));
    HIP_TRY(s, hipMemcpyAsync(s->host_flag, s->flag.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIP_TRY(s, hipStreamSynchronize(st));
    if (*s->host_flag != 0)
        return fail(s, RPY_ERR_NONFINITE, std::to_string(*s->host_flag) + " particle positions are not finite");
    s->n = n;
    s->dtype = dtype;
    s->have_pos = true;
    ++s->pos_version;
    s->err.clear();
    return RPY_OK;
}

rpy_status rpy_mdot(rpy_solver *s, const void *forces, const void *torques, void *lin_out, void *ang_out,
                    void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!forces && !torques) return fail(s, RPY_ERR_INVALID_ARG, "need forces, torques or both");
    if (!lin_out) return fail(s, RPY_ERR_INVALID_ARG, "linear output pointer is NULL");
    if ((torques || ang_out) && !s->angular)
        return fail(s, RPY_ERR_ANGULAR_DISABLED, "torques / angular output need include_angular");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return mdot_typed<double>(s, static_cast<const double *>(forces), static_cast<const double *>(torques),
                                  static_cast<double *>(lin_out), static_cast<double *>(ang_out), st);
    return mdot_typed<float>(s, static_cast<const float *>(forces), static_cast<const float *>(torques),
                             static_cast<float *>(lin_out), static_cast<float *>(ang_out), st);
}

rpy_status rpy_div_m(rpy_solver *s, void *lin_out, void *ang_out, void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!lin_out) return fail(s, RPY_ERR_INVALID_ARG, "linear output pointer is NULL");
    if (ang_out && !s->angular) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    if (s->wall)
        return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY,
                    "the drift above a wall is not zero: use rpy_div_m_rfd (random finite differences)");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // open space and the periodic box (M depends on differences of positions
    // and its kernel is divergence-free): d_X . M = 0
    if (s->dtype == RPY_F64) {
        HIP_TRY(s, launch_fill_zero<double>(static_cast<double *>(lin_out), 3 * s->n, st));
        if (ang_out) HIP_TRY(s, launch_fill_zero<double>(static_cast<double *>(ang_out), 3 * s->n, st));
    } else {
        HIP_TRY(s, launch_fill_zero<float>(static_cast<float *>(lin_out), 3 * s->n, st));
        if (ang_out) HIP_TRY(s, launch_fill_zero<float>(static_cast<float *>(ang_out), 3 * s->n, st));
    }
    return RPY_OK;
}

rpy_status rpy_enable_timing(rpy_solver *s, int enable) {
    if (!s) return RPY_ERR_INVALID_ARG;
    s->timing = enable != 0;
    for (int k = 0; k < kKernelClasses; ++k) {
        s->ev_used[k] = 0;
        s->ev_pairs[k] = 0.0;
    }
    return RPY_OK;
}

rpy_status rpy_kernel_time(rpy_solver *s, rpy_kernel kernel, double *ms_total, int64_t *launches, double *work) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if ((int)kernel < 0 || (int)kernel >= kKernelClasses) return fail(s, RPY_ERR_INVALID_ARG, "unknown kernel class");
    const int k = (int)kernel;
    double total = 0.0;
    for (size_t i = 0; i < s->ev_used[k]; ++i) {
        HIP_TRY(s, hipEventSynchronize(s->ev[k][i].second));
        float ms = 0.f;
        HIP_TRY(s, hipEventElapsedTime(&ms, s->ev[k][i].first, s->ev[k][i].second));
        total += ms;
    }
    if (ms_total) *ms_total = total;
    if (launches) *launches = (int64_t)s->ev_used[k];
    if (work) *work = s->ev_pairs[k];
    return RPY_OK;
}

const char *rpy_last_error(const rpy_solver *s) { return s ? s->err.c_str() : "null solver handle"; }

void rpy_destroy(rpy_solver *s) {
    if (!s) return;
    for (DevBuf *b : {&s->pos, &s->f, &s->t, &s->part, &s->flag, &s->lz_basis, &s->lz_w, &s->lz_scal, &s->lz_red,
                      &s->lz_q, &s->lz_vec, &s->lz_mon, &s->drift, &s->cg_vec, &s->cg_scal, &s->sym_fwd.task,
                      &s->sym_fwd.slot, &s->sym_fwd.order, &s->sym_adj.task, &s->sym_adj.slot, &s->sym_adj.order,
                      &s->sym_jpart, &s->sym_state})
        b->release();
    for (auto &v : s->ev)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    precond_release(s);
    pse_release(s);
    if (s->host_flag) (void)hipHostFree(s->host_flag);
    if (s->host_stat) (void)hipHostFree(s->host_stat);
    if (s->lz_event) (void)hipEventDestroy(s->lz_event);
    delete s;
}

}  // extern "C"

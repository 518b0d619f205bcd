// rpy_mdot_noalloc: the product of rpy_mdot without any device allocation.
//
// rpy_mdot stages forces and torques into solver-owned vec4 buffers and its
// pair kernel writes per-split partial sums into a solver-owned workspace;
// both grow on demand with hipMalloc.  Callers that cannot allocate (code
// under graph capture, tight serving loops) use this variant instead: the
// staged vectors and the partials live in one file-scope device array of
// fixed size, and the ordinary pair kernel and its fixed-order reduction
// run on it.  The number of source splits is the one rpy_mdot's tiles would
// use, lowered until the partials fit; sizes that do not fit even one split
// are rejected before anything is enqueued.
//
// The array exists once per GPU the library runs on.  Its device address is
// taken with hipGetSymbolAddress on the first call made with that device
// current and kept per device; host code only ever passes that address.
// Every call on one GPU shares the array: calls that overlap in time on one
// GPU (two streams, two host threads) race on it.  Nothing in it has to
// start at zero (every slot a kernel reads was written earlier in the same
// call).
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <mutex>

namespace rpy {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (NULL on failure).
hipError_t scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

template <typename Real>
rpy_status mdot_noalloc_typed(rpy_solver *s, const Real *F, const Real *T, Real *lin, Real *ang, hipStream_t st) {
    const bool angmode = (T != nullptr) || (ang != nullptr);
    const int64_t n = s->n;
    const size_t vec_bytes = align256(sizeof(vec4_t<Real>) * (size_t)n);
    const size_t staged = vec_bytes * (angmode ? 2 : 1);
    const int pc = (angmode ? 6 : 3) * (std::is_same<Real, float>::value ? 2 : 1);
    const size_t split_bytes = sizeof(Real) * (size_t)pc * (size_t)n;
    if (staged + split_bytes > kScratchBytes)
        return fail(s, RPY_ERR_INVALID_ARG,
                    "N = " + std::to_string(n) + " exceeds the no-allocation product's fixed workspace of " +
                        std::to_string(kScratchBytes >> 20) + " MiB");
    const int fit = (int)std::min<size_t>((kScratchBytes - staged) / split_bytes, (size_t)max_splits(n));
    TileConfig cfg = s->cfg[angmode ? 1 : 0];
    int splits;
    if (cfg.tm == 0 || cfg.tm == 3) {
        // the symmetric mode needs workspace that grows as N^2, the fused
        // kernel is another kernel: use the ordinary one with its default tiles
        cfg.tm = 2;
        cfg.n_split = 0;
        splits = choose_splits(n, 2, std::is_same<Real, double>::value, angmode);
    } else {
        splits = splits_for(s, angmode);
    }
    splits = std::max(1, std::min(splits, fit));
    void *base = nullptr;
    HIP_TRY(s, scratch_ptr(&base));
    auto *bytes = static_cast<unsigned char *>(base);
    auto *f4 = reinterpret_cast<vec4_t<Real> *>(bytes);
    auto *t4 = angmode ? reinterpret_cast<vec4_t<Real> *>(bytes + vec_bytes) : nullptr;
    Real *part = reinterpret_cast<Real *>(bytes + staged);
    HIP_TRY(s, (launch_stage_vec<Real, Real>(F, n, f4, st)));
    if (angmode) HIP_TRY(s, (launch_stage_vec<Real, Real>(T, n, t4, st)));
    const PairConst<Real> pcst = make_pair_const<Real>(s->radius);
    const auto *pos = s->pos.as<vec4_t<Real>>();
    if (angmode) {
        HIP_TRY(s, (launch_pair<Real, true>(pos, f4, t4, n, pcst, cfg, splits, part, st)));
        HIP_TRY(s, (launch_reduce<Real, Real, true>(part, splits, n, k_factor(s), lin, ang, st)));
    } else {
        HIP_TRY(s, (launch_pair<Real, false>(pos, f4, nullptr, n, pcst, cfg, splits, part, st)));
        HIP_TRY(s, (launch_reduce<Real, Real, false>(part, splits, n, k_factor(s), lin, nullptr, st)));
    }
    return RPY_OK;
}

}  // namespace
}  // namespace rpy

using namespace rpy;

extern "C" rpy_status rpy_mdot_noalloc(rpy_solver *s, const void *forces, const void *torques, void *lin_out,
                                       void *ang_out, void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!forces && !torques) return fail(s, RPY_ERR_INVALID_ARG, "need forces, torques or both");
    if (!lin_out) return fail(s, RPY_ERR_INVALID_ARG, "linear output pointer is NULL");
    if ((torques || ang_out) && !s->angular)
        return fail(s, RPY_ERR_ANGULAR_DISABLED, "torques / angular output need include_angular");
    if (s->wall || s->pse)
        return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY, "the no-allocation product is built for open boundaries");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return mdot_noalloc_typed<double>(s, static_cast<const double *>(forces), static_cast<const double *>(torques),
                                          static_cast<double *>(lin_out), static_cast<double *>(ang_out), st);
    return mdot_noalloc_typed<float>(s, static_cast<const float *>(forces), static_cast<const float *>(torques),
                                     static_cast<float *>(lin_out), static_cast<float *>(ang_out), st);
}

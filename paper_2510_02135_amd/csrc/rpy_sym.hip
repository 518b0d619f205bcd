// Pair kernel that evaluates every unordered pair once (gfx950).
//
// M(X) is symmetric in the pair: the block coupling target j to source i is
// the transpose of the one coupling i to j, with d -> -d (Rotne-Prager-
// Yamakawa blocks of eq. (block_mobility), Sec. 3.5).  The geometry of a
// pair (separation, 1/r, the coefficient functions, the overlap branch) is
// therefore computed once and applied in both directions: to target i from
// source j's vectors, and to target j from i's.  That saves the geometry on
// half the ordered pairs (17 of the 49 instructions of an angular pair in the
// direct form used here) at the price of summing the source-side results.
// The same machinery serves the forward product (FwdPairs) and the adjoint
// (AdjPairs), each a policy giving the target data, the source records and
// the one- and two-sided pair evaluations.
//
// Work decomposition
//   Particles form blocks of 256 x TM (512 for the forward product, 256 for
//   the adjoint).  A task is (target block I, a range of source blocks
//   J >= I): the lanes of its workgroup own the targets of I (TM per lane)
//   in registers, and the source blocks stream through
//   LDS in chunks of 64 (double-buffered: one barrier per chunk, the next
//   chunk's records loaded while this one is evaluated).  On an
//   off-diagonal chunk, lane l pairs its targets
//   with source (l + s) mod 64 at step s, so that in one step the 64 lanes
//   touch 64 different sources.  The wave's running sums for a source
//   travel with it: lane l holds those of source (l + s) mod 64, adds its
//   targets' contributions, and takes the next lane's sums for step s + 1
//   (a DPP rotate of the wavefront by one lane), so no LDS traffic is
//   spent on them.  After the chunk the four waves' sums are combined in
//   order and stored as the source-side
//   partial of (I, source).  The diagonal block J = I (self pair included)
//   is evaluated one-sided with broadcast reads, as in the ordinary kernel.
//   A reduction kernel sums, per particle, the target-side partials of its
//   own block's tasks and the source-side partials of every block before
//   it, in a fixed order (the result does not depend on scheduling).
// Precision: float32 target-side sums are folded into Neumaier pairs after
// every chunk of 64 sources (the angular pair adds four rounded terms to
// each running component, so shorter plain runs keep the error at that of
// the ordinary kernel); the source-side sums of one (I, chunk) are plain
// float32 over 512 targets; the reduction uses Neumaier pairs and float64
// at the end.  float64 runs plain double sums throughout.
// Memory: the source-side partials take (N / 512) x NC x N values and the
// target-side ones 2 NC 512 per task; large N is handled in slabs of
// target blocks whose partials fit a fixed workspace.
#include "rpy_adjoint.hpp"
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"
#include "rpy_sym.hpp"

#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <vector>

namespace rpy {
namespace {

// One task per workgroup (tasks[blockIdx.x]).
template <typename Real, typename P>
__global__ void __launch_bounds__(kSymThreads) __attribute__((amdgpu_waves_per_eu(P::kMinWaves)))
sym_kernel(typename P::Args args, int n, const int4 *__restrict__ tasks, int slot_base, int jbase, PairConst<Real> c,
           Real *__restrict__ ipart, Real *__restrict__ jpart) {
    sym_block_task<Real, P>(args, n, tasks[blockIdx.x], slot_base, jbase, c, ipart, jpart);
}

// The partials of one slab of target blocks s0 .. s1 - 1, per particle i of
// blocks s0 and later and component c = blockIdx.y (NC of them): the
// target-side partials of the tasks of i's own block b when it lies in the
// slab (slots slot0[b] .. slot0[b + 1] - 1, stored from slot_base on), then
// the source-side partials of the slab's blocks before b.  The running sums
// start at zero on the first slab (s0 = 0) and are carried between slabs in
// `state`; a particle is complete after the slab holding its own block,
// which scales by k and writes component c to outs[c / 3][3 i + c % 3]
// (skipped when NULL).  One slab holding every block is the plain order:
// own target-side partials, then the source-side partials of blocks 0 ..
// b - 1.  The loads of kAhead partials are issued before they enter the
// sequential, fixed-order sum.
template <typename Real, typename Tout, int NC, int BLK>
__global__ void __launch_bounds__(256)
sym_reduce_kernel(const Real *__restrict__ ipart, const Real *__restrict__ jpart, const int *__restrict__ slot0,
                  int slot_base, int s0, int s1, int n, double k, Real *__restrict__ state, Tout *o0, Tout *o1,
                  Tout *o2) {
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int PC = COMP ? 2 * NC : NC;
    constexpr int kAhead = 8;
    const int c = blockIdx.y;
    const int i = s0 * BLK + blockIdx.x * blockDim.x + threadIdx.x;
    Tout *o = c < 3 ? o0 : (c < 6 ? o1 : o2);
    if (i >= n || !o) return;
    const int b = i / BLK, t = i % BLK;
    const bool own = b < s1;
    const int ni = own ? slot0[b + 1] - slot0[b] : 0;
    const int jend = own ? b : s1;
    const size_t istride = (size_t)PC * BLK, jstride = (size_t)NC * (size_t)n, nn = (size_t)n;
    const Real *pi = ipart + (size_t)(own ? slot0[b] - slot_base : 0) * istride + (size_t)c * BLK + t;
    const Real *pj = jpart + (size_t)c * nn + i;
    const int nj = jend - s0;
    double v;
    if constexpr (COMP) {
        float s = 0.f, cp = 0.f, extra = 0.f;
        if (s0 > 0) {
            s = state[(size_t)(3 * c) * nn + i];
            cp = state[(size_t)(3 * c + 1) * nn + i];
            extra = state[(size_t)(3 * c + 2) * nn + i];
        }
        int q = 0;
        for (; q + kAhead <= ni; q += kAhead) {
            float x[kAhead], e[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                x[u] = pi[(size_t)(q + u) * istride];
                e[u] = pi[(size_t)(q + u) * istride + (size_t)NC * BLK];
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                neumaier(s, cp, x[u]);
                extra += e[u];
            }
        }
        for (; q < ni; ++q) {
            neumaier(s, cp, pi[(size_t)q * istride]);
            extra += pi[(size_t)q * istride + (size_t)NC * BLK];
        }
        int bb = 0;
        for (; bb + kAhead <= nj; bb += kAhead) {
            float x[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) x[u] = pj[(size_t)(bb + u) * jstride];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) neumaier(s, cp, x[u]);
        }
        for (; bb < nj; ++bb) neumaier(s, cp, pj[(size_t)bb * jstride]);
        if (!own) {
            state[(size_t)(3 * c) * nn + i] = s;
            state[(size_t)(3 * c + 1) * nn + i] = cp;
            state[(size_t)(3 * c + 2) * nn + i] = extra;
            return;
        }
        v = (double)s + ((double)cp + (double)extra);
    } else {
        double s = s0 > 0 ? (double)state[(size_t)c * nn + i] : 0.0;
        int q = 0;
        for (; q + kAhead <= ni; q += kAhead) {
            double x[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) x[u] = pi[(size_t)(q + u) * istride];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) s += x[u];
        }
        for (; q < ni; ++q) s += pi[(size_t)q * istride];
        int bb = 0;
        for (; bb + kAhead <= nj; bb += kAhead) {
            double x[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) x[u] = pj[(size_t)(bb + u) * jstride];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) s += x[u];
        }
        for (; bb < nj; ++bb) s += pj[(size_t)bb * jstride];
        if (!own) {
            state[(size_t)c * nn + i] = (Real)s;
            return;
        }
        v = s;
    }
    o[3 * (size_t)i + (c % 3)] = (Tout)(k * v);
}

// Task list for n particles, blocks of blk and `span` source blocks per
// task (0 = automatic), cached in T.
rpy_status sym_tasks(rpy_solver *s, SymTasks &T, int blk, int span) {
    const int64_t n = s->n;
    const int nb = (int)((n + blk - 1) / blk);
    if (span <= 0) span = std::max(1, std::min(nb, 2));
    if (T.n == n && T.span == span && T.blk == blk) return RPY_OK;
    std::vector<int4> tasks;
    std::vector<int> slot0(nb + 1, 0);
    for (int bi = 0; bi < nb; ++bi) {
        slot0[bi] = (int)tasks.size();
        for (int j0 = bi; j0 < nb; j0 += span)
            tasks.push_back(make_int4(bi, j0, std::min(nb, j0 + span), (int)tasks.size()));
    }
    slot0[nb] = (int)tasks.size();
    T.n = -1;
    HIP_TRY(s, T.task.ensure(sizeof(int4) * tasks.size()));
    HIP_TRY(s, T.slot.ensure(sizeof(int) * slot0.size()));
    HIP_TRY(s, hipMemcpy(T.task.p, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice));
    // Launch order when one launch covers every task: the tasks that hold a
    // diagonal block (its pairs evaluated one-sided, the cheaper loop) after
    // all others, so that the last wave of workgroups is made of the shorter
    // tasks.  A task's partials go to its own slot wherever it is launched,
    // so the results do not depend on the order.
    std::stable_partition(tasks.begin(), tasks.end(), [](const int4 &t) { return t.y != t.x; });
    HIP_TRY(s, T.order.ensure(sizeof(int4) * tasks.size()));
    HIP_TRY(s, hipMemcpy(T.order.p, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(T.slot.p, slot0.data(), sizeof(int) * slot0.size(), hipMemcpyHostToDevice));
    T.slot_host = std::move(slot0);
    T.n = n;
    T.span = span;
    T.blk = blk;
    T.ntasks = (int)tasks.size();
    return RPY_OK;
}

// Workspace of one slab (source-side partials of its blocks plus the
// target-side partials of their tasks): slabs of consecutive target blocks
// are formed so that each stays within this many bytes (a single block may
// exceed it).  RPY_SYM_SLAB_BLOCKS=m also caps a slab at m blocks.
constexpr size_t kSymSlabBytes = (size_t)8 << 30;

std::vector<int> sym_slabs(const SymTasks &T, int nb, size_t block_bytes, size_t task_bytes) {
    const char *env = std::getenv("RPY_SYM_SLAB_BLOCKS");
    const int cap = env && std::atoi(env) > 0 ? std::atoi(env) : nb;
    std::vector<int> bounds{0};
    size_t used = 0;
    for (int b = 0; b < nb; ++b) {
        const size_t add = block_bytes + task_bytes * (size_t)(T.slot_host[b + 1] - T.slot_host[b]);
        if (b > bounds.back() && (used + add > kSymSlabBytes || b - bounds.back() >= cap)) {
            bounds.push_back(b);
            used = 0;
        }
        used += add;
    }
    bounds.push_back(nb);
    return bounds;
}

// Launch the symmetric kernel of policy P and its reduction into outs, one
// slab of target blocks at a time.
template <typename Real, typename P, typename Tout>
rpy_status run_sym(rpy_solver *s, SymTasks &T, int span, const typename P::Args &args, int kind, Tout *o0, Tout *o1,
                   Tout *o2, hipStream_t st) {
    constexpr int BLK = kSymThreads * P::TM;
    constexpr bool COMP = std::is_same<Real, float>::value;
    const int64_t n = s->n;
    rpy_status r = sym_tasks(s, T, BLK, span);
    if (r != RPY_OK) return r;
    const int nb = (int)((n + BLK - 1) / BLK);
    const int pc = P::NC * (COMP ? 2 : 1);
    const size_t block_bytes = sizeof(Real) * P::NC * (size_t)n, task_bytes = sizeof(Real) * pc * BLK;
    const std::vector<int> slab = sym_slabs(T, nb, block_bytes, task_bytes);
    const int nslab = (int)slab.size() - 1;
    int max_blocks = 0, max_tasks = 0;
    for (int q = 0; q < nslab; ++q) {
        max_blocks = std::max(max_blocks, slab[q + 1] - slab[q]);
        max_tasks = std::max(max_tasks, T.slot_host[slab[q + 1]] - T.slot_host[slab[q]]);
    }
    HIP_TRY(s, s->part.ensure(task_bytes * (size_t)max_tasks));
    HIP_TRY(s, s->sym_jpart.ensure(block_bytes * (size_t)max_blocks));
    if (nslab > 1) HIP_TRY(s, s->sym_state.ensure(sizeof(Real) * (COMP ? 3 : 1) * P::NC * (size_t)n));
    const PairConst<Real> c = make_pair_const<Real>(s->radius);
    // with several slabs the timed span also holds the reductions between them
    hipEvent_t e0 = timing_begin(s, kind, (double)n * (double)n);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    for (int q = 0; q < nslab; ++q) {
        const int s0 = slab[q], s1 = slab[q + 1];
        const int t0 = T.slot_host[s0], t1 = T.slot_host[s1];
        const int4 *list = nslab == 1 ? T.order.as<int4>() : T.task.as<int4>() + t0;
        hipLaunchKernelGGL((sym_kernel<Real, P>), dim3((unsigned)(t1 - t0)), dim3(kSymThreads), 0, st, args, (int)n,
                           list, t0, s0, c, s->part.as<Real>(), s->sym_jpart.as<Real>());
        HIP_TRY(s, hipGetLastError());
        if (q == nslab - 1)
            if (hipEvent_t e1 = timing_end(s, kind)) HIP_TRY(s, hipEventRecord(e1, st));
        const dim3 rg((unsigned)((n - (int64_t)s0 * BLK + 255) / 256), (unsigned)P::NC);
        hipLaunchKernelGGL((sym_reduce_kernel<Real, Tout, P::NC, BLK>), rg, dim3(256), 0, st, s->part.as<Real>(),
                           s->sym_jpart.as<Real>(), T.slot.as<int>(), t0, s0, s1, (int)n, k_factor(s),
                           nslab > 1 ? s->sym_state.as<Real>() : (Real *)nullptr, o0, o1, o2);
        HIP_TRY(s, hipGetLastError());
    }
    return RPY_OK;
}

}  // namespace

int64_t sym_max_n() { return (int64_t)1 << 18; }   // the autotuner's range for the mode

// M [F; T] for the stored positions with F (and T) staged in s->f (s->t), by
// the symmetric pair kernel; `span` = source blocks per task.
template <typename Real, typename Tout>
rpy_status apply_sym(rpy_solver *s, bool ang, int span, Tout *lin, Tout *ang_out, hipStream_t st, const void *pos_in) {
    // automatic span of the product: one source block per task up to 128
    // target blocks (N <= 65,536), two above.  With two, N = 32,768 and
    // 65,536 leave a larger part of the chip idle at the end of the launch
    // (1,056 and 4,160 tasks); measured 12-14 % and 2-3 % slower there,
    // within 1 % of one block from N = 131,072 on (fewer partials)
    constexpr int64_t kBlk = kSymThreads * FwdPairs<Real, false>::TM;
    if (span <= 0) span = (s->n + kBlk - 1) / kBlk <= 128 ? 1 : 2;
    const auto *pos = pos_in ? static_cast<const vec4_t<Real> *>(pos_in) : s->pos.as<vec4_t<Real>>();
    const auto *f = s->f.as<vec4_t<Real>>();
    if (ang) {
        typename FwdPairs<Real, true>::Args a{pos, f, s->t.as<vec4_t<Real>>()};
        return run_sym<Real, FwdPairs<Real, true>, Tout>(s, s->sym_fwd, span, a, RPY_KERNEL_PAIR, lin, ang_out,
                                                         (Tout *)nullptr, st);
    }
    typename FwdPairs<Real, false>::Args a{pos, f, nullptr};
    return run_sym<Real, FwdPairs<Real, false>, Tout>(s, s->sym_fwd, span, a, RPY_KERNEL_PAIR, lin, (Tout *)nullptr,
                                                      (Tout *)nullptr, st);
}

// Adjoint by the symmetric mode: staged vectors f, g (, t, h) as vec4 of
// Real; outputs grad_pos, M g linear rows, angular rows (each may be NULL).
template <typename Real>
rpy_status adjoint_sym(rpy_solver *s, bool ang, const vec4_t<Real> *f, const vec4_t<Real> *g,
                       const vec4_t<Real> *t, const vec4_t<Real> *h, Real *gp, Real *gf, Real *gt, hipStream_t st) {
    const auto *pos = s->pos.as<vec4_t<Real>>();
    if (ang) {
        typename AdjPairs<Real, true>::Args a{pos, f, g, t, h};
        return run_sym<Real, AdjPairs<Real, true>, Real>(s, s->sym_adj, 0, a, RPY_KERNEL_ADJOINT, gp, gf, gt, st);
    }
    typename AdjPairs<Real, false>::Args a{pos, f, g, nullptr, nullptr};
    return run_sym<Real, AdjPairs<Real, false>, Real>(s, s->sym_adj, 0, a, RPY_KERNEL_ADJOINT, gp, gf, (Real *)nullptr,
                                                      st);
}

template rpy_status apply_sym<float, float>(rpy_solver *, bool, int, float *, float *, hipStream_t, const void *);
template rpy_status apply_sym<float, double>(rpy_solver *, bool, int, double *, double *, hipStream_t, const void *);
template rpy_status apply_sym<double, double>(rpy_solver *, bool, int, double *, double *, hipStream_t,
                                              const void *);
template rpy_status adjoint_sym<float>(rpy_solver *, bool, const float4 *, const float4 *, const float4 *,
                                       const float4 *, float *, float *, float *, hipStream_t);
template rpy_status adjoint_sym<double>(rpy_solver *, bool, const double4 *, const double4 *, const double4 *,
                                        const double4 *, double *, double *, double *, hipStream_t);

}  // namespace rpy

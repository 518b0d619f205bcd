// Batched solver: many independent open-boundary systems of uneven N.
//
// Mdot for every system runs in one persistent kernel: work items are
// (system, 64-target tile) pairs, ordered longest-system first and claimed
// one wavefront at a time from an atomic counter; a wavefront keeps its 64
// targets in registers and streams the system's sources with wave-uniform
// (scalar) loads, so systems of a few dozen particles and of thousands share
// the machine without per-system launches.  float32 mode folds per-256-source
// sums into Neumaier pairs like the single-system kernel.
//
// sqrtMdotW runs the Lanczos iteration of Sec. 3.3 for all systems in lock
// step on one global iteration counter kept in device memory, so the kernel
// sequence of one iteration is captured once into a HIP graph and replayed;
// float64 vector operations are segmented (every block of the segmented
// kernels lies inside one system) with fixed-order two-stage reductions, and
// converged systems drop out of all work.  Every iteration ends with the
// stopping rule of the single-system solver, decided on the device per
// system: the quadrature monitor computes each system's s_{k-1}, s_k and
// increment (to rounding, for safely positive definite T_k); only systems
// whose estimate cannot decide (within 0.1 % of tol, spectrum outside the
// quadrature's range, breakdown, max_iter) run the exact eigensolves of
// T_{k-1} and T_k.  A system that stops writes its result at once.  The
// host only polls the number of systems still active, every `check_every`
// iterations.
#include "rpy_device.hpp"
#include "rpy_krylov.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"
#include "rpy_sym.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

namespace rpy {
namespace {

constexpr int kBatchBlock = 256;   // 4 wavefronts per workgroup of the pair kernel
constexpr int kSrcChunk = 256;     // sources per compensated fold (float32)
constexpr int kSegChunk = 2048;    // vector elements per segmented block
constexpr int kSegThreads = 256;

// per-system status (double): beta0, increment, not-SPD flag, running
// max(|alpha|, beta), first breakdown iteration, iterations at stop
// (0 while active), result code (0 ok, 1 not converged, 2 not SPD),
// estimated increment (quadrature monitor), source of the final s (0 the
// eigensolver, 1 the quadrature estimate), spare
enum { BS_BETA0 = 0, BS_INCR, BS_NSPD, BS_TSCALE, BS_BREAK, BS_DONE, BS_CODE, BS_EST, BS_SRC, BS_SIZE = 10 };

// ---------------------------------------------------------------------------
// persistent batched pair kernel
// ---------------------------------------------------------------------------
// A task is (system, tile of 64 TM targets); lane l of the wave owns targets
// tile * 64 TM + m * 64 + l, m < TM.  The wave walks its system's sources in
// chunks of 64: each lane loads one source record (coalesced, issued one
// chunk ahead) into the wave's own LDS slots, and the chunk is then read by
// broadcast.  Only the wave itself touches its slots, and a wave's LDS
// operations complete in program order, so no workgroup barrier is needed.
template <typename Real, typename Tout, int TM>
__global__ void __launch_bounds__(kBatchBlock)
batch_pair_kernel(const vec4_t<Real> *__restrict__ rec, const int64_t *__restrict__ off,
                  const int2 *__restrict__ tasks, int ntasks, unsigned *__restrict__ counter,
                  const PairConst<Real> *__restrict__ pcs, const double *__restrict__ kfac,
                  const int *__restrict__ active, Tout *__restrict__ out) {
    using R4 = vec4_t<Real>;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int kWaves = kBatchBlock / 64;
    static_assert(kSrcChunk % 64 == 0, "fold points must fall on chunk ends");
    __shared__ R4 tile_p[kWaves][64];
    __shared__ R4 tile_f[kWaves][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
    while (true) {
        unsigned t = 0;
        if (lane == 0) t = atomicAdd(counter, 1u);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= (unsigned)ntasks) break;
        const int2 task = tasks[t];
        const int s = task.x;
        if (active && active[s] == 0) continue;
        const int64_t o = off[s];
        const int ns = (int)(off[s + 1] - o);
        const R4 *src = rec + 2 * o;
        R4 p[TM];
#pragma unroll
        for (int m = 0; m < TM; ++m) p[m] = src[2 * min(task.y * 64 * TM + m * 64 + lane, ns - 1)];
        const PairConst<Real> c = pcs[s];
        Real acc[TM][3], sum[TM][3], cmp[TM][3];
#pragma unroll
        for (int m = 0; m < TM; ++m)
#pragma unroll
            for (int d = 0; d < 3; ++d) acc[m][d] = sum[m][d] = cmp[m][d] = Real(0);
        // this lane's record of the first chunk
        R4 np = zero4, nf = zero4;
        if (lane < ns) {
            np = src[2 * lane];
            nf = src[2 * lane + 1];
        }
        for (int j0 = 0; j0 < ns; j0 += 64) {
            tile_p[wv][lane] = np;
            tile_f[wv][lane] = nf;
            // the next chunk's record, loaded while this chunk is evaluated
            const int jn = j0 + 64 + lane;
            if (jn < ns) {
                np = src[2 * jn];
                nf = src[2 * jn + 1];
            }
            __builtin_amdgcn_wave_barrier();
            const int cnt = min(64, ns - j0);
#pragma unroll 4
            for (int q = 0; q < cnt; ++q) {
                const R4 sp = tile_p[wv][q];
                const R4 sf = tile_f[wv][q];
#pragma unroll
                for (int m = 0; m < TM; ++m) interact<Real, false>(p[m].x, p[m].y, p[m].z, sp, sf, zero4, c, acc[m], nullptr);
            }
            __builtin_amdgcn_wave_barrier();
            if constexpr (COMP) {
                // fold every kSrcChunk sources and at the end, as before the staging
                if ((j0 + 64) % kSrcChunk == 0 || j0 + 64 >= ns) {
#pragma unroll
                    for (int m = 0; m < TM; ++m)
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            neumaier(sum[m][d], cmp[m][d], acc[m][d]);
                            acc[m][d] = Real(0);
                        }
                }
            }
        }
        const double kk = kfac[s];
#pragma unroll
        for (int m = 0; m < TM; ++m) {
            const int i = task.y * 64 * TM + m * 64 + lane;
            if (i < ns) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double v = COMP ? ((double)sum[m][d] + (double)cmp[m][d]) : (double)acc[m][d];
                    out[3 * (o + i) + d] = (Tout)(kk * v);
                }
            }
        }
    }
}

// positions (AoS total x 3) -> slot 0 of the nrs records of each particle,
// counting non-finite entries
template <typename Real>
__global__ void batch_stage_pos(const Real *__restrict__ in, int64_t ntot, int nrs, vec4_t<Real> *__restrict__ rec,
                                unsigned *__restrict__ nonfinite) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    const Real x = in[3 * i], y = in[3 * i + 1], z = in[3 * i + 2];
    if (!(isfinite((double)x) && isfinite((double)y) && isfinite((double)z))) atomicAdd(nonfinite, 1u);
    vec4_t<Real> v;
    v.x = x;
    v.y = y;
    v.z = z;
    v.w = Real(0);
    rec[(int64_t)nrs * i] = v;
}

// A 3-vector per particle -> record slot `slot` (1 force, 2 torque) of the
// nrs records of each particle.  Sources: the caller's AoS total x 3 array
// (NULL = zeros), or (kdev != NULL) column kdev[0] - 1 of the float64
// Lanczos basis, whose layout gives system s the entries
// [vmul o_s, vmul o_{s+1}): its 3 n_s linear rows, then (vmul = 6) its 3 n_s
// angular rows; psys (particle -> system) is needed for vmul = 6.
template <typename Tin, typename Real>
__global__ void batch_stage_vec(const Tin *__restrict__ in, const int *__restrict__ kdev, int64_t ld, int64_t ntot,
                                int nrs, int slot, int vmul, const int *__restrict__ psys,
                                const int64_t *__restrict__ off, vec4_t<Real> *__restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    vec4_t<Real> r;
    r.w = Real(0);
    if (!in) {
        r.x = r.y = r.z = Real(0);
    } else {
        const Tin *v = kdev ? in + (size_t)(kdev[0] - 1) * ld : in;
        int64_t e = 3 * i;
        if (kdev && vmul == 6) {
            const int s = psys[i];
            e = 3 * ((slot == 2 ? off[s + 1] : off[s]) + i);
        }
        r.x = (Real)v[e];
        r.y = (Real)v[e + 1];
        r.z = (Real)v[e + 2];
    }
    rec[(int64_t)nrs * i + slot] = r;
}

// ---------------------------------------------------------------------------
// block mode: each system's unordered pairs evaluated once (the symmetric
// pair machinery of rpy_sym.hpp), all systems' block tasks in one launch
// ---------------------------------------------------------------------------
// Records of the batch: NRS = 2 (position, force) or 3 (+ torque) vec4 per
// particle, systems contiguous.
template <typename Real, bool ANG>
struct BatchPairs : FwdPairs<Real, ANG> {
    using R4 = vec4_t<Real>;
    using Tgt = typename FwdPairs<Real, ANG>::Tgt;
    static constexpr int NRS = ANG ? 3 : 2;
    struct Args {
        const R4 *rec;   // the system's first record
    };
    __device__ static Tgt target(const Args &a, const PairConst<Real> &c, int idx, int n) {
        (void)c;
        const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
        const R4 p = a.rec[NRS * min(idx, n - 1)];
        Tgt k;
        k.x = p.x;
        k.y = p.y;
        k.z = p.z;
        k.f = idx < n ? a.rec[NRS * idx + 1] : zero4;
        k.t = zero4;
        if constexpr (ANG) k.t = idx < n ? a.rec[NRS * idx + 2] : zero4;
        return k;
    }
    // record r of source js as stored (a padding source js >= n reads
    // particle n - 1; sym_block_task zeroes its records r > 0)
    __device__ static R4 record(const Args &a, const PairConst<Real> &c, int r, int js, int n) {
        (void)c;
        return a.rec[NRS * min(js, n - 1) + r];
    }
};

// One block task per workgroup: tasks[b] = (target block, first source
// block, end source block, slot) of system task_sys[b]; its source-side
// partials go to jpart + joff[s] ([block][NC][n_s]), its target-side ones to
// slot `slot` of ipart.  Tasks of inactive systems (converged Lanczos
// recurrences) return at once.
template <typename Real, bool ANG>
__global__ void __launch_bounds__(kSymThreads) __attribute__((amdgpu_waves_per_eu(BatchPairs<Real, ANG>::kMinWaves)))
batch_block_kernel(const vec4_t<Real> *__restrict__ rec, const int64_t *__restrict__ off,
                   const int4 *__restrict__ tasks, const int *__restrict__ task_sys, const int64_t *__restrict__ joff,
                   const PairConst<Real> *__restrict__ pcs, const int *__restrict__ active, Real *__restrict__ ipart,
                   Real *__restrict__ jpart) {
    using P = BatchPairs<Real, ANG>;
    const int s = task_sys[blockIdx.x];
    if (active && active[s] == 0) return;
    const int64_t o = off[s];
    const int n = (int)(off[s + 1] - o);
    const typename P::Args a{rec + (int64_t)P::NRS * o};
    const PairConst<Real> c = pcs[s];
    sym_block_task<Real, P>(a, n, tasks[blockIdx.x], 0, 0, c, ipart, jpart + joff[s]);
}

// Per particle i of system s (chunks of 256 particles: chunks[x] = (s,
// first particle)) and component c = blockIdx.y: the target-side partials
// of the tasks of i's block b (slots slot0[soff[s] + b] ..
// slot0[soff[s] + b + 1] - 1), then the source-side partials of the
// system's blocks 0 .. b - 1, in that fixed order; scaled by k_s.  Output
// component c < 3 goes to lin[3 (o_s + i) + c] and c >= 3 to
// ang[3 (o_s + i) + c - 3] (separate outputs, vec_layout = 0), or, for a
// Lanczos vector with angular rows (vec_layout = 1, lin = ang = the
// vector), to entries 6 o_s + 3 i + c and 6 o_s + 3 n_s + 3 i + c - 3.
template <typename Real, typename Tout, int NC>
__global__ void __launch_bounds__(256)
batch_block_reduce(const Real *__restrict__ ipart, const Real *__restrict__ jpart, const int64_t *__restrict__ joff,
                   const int *__restrict__ slot0, const int *__restrict__ soff, const int2 *__restrict__ chunks,
                   const int64_t *__restrict__ off, const double *__restrict__ kfac, const int *__restrict__ active,
                   int vec_layout, Tout *__restrict__ lin, Tout *__restrict__ ang) {
    constexpr int BLK = kSymThreads * 2;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int PC = COMP ? 2 * NC : NC;
    constexpr int kAhead = 8;
    const int2 ch = chunks[blockIdx.x];
    const int s = ch.x;
    if (active && active[s] == 0) return;
    const int64_t o = off[s];
    const int n = (int)(off[s + 1] - o);
    const int i = ch.y + (int)threadIdx.x;
    if (i >= n) return;
    const int c = blockIdx.y;
    const int b = i / BLK, t = i % BLK;
    const int q0 = slot0[soff[s] + b], ni = slot0[soff[s] + b + 1] - q0;
    const size_t istride = (size_t)PC * BLK, jstride = (size_t)NC * (size_t)n;
    const Real *pi = ipart + (size_t)q0 * istride + (size_t)c * BLK + t;
    const Real *pj = jpart + joff[s] + (size_t)c * n + i;
    double v;
    if constexpr (COMP) {
        float sm = 0.f, cp = 0.f, extra = 0.f;
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
                neumaier(sm, cp, x[u]);
                extra += e[u];
            }
        }
        for (; q < ni; ++q) {
            neumaier(sm, cp, pi[(size_t)q * istride]);
            extra += pi[(size_t)q * istride + (size_t)NC * BLK];
        }
        int bb = 0;
        for (; bb + kAhead <= b; bb += kAhead) {
            float x[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) x[u] = pj[(size_t)(bb + u) * jstride];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) neumaier(sm, cp, x[u]);
        }
        for (; bb < b; ++bb) neumaier(sm, cp, pj[(size_t)bb * jstride]);
        v = (double)sm + ((double)cp + (double)extra);
    } else {
        double sm = 0.0;
        int q = 0;
        for (; q + kAhead <= ni; q += kAhead) {
            double x[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) x[u] = pi[(size_t)(q + u) * istride];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) sm += x[u];
        }
        for (; q < ni; ++q) sm += pi[(size_t)q * istride];
        int bb = 0;
        for (; bb + kAhead <= b; bb += kAhead) {
            double x[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) x[u] = pj[(size_t)(bb + u) * jstride];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) sm += x[u];
        }
        for (; bb < b; ++bb) sm += pj[(size_t)bb * jstride];
        v = sm;
    }
    v *= kfac[s];
    // separate outputs: particle o + i of each; a Lanczos vector with angular
    // rows: system s's linear entries from 6 o, its angular ones from 6 o + 3 n
    if (c < 3)
        lin[3 * ((vec_layout ? 2 * o : o) + i) + c] = (Tout)v;
    else
        ang[3 * ((vec_layout ? o + off[s + 1] : o) + i) + (c - 3)] = (Tout)v;
}

// ---------------------------------------------------------------------------
// segmented float64 vector kernels (block b covers [blk_lo[b], blk_hi[b]) of system blk_sys[b])
// ---------------------------------------------------------------------------
struct SegMap {
    const int *sys;
    const int64_t *lo, *hi;
};

__device__ __forceinline__ bool seg_skip(const SegMap &m, const int *active, int &s, int64_t &lo, int64_t &hi) {
    s = m.sys[blockIdx.x];
    lo = m.lo[blockIdx.x];
    hi = m.hi[blockIdx.x];
    return active[s] == 0;
}

// partial[b] = sum of w*w (or of in*in for the caller's W) over block b
template <typename Tin>
__global__ void seg_sumsq(const Tin *__restrict__ v, SegMap m, double *__restrict__ partial) {
    __shared__ double sh[kSegThreads];
    const int64_t lo = m.lo[blockIdx.x], hi = m.hi[blockIdx.x];
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double x = (double)v[i];
        acc = fma(x, x, acc);
    }
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// out[s * ostride + (kdev ? kdev[0] - 1 : 0)] = sum (or sqrt of the sum) of the partials of system s
__global__ void seg_sys_reduce(const double *__restrict__ partial, const int *__restrict__ b0,
                               const int *__restrict__ b1, int nsys, const int *__restrict__ active,
                               const int *__restrict__ kdev, double *__restrict__ out, int64_t ostride,
                               int take_sqrt) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys || (active && active[s] == 0)) return;
    double acc = 0.0;
    for (int b = b0[s]; b < b1[s]; ++b) acc += partial[b];
    const int col = kdev ? kdev[0] - 1 : 0;
    out[(size_t)s * ostride + col] = take_sqrt ? sqrt(acc) : acc;
}

// v1 = W / beta0 (system-wise)
template <typename Tin>
__global__ void seg_init_basis(double *__restrict__ v, const Tin *__restrict__ w, SegMap m,
                               const double *__restrict__ status, const int *__restrict__ active) {
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    const double inv = 1.0 / status[(size_t)s * BS_SIZE + BS_BETA0];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v[i] = (double)w[i] * inv;
}

// w -= beta_{k-1} v_{k-1} (k > 1), then partial[b] = v_k . w over the block
__global__ void seg_recur_dot(double *__restrict__ w, const double *__restrict__ V, int64_t ld,
                              const double *__restrict__ beta, int64_t lstride, SegMap m,
                              const int *__restrict__ active, const int *__restrict__ kdev,
                              double *__restrict__ partial) {
    __shared__ double sh[kSegThreads];
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    const int k = kdev[0];
    const double *vk = V + (size_t)(k - 1) * ld;
    const double *vp = k > 1 ? V + (size_t)(k - 2) * ld : nullptr;
    const double bp = k > 1 ? beta[(size_t)s * lstride + k - 2] : 0.0;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        double x = w[i];
        if (vp) x = fma(-bp, vp[i], x);
        w[i] = x;
        acc = fma(vk[i], x, acc);
    }
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// w -= alpha_k v_k
__global__ void seg_sub_alpha(double *__restrict__ w, const double *__restrict__ V, int64_t ld,
                              const double *__restrict__ alpha, int64_t lstride, SegMap m,
                              const int *__restrict__ active, const int *__restrict__ kdev) {
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    const int k = kdev[0];
    const double *vk = V + (size_t)(k - 1) * ld;
    const double a = alpha[(size_t)s * lstride + k - 1];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) w[i] = fma(-a, vk[i], w[i]);
}

// partial[b * kcap + j] = V[j][block] . w[block], j < k.  Each thread keeps
// its kSegChunk / kSegThreads entries of w in registers and, per group of
// eight columns, issues all its loads of the group before the first
// multiply-add (enough loads in flight to stream V near the HBM rate); the
// columns' sums are then added by wavefront butterflies and the wavefronts'
// values in order (one barrier pair per group).
__global__ void __launch_bounds__(kSegThreads)
seg_gemv_t_partial(const double *__restrict__ V, int64_t ld, const double *__restrict__ w, SegMap m,
                   const int *__restrict__ active, const int *__restrict__ kdev, int kcap,
                   double *__restrict__ partial) {
    constexpr int kCols = 8;
    constexpr int kRows = kSegChunk / kSegThreads;
    constexpr int kWaves = kSegThreads / 64;
    static_assert(kSegChunk % kSegThreads == 0, "whole rows per thread");
    __shared__ double sh[kWaves][kCols];
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    const int k = kdev[0];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double wr[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const int64_t i = lo + tid + (int64_t)q * kSegThreads;
        wr[q] = i < hi ? w[i] : 0.0;
    }
    for (int j0 = 0; j0 < k; j0 += kCols) {
        double x[kCols][kRows];
#pragma unroll
        for (int c = 0; c < kCols; ++c)
#pragma unroll
            for (int q = 0; q < kRows; ++q) {
                const int64_t i = lo + tid + (int64_t)q * kSegThreads;
                x[c][q] = (j0 + c < k && i < hi) ? V[(size_t)(j0 + c) * ld + i] : 0.0;
            }
        double acc[kCols];
#pragma unroll
        for (int c = 0; c < kCols; ++c) {
            acc[c] = 0.0;
#pragma unroll
            for (int q = 0; q < kRows; ++q) acc[c] = fma(x[c][q], wr[q], acc[c]);
            acc[c] = wave_sum(acc[c]);
        }
        __syncthreads();   // the previous group's values have been read
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < kCols; ++c) sh[wv][c] = acc[c];
        }
        __syncthreads();
        if (tid < kCols && j0 + tid < k) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) t += sh[q][tid];
            partial[(size_t)blockIdx.x * kcap + j0 + tid] = t;
        }
    }
}

// h[s * lstride + j] = sum over the blocks of system s of partial[b * kcap + j]
__global__ void seg_gemv_t_final(const double *__restrict__ partial, const int *__restrict__ b0,
                                 const int *__restrict__ b1, const int *__restrict__ active,
                                 const int *__restrict__ kdev, int kcap, double *__restrict__ h, int64_t lstride) {
    const int s = blockIdx.x;
    if (active[s] == 0) return;
    const int k = kdev[0];
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double acc = 0.0;
        for (int b = b0[s]; b < b1[s]; ++b) acc += partial[(size_t)b * kcap + j];
        h[(size_t)s * lstride + j] = acc;
    }
}

// w -= V_k h_s over the block: each thread takes its kSegChunk / kSegThreads
// rows at once and, per group of eight columns, issues all the group's
// loads before its multiply-adds (each row's sum in column order).
__global__ void __launch_bounds__(kSegThreads)
seg_gemv_n_sub(const double *__restrict__ V, int64_t ld, const double *__restrict__ h, int64_t lstride,
               double *__restrict__ w, SegMap m, const int *__restrict__ active, const int *__restrict__ kdev) {
    constexpr int kCols = 8;
    constexpr int kRows = kSegChunk / kSegThreads;
    __shared__ double hs[kMaxK];
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    const int k = kdev[0];
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = h[(size_t)s * lstride + j];
    __syncthreads();
    double acc[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) acc[q] = 0.0;
    for (int j0 = 0; j0 < k; j0 += kCols) {
        double x[kCols][kRows];
#pragma unroll
        for (int c = 0; c < kCols; ++c)
#pragma unroll
            for (int q = 0; q < kRows; ++q) {
                const int64_t i = lo + threadIdx.x + (int64_t)q * kSegThreads;
                x[c][q] = (j0 + c < k && i < hi) ? V[(size_t)(j0 + c) * ld + i] : 0.0;
            }
#pragma unroll
        for (int c = 0; c < kCols; ++c)
            if (j0 + c < k)
#pragma unroll
                for (int q = 0; q < kRows; ++q) acc[q] = fma(x[c][q], hs[j0 + c], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const int64_t i = lo + threadIdx.x + (int64_t)q * kSegThreads;
        if (i < hi) w[i] -= acc[q];
    }
}

// partial[b] = w . w over the block
__global__ void seg_norm_partial(const double *__restrict__ w, SegMap m, const int *__restrict__ active,
                                 double *__restrict__ partial) {
    __shared__ double sh[kSegThreads];
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) acc = fma(w[i], w[i], acc);
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// running max(|alpha|, beta) and first breakdown per system; reaching the
// system's dimension 3N_s (the whole space) counts as a breakdown too
__global__ void seg_finish_iter(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t lstride,
                                int nsys, const int *__restrict__ active, const int *__restrict__ kdev,
                                const int *__restrict__ dim_sys, double *__restrict__ status) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys || active[s] == 0) return;
    const int k = kdev[0];
    double *st = status + (size_t)s * BS_SIZE;
    const double a = fabs(alpha[(size_t)s * lstride + k - 1]), b = beta[(size_t)s * lstride + k - 1];
    const double sc = fmax(st[BS_TSCALE], fmax(a, b));
    st[BS_TSCALE] = sc;
    if (st[BS_BREAK] == 0.0 && (!(b > 1e-14 * sc) || k >= dim_sys[s])) st[BS_BREAK] = (double)k;
}

// V[k] = w / beta_k, or zeros after a breakdown
__global__ void seg_next_basis(double *__restrict__ V, int64_t ld, const double *__restrict__ w,
                               const double *__restrict__ beta, int64_t lstride, const double *__restrict__ status,
                               SegMap m, const int *__restrict__ active, const int *__restrict__ kdev) {
    int s;
    int64_t lo, hi;
    if (seg_skip(m, active, s, lo, hi)) return;
    const int k = kdev[0];
    const bool broken = status[(size_t)s * BS_SIZE + BS_BREAK] != 0.0;
    const double inv = broken ? 0.0 : 1.0 / beta[(size_t)s * lstride + k - 1];
    double *dst = V + (size_t)k * ld;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) dst[i] = broken ? 0.0 : w[i] * inv;
}

__global__ void advance_k(int *kdev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) kdev[0] += 1;
}

// eigensolves of T_{kc-1} (workgroup 0) and T_kc (workgroup 1) of every
// active system, kc = kdev[0] - 1 (the last completed iteration)
__global__ void __launch_bounds__(kEigThreads)
batch_tridiag(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t lstride,
              double *__restrict__ s_prev, double *__restrict__ s_cur, double *__restrict__ Q, int64_t qstride,
              double *__restrict__ status, const int *__restrict__ need, const int *__restrict__ kdev) {
    const int s = blockIdx.y;
    if (need[s] != 1) return;
    const int kc = kdev[0] - 1;
    const int kk = kc - 1 + (int)blockIdx.x;
    if (kk <= 0) return;
    tridiag_sqrt_block(alpha + (size_t)s * lstride, beta + (size_t)s * lstride, kk,
                       (blockIdx.x == 0 ? s_prev : s_cur) + (size_t)s * lstride,
                       Q + ((size_t)s * 2 + blockIdx.x) * qstride,
                       blockIdx.x == 1 ? status + (size_t)s * BS_SIZE + BS_NSPD : nullptr);
}

// status[slot] of system s = |b - [a; 0]| / |b| for the vectors a (length
// k-1) and b (length k) of the system, k = kdev[0] - koff, for the systems
// with gate[s] == 1.
__global__ void batch_increment(const double *__restrict__ s_prev, const double *__restrict__ s_cur, int64_t lstride,
                                double *__restrict__ status, const int *__restrict__ gate,
                                const int *__restrict__ kdev, int koff, int slot) {
    __shared__ double red[kSegThreads];
    const int s = blockIdx.x;
    if (gate[s] != 1) return;
    const int k = kdev[0] - koff;
    const double *a = s_prev + (size_t)s * lstride, *b = s_cur + (size_t)s * lstride;
    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double prev = (i < k - 1) ? a[i] : 0.0;
        const double dl = b[i] - prev;
        num = fma(dl, dl, num);
        den = fma(b[i], b[i], den);
    }
    num = block_sum(num, red);
    den = block_sum(den, red);
    if (threadIdx.x == 0) status[(size_t)s * BS_SIZE + slot] = (k >= 2 && den > 0.0) ? sqrt(num / den) : INFINITY;
}

// quadrature estimates of s_{k-1} (workgroup x = 0) and s_k (x = 1) of every
// active system at the current iteration k = kdev[0], k >= 2
__global__ void __launch_bounds__(kMonThreads)
batch_monitor(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t lstride,
              double *__restrict__ scratch, int64_t sstride, double *__restrict__ est_prev,
              double *__restrict__ est_cur, const int *__restrict__ active, const int *__restrict__ kdev) {
    const int s = blockIdx.y;
    if (active[s] == 0) return;
    const int k = kdev[0];
    const int kk = k - 1 + (int)blockIdx.x;
    if (k < 2 || kk <= 0) return;
    monitor_block(alpha + (size_t)s * lstride, beta + (size_t)s * lstride, k, kk,
                  scratch + ((size_t)s * 2 + blockIdx.x) * sstride,
                  (blockIdx.x == 0 ? est_prev : est_cur) + (size_t)s * lstride);
}

// Decision after iteration k = kdev[0] for every active system:
//   need[s] = 1  take the exact test (eigensolves of T_{k-1}, T_k): a
//                recorded breakdown, the iteration cap, an estimate that is
//                NaN (spectrum outside the quadrature's range) or within
//                0.1 % of tol, or every iteration (`every`);
//   need[s] = 2  converged on the estimate (below tol, which is accurate to
//                rounding), the result uses the quadrature s_k;
//   need[s] = 0  continue.
__global__ void batch_flag(const double *__restrict__ status, const int *__restrict__ active, int *__restrict__ need,
                           int nsys, int kcap, double tol, int every, const int *__restrict__ kdev) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    const int k = kdev[0];
    const double *st = status + (size_t)s * BS_SIZE;
    int f = 0;
    if (active[s] != 0) {
        const double est = st[BS_EST];
        if (every || k >= kcap || st[BS_BREAK] > 0.0 ||
            (k >= 2 && (!isfinite(est) || fabs(est - tol) <= 1e-3 * tol)))
            f = 1;
        else if (k >= 2 && est < tol)
            f = 2;
    }
    need[s] = f;
}

// Stopping decisions after iteration kc of the active systems that took the
// exact test; systems that stop are marked in `fresh` for the combine
// kernel.  kdev[1] receives the number of systems still active.
__global__ void batch_converge(double *__restrict__ status, int *__restrict__ active, int *__restrict__ fresh,
                               const int *__restrict__ need, int kcap, int nsys, double tol,
                               int *__restrict__ kdev) {
    __shared__ int cnt[kSegThreads];
    const int kc = kdev[0] - 1;
    int mine = 0;
    for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
        if (active[s] == 0) continue;
        if (need[s] == 0) {   // not tested this iteration: stays active
            ++mine;
            continue;
        }
        double *st = status + (size_t)s * BS_SIZE;
        if (need[s] == 2) {   // converged on the quadrature estimate
            st[BS_INCR] = st[BS_EST];
            st[BS_DONE] = (double)kc;
            st[BS_CODE] = 0.0;
            st[BS_SRC] = 1.0;
            active[s] = 0;
            fresh[s] = 1;
            continue;
        }
        st[BS_SRC] = 0.0;
        const int kb = (int)st[BS_BREAK];
        int done = 0;
        double code = 0.0;
        if (kb > 0) {
            done = kb;                   // invariant Krylov space: s_kc = [s_kb; 0]
        } else if (st[BS_NSPD] != 0.0) {
            done = kc;
            code = 2.0;
        } else if (kc >= 2 && st[BS_INCR] < tol) {
            done = kc;
        } else if (kc >= kcap) {
            done = kc;                   // max_iter reached
            code = 1.0;
        }
        if (done > 0) {
            st[BS_DONE] = (double)done;
            st[BS_CODE] = code;
            active[s] = 0;
            fresh[s] = 1;
        } else {
            ++mine;
        }
    }
    cnt[threadIdx.x] = mine;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) kdev[1] = cnt[0];
}

// y_s = prefactor beta0_s V_{k_s} s_s for every system that just stopped
template <typename Tout>
__global__ void batch_combine(const double *__restrict__ V, int64_t ld, const double *__restrict__ s_cur,
                              const double *__restrict__ s_est, int64_t lstride, const double *__restrict__ status,
                              const int *__restrict__ fresh, const double *__restrict__ prefactor, SegMap m,
                              const int64_t *__restrict__ off, Tout *__restrict__ out, Tout *__restrict__ ang) {
    __shared__ double hs[kMaxK];
    const int s = m.sys[blockIdx.x];
    if (fresh[s] == 0) return;
    const int64_t lo = m.lo[blockIdx.x], hi = m.hi[blockIdx.x];
    const double *st = status + (size_t)s * BS_SIZE;
    const int kf = (int)st[BS_DONE];
    const double *src = (st[BS_SRC] != 0.0 ? s_est : s_cur) + (size_t)s * lstride;
    for (int j = threadIdx.x; j < kf; j += blockDim.x) hs[j] = src[j];
    __syncthreads();
    const double scale = prefactor[0] * st[BS_BETA0];
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < kf; ++j) acc = fma(V[(size_t)j * ld + i], hs[j], acc);
        const Tout y = (Tout)(scale * acc);
        if (!ang) {
            out[i] = y;
        } else {
            // entries [6 o_s, 6 o_s + 3 n_s) are linear rows, the rest angular
            const int64_t o = off[s], r = i - 6 * o, n3 = 3 * (off[s + 1] - o);
            if (r < n3)
                out[3 * o + r] = y;
            else
                ang[3 * o + (r - n3)] = y;
        }
    }
}

__global__ void clear_ints(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// initial activity: systems with W = 0 produce zeros and never run
__global__ void batch_init_status(double *__restrict__ status, int *__restrict__ active, int *__restrict__ fresh,
                                  int nsys, int *__restrict__ kdev, int *__restrict__ nonfinite) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) kdev[0] = 1;
    if (s >= nsys) return;
    double *st = status + (size_t)s * BS_SIZE;
    const double b0 = st[BS_BETA0];
    if (!isfinite(b0)) atomicAdd(nonfinite, 1);
    active[s] = (b0 > 0.0 && isfinite(b0)) ? 1 : 0;
    fresh[s] = 0;
    for (int q = 1; q < BS_SIZE; ++q) st[q] = 0.0;
}

template <typename T>
__global__ void seg_zero_inactive(T *__restrict__ out, T *__restrict__ ang, const int64_t *__restrict__ off, SegMap m,
                                  const int *__restrict__ active, const double *__restrict__ status) {
    const int s = m.sys[blockIdx.x];
    if (active[s] != 0 || status[(size_t)s * BS_SIZE + BS_BETA0] != 0.0) return;
    for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < m.hi[blockIdx.x]; i += blockDim.x) {
        if (!ang) {
            out[i] = T(0);
        } else {
            const int64_t o = off[s], r = i - 6 * o, n3 = 3 * (off[s + 1] - o);
            if (r < n3)
                out[3 * o + r] = T(0);
            else
                ang[3 * o + (r - n3)] = T(0);
        }
    }
}

}  // namespace
}  // namespace rpy

using namespace rpy;

struct rpy_batch {
    int nsys = 0;
    int64_t ntot = 0;
    rpy_dtype dtype = RPY_F32;
    std::vector<int64_t> off;
    std::vector<double> eta, radius;
    bool have_pos = false;
    int ntasks = 0, nblk = 0;
    int max_sys_n = 0;
    // angular blocks: records per particle (position, force[, torque]) and
    // entries per particle of a Lanczos vector
    bool angular = false;
    int nrs = 2, vmul = 3;
    // pair-kernel configuration: targets per lane (tasks of 64 tm targets)
    // and persistent workgroups per CU, or tm = 0: the block mode (each
    // system's unordered pairs once); systems longest first
    int tm = 0, wg_per_cu = 8;
    std::vector<int> order;
    DevBuf d_off, d_kfac, d_pc, d_tasks, d_counter, d_rec, d_flag;
    // block mode: tasks (int4) and their systems, per-system offsets of the
    // source-side partials and of the slot table, chunks of the reduction,
    // particle -> system, and the partials
    int nbtasks = 0, nchunks = 0;
    DevBuf d_btask, d_bsys, d_joff, d_bslot0, d_soff, d_chunks, d_psys, d_ipart, d_jpart;
    DevBuf d_blk_sys, d_blk_lo, d_blk_hi, d_sys_b0, d_sys_b1, d_kmax;
    DevBuf V, w, lanc, red, Q, status, ints, pref, mon;
    unsigned *host_u = nullptr;
    int *host_i = nullptr;
    std::string err;
};

namespace {

rpy_status bfail(rpy_batch *b, rpy_status code, const std::string &msg) {
    if (b) b->err = msg;
    return code;
}

rpy_status bhip(rpy_batch *b, hipError_t e, const char *what) {
    if (b) b->err = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
    return e == hipErrorOutOfMemory ? RPY_ERR_OUT_OF_MEMORY : RPY_ERR_HIP;
}

#define BHIP(b, expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return bhip((b), e_, #expr);   \
    } while (0)

SegMap seg_map(const rpy_batch *b) {
    return SegMap{b->d_blk_sys.as<int>(), b->d_blk_lo.as<int64_t>(), b->d_blk_hi.as<int64_t>()};
}

// persistent grid: one wave per task at most, wg_per_cu workgroups per CU
unsigned persistent_blocks(const rpy_batch *b) {
    const int waves = std::max(1, b->ntasks);
    return (unsigned)std::min((waves + 3) / 4, 256 * b->wg_per_cu);
}

// task list (system, tile of 64 tm targets) in b->order, uploaded to d_tasks
hipError_t build_tasks(rpy_batch *b) {
    std::vector<int2> tasks;
    if (b->tm == 0) {   // block mode: its task list is built once (build_block_tasks)
        b->ntasks = 0;
        return hipSuccess;
    }
    const int tile = 64 * b->tm;
    for (int s : b->order) {
        const int64_t ns = b->off[s + 1] - b->off[s];
        for (int64_t t = 0; t < (ns + tile - 1) / tile; ++t) tasks.push_back(make_int2(s, (int)t));
    }
    b->ntasks = (int)tasks.size();
    hipError_t e = b->d_tasks.ensure(sizeof(int2) * tasks.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(b->d_tasks.p, tasks.data(), sizeof(int2) * tasks.size(), hipMemcpyHostToDevice);
}

// Block-mode tasks: per system, target blocks of BLK = 512 particles, one
// task per (target block I, source block J >= I); systems longest first,
// tasks of a block contiguous (their slot = their index).  Also the
// reduction's chunks and the particle -> system map.
hipError_t build_block_tasks(rpy_batch *b) {
    constexpr int BLK = kSymThreads * 2;
    const int nc = b->angular ? 6 : 3;
    std::vector<int4> tasks;
    std::vector<int> tsys, slot0, soff(b->nsys), psys((size_t)b->ntot);
    std::vector<int64_t> joff(b->nsys);
    std::vector<int2> chunks;
    int64_t jtot = 0;
    for (int s : b->order) {
        const int64_t n = b->off[s + 1] - b->off[s];
        const int nb = (int)((n + BLK - 1) / BLK);
        soff[s] = (int)slot0.size();
        joff[s] = jtot;
        jtot += (int64_t)nb * nc * n;
        for (int bi = 0; bi < nb; ++bi) {
            slot0.push_back((int)tasks.size());
            for (int j = bi; j < nb; ++j) {
                tasks.push_back(make_int4(bi, j, j + 1, (int)tasks.size()));
                tsys.push_back(s);
            }
        }
        slot0.push_back((int)tasks.size());
        for (int64_t c = 0; c < n; c += 256) chunks.push_back(make_int2(s, (int)c));
        for (int64_t i = b->off[s]; i < b->off[s + 1]; ++i) psys[(size_t)i] = s;
    }
    b->nbtasks = (int)tasks.size();
    b->nchunks = (int)chunks.size();
    const size_t pc = (size_t)nc * (b->dtype == RPY_F32 ? 2 : 1);
    const size_t elt = b->dtype == RPY_F64 ? sizeof(double) : sizeof(float);
    auto up = [&](DevBuf &d, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = d.ensure(bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = up(b->d_btask, tasks.data(), sizeof(int4) * tasks.size());
    if (e == hipSuccess) e = up(b->d_bsys, tsys.data(), sizeof(int) * tsys.size());
    if (e == hipSuccess) e = up(b->d_joff, joff.data(), sizeof(int64_t) * joff.size());
    if (e == hipSuccess) e = up(b->d_bslot0, slot0.data(), sizeof(int) * slot0.size());
    if (e == hipSuccess) e = up(b->d_soff, soff.data(), sizeof(int) * soff.size());
    if (e == hipSuccess) e = up(b->d_chunks, chunks.data(), sizeof(int2) * chunks.size());
    if (e == hipSuccess) e = up(b->d_psys, psys.data(), sizeof(int) * psys.size());
    if (e == hipSuccess) e = b->d_ipart.ensure(elt * pc * BLK * tasks.size());
    if (e == hipSuccess) e = b->d_jpart.ensure(elt * (size_t)std::max<int64_t>(jtot, 1));
    return e;
}

// M [F; T] of every (active) system by the block mode into lin / ang (see
// batch_block_reduce for the output layouts).
template <typename Real, typename Tout>
void launch_batch_block(rpy_batch *b, const int *active, Tout *lin, Tout *ang, int vec_layout, hipStream_t st) {
    const dim3 rgrid((unsigned)b->nchunks, b->angular ? 6 : 3);
    if (b->angular) {
        hipLaunchKernelGGL((batch_block_kernel<Real, true>), dim3((unsigned)b->nbtasks), dim3(kSymThreads), 0, st,
                           b->d_rec.as<vec4_t<Real>>(), b->d_off.as<int64_t>(), b->d_btask.as<int4>(),
                           b->d_bsys.as<int>(), b->d_joff.as<int64_t>(), b->d_pc.as<PairConst<Real>>(), active,
                           b->d_ipart.as<Real>(), b->d_jpart.as<Real>());
        hipLaunchKernelGGL((batch_block_reduce<Real, Tout, 6>), rgrid, dim3(256), 0, st, b->d_ipart.as<Real>(),
                           b->d_jpart.as<Real>(), b->d_joff.as<int64_t>(), b->d_bslot0.as<int>(), b->d_soff.as<int>(),
                           b->d_chunks.as<int2>(), b->d_off.as<int64_t>(), b->d_kfac.as<double>(), active, vec_layout,
                           lin, ang);
    } else {
        hipLaunchKernelGGL((batch_block_kernel<Real, false>), dim3((unsigned)b->nbtasks), dim3(kSymThreads), 0, st,
                           b->d_rec.as<vec4_t<Real>>(), b->d_off.as<int64_t>(), b->d_btask.as<int4>(),
                           b->d_bsys.as<int>(), b->d_joff.as<int64_t>(), b->d_pc.as<PairConst<Real>>(), active,
                           b->d_ipart.as<Real>(), b->d_jpart.as<Real>());
        hipLaunchKernelGGL((batch_block_reduce<Real, Tout, 3>), rgrid, dim3(256), 0, st, b->d_ipart.as<Real>(),
                           b->d_jpart.as<Real>(), b->d_joff.as<int64_t>(), b->d_bslot0.as<int>(), b->d_soff.as<int>(),
                           b->d_chunks.as<int2>(), b->d_off.as<int64_t>(), b->d_kfac.as<double>(), active, vec_layout,
                           lin, (Tout *)nullptr);
    }
}

template <typename Real, typename Tout>
void launch_batch_pair(rpy_batch *b, const int *active, Tout *out, hipStream_t st) {
    const dim3 grid(persistent_blocks(b)), block(kBatchBlock);
    if (b->tm == 2)
        hipLaunchKernelGGL((batch_pair_kernel<Real, Tout, 2>), grid, block, 0, st, b->d_rec.as<vec4_t<Real>>(),
                           b->d_off.as<int64_t>(), b->d_tasks.as<int2>(), b->ntasks, b->d_counter.as<unsigned>(),
                           b->d_pc.as<PairConst<Real>>(), b->d_kfac.as<double>(), active, out);
    else
        hipLaunchKernelGGL((batch_pair_kernel<Real, Tout, 1>), grid, block, 0, st, b->d_rec.as<vec4_t<Real>>(),
                           b->d_off.as<int64_t>(), b->d_tasks.as<int2>(), b->ntasks, b->d_counter.as<unsigned>(),
                           b->d_pc.as<PairConst<Real>>(), b->d_kfac.as<double>(), active, out);
}

template <typename Real>
rpy_status batch_mdot_typed(rpy_batch *b, const Real *F, const Real *T, Real *out, Real *ang, hipStream_t st) {
    const dim3 g((unsigned)((b->ntot + 255) / 256));
    hipLaunchKernelGGL((batch_stage_vec<Real, Real>), g, dim3(256), 0, st, F, (const int *)nullptr, (int64_t)0,
                       b->ntot, b->nrs, 1, 3, (const int *)nullptr, (const int64_t *)nullptr,
                       b->d_rec.as<vec4_t<Real>>());
    if (b->angular)
        hipLaunchKernelGGL((batch_stage_vec<Real, Real>), g, dim3(256), 0, st, T, (const int *)nullptr, (int64_t)0,
                           b->ntot, b->nrs, 2, 3, (const int *)nullptr, (const int64_t *)nullptr,
                           b->d_rec.as<vec4_t<Real>>());
    if (b->tm == 0) {
        launch_batch_block<Real, Real>(b, nullptr, out, ang, 0, st);
    } else {
        BHIP(b, launch_fill_zero<unsigned>(b->d_counter.as<unsigned>(), 1, st));
        launch_batch_pair<Real, Real>(b, nullptr, out, st);
    }
    BHIP(b, hipGetLastError());
    return RPY_OK;
}

// Enqueue one Lanczos iteration for all active systems, with its stopping
// test, as one graph.
template <typename Real>
void enqueue_iteration(rpy_batch *b, int kcap, double tol, int every, Real *out, Real *ang, hipStream_t st) {
    const int64_t n = (int64_t)b->vmul * b->ntot;
    const int64_t ld = (n + 63) / 64 * 64;
    const int64_t L = kcap + 1;
    double *lan = b->lanc.as<double>();
    double *alpha = lan, *beta = lan + b->nsys * L, *h = lan + 2 * b->nsys * L;
    int *ints = b->ints.as<int>();
    int *kdev = ints, *active = ints + 2;
    const SegMap m = seg_map(b);
    const dim3 gb((unsigned)b->nblk), tb(kSegThreads);
    const dim3 gs((unsigned)((b->nsys + 255) / 256));
    double *V = b->V.as<double>(), *w = b->w.as<double>(), *red = b->red.as<double>();
    // w = M v_k (only active systems' tasks do work)
    const dim3 gp((unsigned)((b->ntot + 255) / 256));
    hipLaunchKernelGGL((batch_stage_vec<double, Real>), gp, dim3(256), 0, st, V, kdev, ld, b->ntot, b->nrs, 1,
                       b->vmul, b->d_psys.as<int>(), b->d_off.as<int64_t>(), b->d_rec.as<vec4_t<Real>>());
    if (b->angular)
        hipLaunchKernelGGL((batch_stage_vec<double, Real>), gp, dim3(256), 0, st, V, kdev, ld, b->ntot, b->nrs, 2,
                           b->vmul, b->d_psys.as<int>(), b->d_off.as<int64_t>(), b->d_rec.as<vec4_t<Real>>());
    if (b->tm == 0) {
        launch_batch_block<Real, double>(b, active, w, w, b->angular ? 1 : 0, st);
    } else {
        hipLaunchKernelGGL(clear_ints, dim3(1), dim3(64), 0, st, (int *)b->d_counter.p, 1);
        launch_batch_pair<Real, double>(b, active, w, st);
    }
    // recurrence
    hipLaunchKernelGGL(seg_recur_dot, gb, tb, 0, st, w, V, ld, beta, L, m, active, kdev, red);
    hipLaunchKernelGGL(seg_sys_reduce, gs, dim3(256), 0, st, red, b->d_sys_b0.as<int>(), b->d_sys_b1.as<int>(),
                       b->nsys, active, kdev, alpha, L, 0);
    hipLaunchKernelGGL(seg_sub_alpha, gb, tb, 0, st, w, V, ld, alpha, L, m, active, kdev);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(seg_gemv_t_partial, gb, tb, 0, st, V, ld, w, m, active, kdev, kcap, red);
        hipLaunchKernelGGL(seg_gemv_t_final, dim3((unsigned)b->nsys), dim3(256), 0, st, red, b->d_sys_b0.as<int>(),
                           b->d_sys_b1.as<int>(), active, kdev, kcap, h, L);
        hipLaunchKernelGGL(seg_gemv_n_sub, gb, tb, 0, st, V, ld, h, L, w, m, active, kdev);
    }
    hipLaunchKernelGGL(seg_norm_partial, gb, tb, 0, st, w, m, active, red);
    hipLaunchKernelGGL(seg_sys_reduce, gs, dim3(256), 0, st, red, b->d_sys_b0.as<int>(), b->d_sys_b1.as<int>(),
                       b->nsys, active, kdev, beta, L, 1);
    hipLaunchKernelGGL(seg_finish_iter, gs, dim3(256), 0, st, alpha, beta, L, b->nsys, active, kdev,
                       b->d_kmax.as<int>(), b->status.as<double>());
    hipLaunchKernelGGL(seg_next_basis, gb, tb, 0, st, V, ld, w, beta, L, b->status.as<double>(), m, active, kdev);
    // which systems take the exact test at this k
    double *s_prev = lan + 3 * b->nsys * L, *s_cur = lan + 4 * b->nsys * L;
    double *e_prev = lan + 5 * b->nsys * L, *e_cur = lan + 6 * b->nsys * L;
    int *fresh = ints + 2 + b->nsys, *need = ints + 3 + 2 * b->nsys;
    if (!every) {
        hipLaunchKernelGGL(batch_monitor, dim3(2, (unsigned)b->nsys), dim3(kMonThreads), 0, st, alpha, beta, L,
                           b->mon.as<double>(), (int64_t)kcap * kMonNodes, e_prev, e_cur, active, kdev);
        hipLaunchKernelGGL(batch_increment, dim3((unsigned)b->nsys), dim3(kSegThreads), 0, st, e_prev, e_cur, L,
                           b->status.as<double>(), active, kdev, 0, (int)BS_EST);
    }
    hipLaunchKernelGGL(batch_flag, gs, dim3(256), 0, st, b->status.as<double>(), active, need, b->nsys, kcap, tol,
                       every, kdev);
    hipLaunchKernelGGL(advance_k, dim3(1), dim3(64), 0, st, kdev);
    // exact test of the flagged systems (kc = kdev[0] - 1 from here on)
    hipLaunchKernelGGL(batch_tridiag, dim3(2, (unsigned)b->nsys), dim3(kEigThreads), 0, st, alpha, beta, L, s_prev,
                       s_cur, b->Q.as<double>(), (int64_t)kcap * kcap, b->status.as<double>(), need, kdev);
    hipLaunchKernelGGL(batch_increment, dim3((unsigned)b->nsys), dim3(kSegThreads), 0, st, s_prev, s_cur, L,
                       b->status.as<double>(), need, kdev, 1, (int)BS_INCR);
    hipLaunchKernelGGL(batch_converge, dim3(1), dim3(kSegThreads), 0, st, b->status.as<double>(), active, fresh, need,
                       kcap, b->nsys, tol, kdev);
    hipLaunchKernelGGL((batch_combine<Real>), dim3((unsigned)b->nblk), dim3(kSegThreads), 0, st, V, ld, s_cur, e_cur,
                       L, b->status.as<double>(), fresh, b->pref.as<double>(), m, b->d_off.as<int64_t>(), out, ang);
    hipLaunchKernelGGL(clear_ints, dim3((unsigned)((b->nsys + 255) / 256)), dim3(256), 0, st, fresh, b->nsys);
}

template <typename Real>
rpy_status batch_sqrt_typed(rpy_batch *b, const Real *w_in, double prefactor, double tol, int max_iter,
                            int check_every, Real *out, Real *ang, int *iters_out, hipStream_t st) {
    const int64_t n = (int64_t)b->vmul * b->ntot;
    const int64_t ld = (n + 63) / 64 * 64;
    const int kcap = std::min({max_iter, kMaxK, b->vmul * b->max_sys_n});
    const int64_t L = kcap + 1;
    BHIP(b, b->V.ensure((size_t)(kcap + 1) * ld * sizeof(double)));
    BHIP(b, b->w.ensure((size_t)ld * sizeof(double)));
    BHIP(b, b->lanc.ensure((size_t)7 * b->nsys * L * sizeof(double)));
    BHIP(b, b->mon.ensure((size_t)b->nsys * 2 * kcap * kMonNodes * sizeof(double)));
    BHIP(b, b->red.ensure((size_t)b->nblk * std::max(kcap, 1) * sizeof(double)));
    BHIP(b, b->Q.ensure((size_t)b->nsys * 2 * kcap * kcap * sizeof(double)));
    BHIP(b, b->status.ensure((size_t)b->nsys * BS_SIZE * sizeof(double)));
    BHIP(b, b->ints.ensure((size_t)(3 + 3 * b->nsys) * sizeof(int)));
    BHIP(b, b->pref.ensure(sizeof(double)));
    int *ints = b->ints.as<int>();
    int *kdev = ints, *active = ints + 2, *fresh = ints + 2 + b->nsys, *nonfin = ints + 2 + 2 * b->nsys;
    const SegMap m = seg_map(b);
    // per-system dimension 3 N_s (the Krylov space cannot grow beyond it)
    {
        std::vector<int> dims(b->nsys);
        for (int s = 0; s < b->nsys; ++s) dims[s] = (int)(b->vmul * (b->off[s + 1] - b->off[s]));
        BHIP(b, b->d_kmax.ensure(sizeof(int) * b->nsys));
        BHIP(b, hipMemcpy(b->d_kmax.p, dims.data(), sizeof(int) * b->nsys, hipMemcpyHostToDevice));
    }
    BHIP(b, hipMemcpy(b->pref.p, &prefactor, sizeof(double), hipMemcpyHostToDevice));
    // beta0 per system, activity, v1
    hipLaunchKernelGGL(clear_ints, dim3(1), dim3(64), 0, st, nonfin, 1);
    hipLaunchKernelGGL((seg_sumsq<Real>), dim3((unsigned)b->nblk), dim3(kSegThreads), 0, st, w_in, m, b->red.as<double>());
    hipLaunchKernelGGL(seg_sys_reduce, dim3((unsigned)((b->nsys + 255) / 256)), dim3(256), 0, st, b->red.as<double>(),
                       b->d_sys_b0.as<int>(), b->d_sys_b1.as<int>(), b->nsys, (const int *)nullptr,
                       (const int *)nullptr, b->status.as<double>(), (int64_t)BS_SIZE, 1);
    hipLaunchKernelGGL(batch_init_status, dim3((unsigned)((b->nsys + 255) / 256)), dim3(256), 0, st,
                       b->status.as<double>(), active, fresh, b->nsys, kdev, nonfin);
    hipLaunchKernelGGL((seg_zero_inactive<Real>), dim3((unsigned)b->nblk), dim3(kSegThreads), 0, st, out, ang,
                       b->d_off.as<int64_t>(), m, active, b->status.as<double>());
    hipLaunchKernelGGL((seg_init_basis<Real>), dim3((unsigned)b->nblk), dim3(kSegThreads), 0, st, b->V.as<double>(),
                       w_in, m, b->status.as<double>(), active);
    BHIP(b, hipGetLastError());
    BHIP(b, hipMemcpyAsync(b->host_i, nonfin, sizeof(int), hipMemcpyDeviceToHost, st));
    BHIP(b, hipStreamSynchronize(st));
    if (b->host_i[0] != 0) return bfail(b, RPY_ERR_NONFINITE, "the noise vector W is not finite");

    // capture one iteration (with its stopping test) as a graph
    const char *check_env = std::getenv("RPY_LANCZOS_CHECK");
    const int every = (check_env && std::string(check_env) == "every") ? 1 : 0;
    hipStream_t cap = nullptr;
    BHIP(b, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g_iter = nullptr;
    hipGraphExec_t x_iter = nullptr;
    auto cleanup = [&]() {
        if (x_iter) (void)hipGraphExecDestroy(x_iter);
        if (g_iter) (void)hipGraphDestroy(g_iter);
        (void)hipStreamDestroy(cap);
    };
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue_iteration<Real>(b, kcap, tol, every, out, ang, cap);
        e = hipStreamEndCapture(cap, &g_iter);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&x_iter, g_iter, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        cleanup();
        return bhip(b, e, "graph capture of the batched Lanczos iteration");
    }
    // systems stop on the device at their own first k meeting the rule; the
    // host polls the number still active every check_every iterations
    int n_active = 1;
    for (int k = 1; k <= kcap && n_active > 0; ++k) {
        e = hipGraphLaunch(x_iter, st);
        if (e == hipSuccess && (k % check_every == 0 || k == kcap)) {
            e = hipMemcpyAsync(b->host_i, kdev + 1, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e == hipSuccess) n_active = b->host_i[0];
        }
        if (e != hipSuccess) {
            cleanup();
            return bhip(b, e, "batched Lanczos iteration");
        }
    }
    cleanup();
    // per-system iteration counts and codes
    std::vector<double> stat((size_t)b->nsys * BS_SIZE);
    BHIP(b, hipMemcpyAsync(stat.data(), b->status.p, stat.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    BHIP(b, hipStreamSynchronize(st));
    bool nconv = false, nspd = false;
    for (int s = 0; s < b->nsys; ++s) {
        if (iters_out) iters_out[s] = (int)stat[(size_t)s * BS_SIZE + BS_DONE];
        const double c = stat[(size_t)s * BS_SIZE + BS_CODE];
        if (c == 1.0) nconv = true;
        if (c == 2.0) nspd = true;
    }
    if (nspd) return bfail(b, RPY_ERR_NOT_SPD, "a system's mobility matrix is not positive definite");
    if (nconv) return bfail(b, RPY_ERR_NOT_CONVERGED, "some systems did not converge within max_iter");
    return RPY_OK;
}

// out[i] = a fixed pseudo-random value in [-1, 1) (timing data for the tuner)
template <typename Real>
__global__ void batch_fill_pattern(Real *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned x = (unsigned)i * 2654435761u ^ 0x9e3779b9u;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    out[i] = Real((double)x * (2.0 / 4294967296.0) - 1.0);
}

// milliseconds per batched product over `burst` back-to-back products
template <typename Real>
rpy_status batch_time(rpy_batch *b, const Real *F, const Real *T, Real *out, Real *ang, int burst, hipStream_t st,
                      hipEvent_t e0, hipEvent_t e1, double *ms) {
    BHIP(b, hipEventRecord(e0, st));
    for (int r = 0; r < burst; ++r) {
        rpy_status q = batch_mdot_typed<Real>(b, F, T, out, ang, st);
        if (q != RPY_OK) return q;
    }
    BHIP(b, hipEventRecord(e1, st));
    BHIP(b, hipEventSynchronize(e1));
    float f = 0.f;
    BHIP(b, hipEventElapsedTime(&f, e0, e1));
    *ms = f / burst;
    return RPY_OK;
}

// Screen the block mode and every (targets per lane, workgroups per CU) of
// the one-sided kernel with single products, then re-time the best of each
// in interleaved rounds of ~100 ms bursts and keep the fastest (as the
// single-system tuner does).  With angular blocks only the block mode
// exists, and nothing is timed.
template <typename Real>
rpy_status batch_tune(rpy_batch *b, hipStream_t st) {
    if (b->angular) {
        b->tm = 0;
        return RPY_OK;
    }
    DevBuf data;
    const int64_t n3 = 3 * b->ntot;
    BHIP(b, data.ensure(2 * sizeof(Real) * (size_t)n3));
    Real *F = data.as<Real>(), *out = F + n3;
    hipLaunchKernelGGL((batch_fill_pattern<Real>), dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, F, n3);
    BHIP(b, hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIP(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, RPY_ERR_HIP, "hipEventCreate failed");
    }
    struct Cand {
        int tm, wg;
        double ms;
    };
    std::vector<Cand> cands{{0, 8, 0.0}};
    for (int tm : {1, 2})
        for (int wg : {4, 8, 16}) cands.push_back({tm, wg, 0.0});
    std::vector<Cand> screen;
    rpy_status r = RPY_OK;
    for (const Cand &cd : cands) {
        if (r != RPY_OK) break;
        b->tm = cd.tm;
        b->wg_per_cu = cd.wg;
        if (build_tasks(b) != hipSuccess) {
            r = bfail(b, RPY_ERR_HIP, "task list upload failed");
            break;
        }
        std::vector<double> t;
        for (int q = 0; q < 4 && r == RPY_OK; ++q) {
            double ms = 0.0;
            r = batch_time<Real>(b, F, nullptr, out, nullptr, 1, st, e0, e1, &ms);
            if (q > 0) t.push_back(ms);   // the first product is a warm-up
        }
        if (r == RPY_OK) {
            std::sort(t.begin(), t.end());
            screen.push_back({cd.tm, cd.wg, t[t.size() / 2]});
        }
    }
    Cand best{0, 8, 1e300};
    if (r == RPY_OK) {
        std::vector<Cand> fin;
        for (int tm : {0, 1, 2}) {
            Cand c{tm, 8, 1e300};
            for (const Cand &x : screen)
                if (x.tm == tm && x.ms < c.ms) c = x;
            fin.push_back(c);
        }
        const int burst = std::max(2, (int)std::min(64.0, 100.0 / std::max(fin[0].ms, 1e-3)));
        std::vector<std::vector<double>> t(fin.size());
        for (int round = 0; round < 5 && r == RPY_OK; ++round)
            for (size_t i = 0; i < fin.size() && r == RPY_OK; ++i) {
                b->tm = fin[i].tm;
                b->wg_per_cu = fin[i].wg;
                if (build_tasks(b) != hipSuccess) {
                    r = bfail(b, RPY_ERR_HIP, "task list upload failed");
                    break;
                }
                double ms = 0.0;
                r = batch_time<Real>(b, F, nullptr, out, nullptr, burst, st, e0, e1, &ms);
                t[i].push_back(ms);
            }
        for (size_t i = 0; i < fin.size() && r == RPY_OK; ++i) {
            std::sort(t[i].begin(), t[i].end());
            const double med = t[i][t[i].size() / 2];
            if (med < best.ms) best = {fin[i].tm, fin[i].wg, med};
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tm = best.tm;
    b->wg_per_cu = best.wg;
    if (build_tasks(b) != hipSuccess && r == RPY_OK) r = bfail(b, RPY_ERR_HIP, "task list upload failed");
    return r;
}

}  // namespace

extern "C" {

rpy_status rpy_batch_create(int32_t n_systems, const int64_t *offsets, const double *viscosity, const double *radius,
                            int include_angular, rpy_dtype dtype, rpy_batch **out) {
    if (!out) return RPY_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_systems <= 0 || !offsets || !viscosity || !radius) return RPY_ERR_INVALID_ARG;
    if (dtype != RPY_F32 && dtype != RPY_F64) return RPY_ERR_DTYPE_MISMATCH;
    if (offsets[0] != 0) return RPY_ERR_SIZE_MISMATCH;
    for (int s = 0; s < n_systems; ++s) {
        if (offsets[s + 1] <= offsets[s]) return RPY_ERR_SIZE_MISMATCH;
        if (offsets[s + 1] - offsets[s] > (1 << 24)) return RPY_ERR_SIZE_MISMATCH;
        if (!(viscosity[s] > 0.0) || !std::isfinite(viscosity[s]) || !(radius[s] > 0.0) || !std::isfinite(radius[s]))
            return RPY_ERR_INVALID_ARG;
    }
    if (offsets[n_systems] > (int64_t)(1 << 30)) return RPY_ERR_SIZE_MISMATCH;
    rpy_batch *b = new (std::nothrow) rpy_batch();
    if (!b) return RPY_ERR_OUT_OF_MEMORY;
    b->nsys = n_systems;
    b->dtype = dtype;
    b->off.assign(offsets, offsets + n_systems + 1);
    b->eta.assign(viscosity, viscosity + n_systems);
    b->radius.assign(radius, radius + n_systems);
    b->ntot = offsets[n_systems];
    b->angular = include_angular != 0;
    b->nrs = b->angular ? 3 : 2;
    b->vmul = b->angular ? 6 : 3;
    // systems longest first (the task lists are built from this order)
    b->order.resize(n_systems);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (b->off[x + 1] - b->off[x]) > (b->off[y + 1] - b->off[y]);
    });
    for (int s = 0; s < n_systems; ++s) b->max_sys_n = std::max<int>(b->max_sys_n, (int)(b->off[s + 1] - b->off[s]));
    // segmented blocks over the 3N-entry vectors
    std::vector<int> bsys, b0(n_systems), b1(n_systems);
    std::vector<int64_t> blo, bhi;
    for (int s = 0; s < n_systems; ++s) {
        b0[s] = (int)bsys.size();
        for (int64_t lo = b->vmul * b->off[s]; lo < b->vmul * b->off[s + 1]; lo += kSegChunk) {
            bsys.push_back(s);
            blo.push_back(lo);
            bhi.push_back(std::min<int64_t>(lo + kSegChunk, b->vmul * b->off[s + 1]));
        }
        b1[s] = (int)bsys.size();
    }
    b->nblk = (int)bsys.size();
    std::vector<double> kfac(n_systems);
    std::vector<PairConst<float>> pcf(n_systems);
    std::vector<PairConst<double>> pcd(n_systems);
    for (int s = 0; s < n_systems; ++s) {
        kfac[s] = 1.0 / (8.0 * M_PI * viscosity[s]);
        pcf[s] = make_pair_const<float>(radius[s]);
        pcd[s] = make_pair_const<double>(radius[s]);
    }
    auto up = [&](DevBuf &d, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = d.ensure(bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = up(b->d_off, b->off.data(), sizeof(int64_t) * (n_systems + 1));
    if (e == hipSuccess) e = up(b->d_kfac, kfac.data(), sizeof(double) * n_systems);
    if (e == hipSuccess)
        e = dtype == RPY_F64 ? up(b->d_pc, pcd.data(), sizeof(PairConst<double>) * n_systems)
                             : up(b->d_pc, pcf.data(), sizeof(PairConst<float>) * n_systems);
    if (e == hipSuccess) e = build_tasks(b);
    if (e == hipSuccess) e = build_block_tasks(b);
    if (e == hipSuccess) e = up(b->d_blk_sys, bsys.data(), sizeof(int) * bsys.size());
    if (e == hipSuccess) e = up(b->d_blk_lo, blo.data(), sizeof(int64_t) * blo.size());
    if (e == hipSuccess) e = up(b->d_blk_hi, bhi.data(), sizeof(int64_t) * bhi.size());
    if (e == hipSuccess) e = up(b->d_sys_b0, b0.data(), sizeof(int) * n_systems);
    if (e == hipSuccess) e = up(b->d_sys_b1, b1.data(), sizeof(int) * n_systems);
    if (e == hipSuccess) e = b->d_counter.ensure(sizeof(unsigned) * 4);
    if (e == hipSuccess) e = b->d_flag.ensure(sizeof(unsigned) * 4);
    const size_t elt = dtype == RPY_F64 ? sizeof(double4) : sizeof(float4);
    if (e == hipSuccess) e = b->d_rec.ensure((size_t)b->nrs * elt * b->ntot);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->host_u, sizeof(unsigned) * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->host_i, sizeof(int) * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        rpy_batch_destroy(b);
        return e == hipErrorOutOfMemory ? RPY_ERR_OUT_OF_MEMORY : RPY_ERR_HIP;
    }
    *out = b;
    return RPY_OK;
}

rpy_status rpy_batch_set_positions(rpy_batch *b, const void *pos, void *hip_stream) {
    if (!b) return RPY_ERR_INVALID_ARG;
    if (!pos) return bfail(b, RPY_ERR_INVALID_ARG, "positions pointer is NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    b->have_pos = false;
    BHIP(b, launch_fill_zero<unsigned>(b->d_flag.as<unsigned>(), 1, st));
    const dim3 g((unsigned)((b->ntot + 255) / 256));
    if (b->dtype == RPY_F64)
        hipLaunchKernelGGL((batch_stage_pos<double>), g, dim3(256), 0, st, static_cast<const double *>(pos), b->ntot,
                           b->nrs, b->d_rec.as<double4>(), b->d_flag.as<unsigned>());
    else
        hipLaunchKernelGGL((batch_stage_pos<float>), g, dim3(256), 0, st, static_cast<const float *>(pos), b->ntot,
                           b->nrs, b->d_rec.as<float4>(), b->d_flag.as<unsigned>());
    BHIP(b, hipGetLastError());
    BHIP(b, hipMemcpyAsync(b->host_u, b->d_flag.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    BHIP(b, hipStreamSynchronize(st));
    if (b->host_u[0] != 0) return bfail(b, RPY_ERR_NONFINITE, "particle positions are not finite");
    b->have_pos = true;
    b->err.clear();
    return RPY_OK;
}

rpy_status rpy_batch_mdot(rpy_batch *b, const void *forces, const void *torques, void *lin_out, void *ang_out,
                          void *hip_stream) {
    if (!b) return RPY_ERR_INVALID_ARG;
    if (!b->have_pos) return bfail(b, RPY_ERR_NO_POSITIONS, "rpy_batch_set_positions has not been called");
    if (!lin_out) return bfail(b, RPY_ERR_INVALID_ARG, "the linear output must not be NULL");
    if (!b->angular && (torques || ang_out))
        return bfail(b, RPY_ERR_ANGULAR_DISABLED, "torques / angular output need include_angular");
    if (b->angular && !ang_out) return bfail(b, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!forces && !torques) return bfail(b, RPY_ERR_INVALID_ARG, "need forces, torques or both");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (b->dtype == RPY_F64)
        return batch_mdot_typed<double>(b, static_cast<const double *>(forces), static_cast<const double *>(torques),
                                        static_cast<double *>(lin_out), static_cast<double *>(ang_out), st);
    return batch_mdot_typed<float>(b, static_cast<const float *>(forces), static_cast<const float *>(torques),
                                   static_cast<float *>(lin_out), static_cast<float *>(ang_out), st);
}

rpy_status rpy_batch_sqrt_mdot_w(rpy_batch *b, const void *w, double prefactor, double tol, int max_iter,
                                 int check_every, void *lin_out, void *ang_out, int *iters_out, void *hip_stream) {
    if (!b) return RPY_ERR_INVALID_ARG;
    if (!b->have_pos) return bfail(b, RPY_ERR_NO_POSITIONS, "rpy_batch_set_positions has not been called");
    if (!w || !lin_out) return bfail(b, RPY_ERR_INVALID_ARG, "W and the output must not be NULL");
    if (!b->angular && ang_out) return bfail(b, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    if (b->angular && !ang_out) return bfail(b, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!(tol > 0.0 && tol < 1.0)) return bfail(b, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (max_iter < 1 || max_iter > kMaxK)
        return bfail(b, RPY_ERR_INVALID_ARG, "max_iter must be in [1, 1024]");
    if (check_every < 1) return bfail(b, RPY_ERR_INVALID_ARG, "check_every must be >= 1");
    if (!std::isfinite(prefactor)) return bfail(b, RPY_ERR_INVALID_ARG, "prefactor must be finite");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (b->dtype == RPY_F64)
        return batch_sqrt_typed<double>(b, static_cast<const double *>(w), prefactor, tol, max_iter, check_every,
                                        static_cast<double *>(lin_out), static_cast<double *>(ang_out), iters_out, st);
    return batch_sqrt_typed<float>(b, static_cast<const float *>(w), prefactor, tol, max_iter, check_every,
                                   static_cast<float *>(lin_out), static_cast<float *>(ang_out), iters_out, st);
}

const char *rpy_batch_last_error(const rpy_batch *b) { return b ? b->err.c_str() : "null batch handle"; }

rpy_status rpy_batch_set_tile_config(rpy_batch *b, int targets_per_lane, int workgroups_per_cu) {
    if (!b) return RPY_ERR_INVALID_ARG;
    if (targets_per_lane != 0 && targets_per_lane != 1 && targets_per_lane != 2)
        return bfail(b, RPY_ERR_INVALID_ARG, "targets per lane must be 0 (block mode), 1 or 2");
    if (b->angular && targets_per_lane != 0)
        return bfail(b, RPY_ERR_INVALID_ARG, "with angular blocks only the block mode (0) exists");
    if (workgroups_per_cu < 1 || workgroups_per_cu > 32)
        return bfail(b, RPY_ERR_INVALID_ARG, "workgroups per CU must be in [1, 32]");
    b->tm = targets_per_lane;
    b->wg_per_cu = workgroups_per_cu;
    BHIP(b, build_tasks(b));
    return RPY_OK;
}

rpy_status rpy_batch_get_tile_config(const rpy_batch *b, int *targets_per_lane, int *workgroups_per_cu) {
    if (!b) return RPY_ERR_INVALID_ARG;
    if (targets_per_lane) *targets_per_lane = b->tm;
    if (workgroups_per_cu) *workgroups_per_cu = b->wg_per_cu;
    return RPY_OK;
}

rpy_status rpy_batch_autotune(rpy_batch *b, void *hip_stream) {
    if (!b) return RPY_ERR_INVALID_ARG;
    if (!b->have_pos) return bfail(b, RPY_ERR_NO_POSITIONS, "rpy_batch_set_positions has not been called");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    return b->dtype == RPY_F64 ? batch_tune<double>(b, st) : batch_tune<float>(b, st);
}

void rpy_batch_destroy(rpy_batch *b) {
    if (!b) return;
    for (DevBuf *d : {&b->d_btask, &b->d_bsys, &b->d_joff, &b->d_bslot0, &b->d_soff, &b->d_chunks, &b->d_psys,
                      &b->d_ipart, &b->d_jpart})
        d->release();
    for (DevBuf *d : {&b->d_off, &b->d_kfac, &b->d_pc, &b->d_tasks, &b->d_counter, &b->d_rec, &b->d_flag,
                      &b->d_blk_sys, &b->d_blk_lo, &b->d_blk_hi, &b->d_sys_b0, &b->d_sys_b1, &b->d_kmax, &b->V,
                      &b->w, &b->lanc, &b->red, &b->Q, &b->status, &b->ints, &b->pref, &b->mon})
        d->release();
    if (b->host_u) (void)hipHostFree(b->host_u);
    if (b->host_i) (void)hipHostFree(b->host_i);
    delete b;
}

}  // extern "C"

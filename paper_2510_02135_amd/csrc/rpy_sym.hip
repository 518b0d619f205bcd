// Pair kernel that evaluates every unordered pair once (gfx950).
//
// M(X) is symmetric in the pair: the block coupling target j to source i is
// the transpose of the one coupling i to j, with d -> -d (Rotne-Prager-
// Yamakawa blocks of eq. (block_mobility), Sec. 3.5).  The geometry of a
// pair (separation, 1/r, the coefficient functions, the overlap branch) is
// therefore computed once and applied in both directions: to target i from
// source j's vectors, and to target j from i's.  That saves the geometry on
// half the ordered pairs (about 12 of the 48 instructions of an angular pair)
// at the price of summing the source-side results.
//
// Work decomposition
//   Particles form blocks of 512.  A task is (target block I, a range of
//   source blocks J >= I): the lanes of its workgroup own the 512 targets
//   of I (two per lane) in registers, and the source blocks stream through
//   LDS in chunks of 64 (double-buffered: one barrier per chunk, the next
//   chunk's records loaded while this one is evaluated).  On an
//   off-diagonal chunk, lane l pairs its targets
//   with source (l + s) mod 64 at step s, so that in one step the 64 lanes
//   touch 64 different sources: each lane adds its targets' contributions
//   to that source into the wave's own LDS accumulator column (no
//   conflicts, in step order).  After the chunk the four
//   waves' columns are summed in order and stored as the source-side
//   partial of (I, source).  The diagonal block J = I (self pair included)
//   is evaluated one-sided with broadcast reads, as in the ordinary kernel.
//   A reduction kernel sums, per particle, the target-side partials of its
//   own block's tasks and the source-side partials of every block before
//   it, in a fixed order (the result does not depend on scheduling).
// Precision: float32 target-side sums are folded into Neumaier pairs every
// 256 sources; the source-side sums of one (I, chunk) are plain float32
// over 512 targets; the reduction uses Neumaier pairs and float64 at the
// end.  float64 runs plain double sums throughout.
// Memory: the source-side partials take (N / 512) x NC x N values, so the
// mode is offered up to N = 2^18 (about 3 GB in float64 with angular
// blocks).
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace rpy {
namespace {

constexpr int kSymThreads = 256;                   // 4 wavefronts
constexpr int kSymBlock = 512;                     // particles per block (two per lane)
constexpr int kSymChunk = 64;                      // sources per LDS chunk
constexpr int kSymChunks = kSymBlock / kSymChunk;  // chunks per block
constexpr int kSymFold = 4;                        // chunks between float32 folds (256 sources)

// Both directions of one angular pair in the regrouped form of interact_ang
// (rpy_device.hpp).  d = X_i - X_j.  Source records of j: p = (x, y, z, F'x),
// f = (F, F'y), t = (T, F'z), h = (T~, 0); the target's own records (fi, ti,
// hi, fpx_i) feed the reversed direction, where d -> -d flips the cross
// products and leaves (d.F) d unchanged.
template <typename Real>
__device__ __forceinline__ void sym_ang(Real xi, Real yi, Real zi, const vec4_t<Real> &p, const vec4_t<Real> &f,
                                        const vec4_t<Real> &t, const vec4_t<Real> &h, Real fpxi,
                                        const vec4_t<Real> &fi, const vec4_t<Real> &ti, const vec4_t<Real> &hi,
                                        const PairConst<Real> &c, Real *u, Real *w, Real *uj, Real *wj) {
    const Real dx = xi - p.x, dy = yi - p.y, dz = zi - p.z;
    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    Real g = ri * ri2;
    Real a1 = ri;
    Real f1 = fma(c.m_two_a2, ri2, Real(1));
    Real f2 = Real(1.5) * ri2;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        const Real rs = sel_pos(r2, ri);
        const Real r = r2 * rs;
        const Real An = fma(c.nA1, r, c.nA0);
        const Real Bn = c.nB * rs;
        const Real Gn = fma(c.nG1, r, c.nG0);
        const Real Dn = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
        const Real En = fma(c.nE_1, rs, c.nE1 * r);
        const Real inv = Real(1) / Gn;
        a1 = fma(-c.two_a2_3, Gn, An);
        f1 = Bn * inv;
        f2 = En * inv;
        g = Gn;
        const Real dd = fma(Real(0.5), Gn, Dn);
        w[0] = fma(dd, t.x, w[0]);
        w[1] = fma(dd, t.y, w[1]);
        w[2] = fma(dd, t.z, w[2]);
        wj[0] = fma(dd, ti.x, wj[0]);
        wj[1] = fma(dd, ti.y, wj[1]);
        wj[2] = fma(dd, ti.z, wj[2]);
    }
    // target i from source j
    {
        const Real s1 = f1 * fma(dx, f.x, fma(dy, f.y, dz * f.z));
        const Real s2 = f2 * fma(dx, t.x, fma(dy, t.y, dz * t.z));
        const Real vux = fma(-t.z, dy, fma(t.y, dz, fma(s1, dx, p.w)));
        const Real vuy = fma(-t.x, dz, fma(t.z, dx, fma(s1, dy, f.w)));
        const Real vuz = fma(-t.y, dx, fma(t.x, dy, fma(s1, dz, t.w)));
        u[0] = fma(a1, f.x, fma(g, vux, u[0]));
        u[1] = fma(a1, f.y, fma(g, vuy, u[1]));
        u[2] = fma(a1, f.z, fma(g, vuz, u[2]));
        const Real vwx = fma(-f.z, dy, fma(f.y, dz, fma(s2, dx, h.x)));
        const Real vwy = fma(-f.x, dz, fma(f.z, dx, fma(s2, dy, h.y)));
        const Real vwz = fma(-f.y, dx, fma(f.x, dy, fma(s2, dz, h.z)));
        w[0] = fma(g, vwx, w[0]);
        w[1] = fma(g, vwy, w[1]);
        w[2] = fma(g, vwz, w[2]);
    }
    // target j from source i (separation -d)
    {
        const Real s1 = f1 * fma(dx, fi.x, fma(dy, fi.y, dz * fi.z));
        const Real s2 = f2 * fma(dx, ti.x, fma(dy, ti.y, dz * ti.z));
        const Real vux = fma(ti.z, dy, fma(-ti.y, dz, fma(s1, dx, fpxi)));
        const Real vuy = fma(ti.x, dz, fma(-ti.z, dx, fma(s1, dy, fi.w)));
        const Real vuz = fma(ti.y, dx, fma(-ti.x, dy, fma(s1, dz, ti.w)));
        uj[0] = fma(a1, fi.x, fma(g, vux, uj[0]));
        uj[1] = fma(a1, fi.y, fma(g, vuy, uj[1]));
        uj[2] = fma(a1, fi.z, fma(g, vuz, uj[2]));
        const Real vwx = fma(fi.z, dy, fma(-fi.y, dz, fma(s2, dx, hi.x)));
        const Real vwy = fma(fi.x, dz, fma(-fi.z, dx, fma(s2, dy, hi.y)));
        const Real vwz = fma(fi.y, dx, fma(-fi.x, dy, fma(s2, dz, hi.z)));
        wj[0] = fma(g, vwx, wj[0]);
        wj[1] = fma(g, vwy, wj[1]);
        wj[2] = fma(g, vwz, wj[2]);
    }
}

// Both directions of one translational pair (U += A F + B (d.F) d; the
// reversed direction has the same A, B and (d.F) d).
template <typename Real>
__device__ __forceinline__ void sym_lin(Real xi, Real yi, Real zi, const vec4_t<Real> &p, const vec4_t<Real> &f,
                                        const vec4_t<Real> &fi, const PairConst<Real> &c, Real *u, Real *uj) {
    const Real dx = xi - p.x, dy = yi - p.y, dz = zi - p.z;
    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    const Real ri3 = ri * ri2;
    Real A = fma(c.two_a2_3, ri3, ri);
    Real B = fma(c.m_two_a2, ri3 * ri2, ri3);
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        const Real rs = sel_pos(r2, ri);
        A = fma(c.nA1, r2 * rs, c.nA0);
        B = c.nB * rs;
    }
    const Real s = B * fma(dx, f.x, fma(dy, f.y, dz * f.z));
    u[0] = fma(A, f.x, fma(s, dx, u[0]));
    u[1] = fma(A, f.y, fma(s, dy, u[1]));
    u[2] = fma(A, f.z, fma(s, dz, u[2]));
    const Real sj = B * fma(dx, fi.x, fma(dy, fi.y, dz * fi.z));
    uj[0] = fma(A, fi.x, fma(sj, dx, uj[0]));
    uj[1] = fma(A, fi.y, fma(sj, dy, uj[1]));
    uj[2] = fma(A, fi.z, fma(sj, dz, uj[2]));
}

// One task per workgroup: tasks[b] = (target block I, first source block,
// end source block, target-side partial slot).
//   ipart: [slot][PC][512]  target-side partials (float32: sums, then
//          compensations; PC = 2 NC, float64: NC)
//   jpart: [I][NC][n]       source-side partials
template <typename Real, bool ANG>
__global__ void __launch_bounds__(kSymThreads)
sym_pair_kernel(const vec4_t<Real> *__restrict__ pos, const vec4_t<Real> *__restrict__ frc,
                const vec4_t<Real> *__restrict__ trq, int n, const int4 *__restrict__ tasks, PairConst<Real> c,
                Real *__restrict__ ipart, Real *__restrict__ jpart) {
    using R4 = vec4_t<Real>;
    constexpr int NC = ANG ? 6 : 3;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int NR = ANG ? 4 : 2;   // records per source
    constexpr int kWaves = kSymThreads / 64;
    // double-buffered source records and source-side accumulators: one
    // barrier per chunk, the next chunk's records loaded during this one
    // the records are stored twice (columns q and q + 64) and the
    // accumulators keep 128 columns (q and q + 64 summed at the end), so a
    // lane's source at step st is column lane + st without a wrap: the
    // addresses are the lane's base plus a constant per step
    __shared__ R4 rec[2][NR][2 * kSymChunk];
    __shared__ Real jl[2][kWaves][NC][2 * kSymChunk];

    const int4 task = tasks[blockIdx.x];
    const int bi = task.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};

    // targets bi * 512 + m * 256 + tid; padding targets beyond n repeat the
    // last position with zero vectors, so their source-side terms vanish
    Real xi[2], yi[2], zi[2], fpx[2];
    R4 fi[2], ti[2], hi[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int idx = bi * kSymBlock + m * kSymThreads + tid;
        const R4 p = pos[min(idx, n - 1)];
        xi[m] = p.x;
        yi[m] = p.y;
        zi[m] = p.z;
        R4 f = idx < n ? frc[idx] : zero4;
        R4 t = (ANG && idx < n) ? trq[idx] : zero4;
        fpx[m] = c.two_a2_3 * f.x;
        f.w = c.two_a2_3 * f.y;
        t.w = c.two_a2_3 * f.z;
        R4 h;
        h.x = Real(-0.5) * t.x;
        h.y = Real(-0.5) * t.y;
        h.z = Real(-0.5) * t.z;
        h.w = Real(0);
        fi[m] = f;
        ti[m] = t;
        hi[m] = h;
    }
    Real acc[2][NC];
    Real sum[2][COMP ? NC : 1], cmp[2][COMP ? NC : 1];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            acc[m][k] = Real(0);
            if constexpr (COMP) {
                sum[m][k] = Real(0);
                cmp[m][k] = Real(0);
            }
        }
#pragma unroll
    for (int bf = 0; bf < 2; ++bf)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            jl[bf][wv][k][lane] = Real(0);
            jl[bf][wv][k][lane + kSymChunk] = Real(0);
        }

    // record `wv` (wave r stages record r) of source base + lane
    auto load_record = [&](int base) -> R4 {
        const int js = base + lane;
        const bool ok = js < n;
        const R4 p = pos[min(js, n - 1)];
        const R4 f = ok ? frc[js] : zero4;
        if constexpr (ANG) {
            const R4 t = ok ? trq[js] : zero4;
            if (wv == 0) return R4{p.x, p.y, p.z, c.two_a2_3 * f.x};
            if (wv == 1) return R4{f.x, f.y, f.z, c.two_a2_3 * f.y};
            if (wv == 2) return R4{t.x, t.y, t.z, c.two_a2_3 * f.z};
            return R4{Real(-0.5) * t.x, Real(-0.5) * t.y, Real(-0.5) * t.z, Real(0)};
        } else {
            return wv == 0 ? R4{p.x, p.y, p.z, Real(0)} : R4{f.x, f.y, f.z, Real(0)};
        }
    };
    // source-side sums of a finished chunk: the four waves in order, stored
    // as the partial of (bi, source); the entries are cleared for reuse
    auto combine = [&](int bf, int base) {
        for (int e = tid; e < NC * kSymChunk; e += kSymThreads) {
            const int k = e / kSymChunk, q = e % kSymChunk;
            Real v = Real(0);
#pragma unroll
            for (int w2 = 0; w2 < kWaves; ++w2) {
                v += jl[bf][w2][k][q] + jl[bf][w2][k][q + kSymChunk];
                jl[bf][w2][k][q] = Real(0);
                jl[bf][w2][k][q + kSymChunk] = Real(0);
            }
            const int js = base + q;
            if (js < n) jpart[((size_t)bi * NC + k) * (size_t)n + js] = v;
        }
    };

    const int nchunks = (task.z - task.y) * kSymChunks;
    auto chunk_base = [&](int ci) { return (task.y + ci / kSymChunks) * kSymBlock + (ci % kSymChunks) * kSymChunk; };
    R4 nxt = zero4;
    if (wv < NR) nxt = load_record(chunk_base(0));
    int chunks_since_fold = 0;
    for (int ci = 0; ci < nchunks; ++ci) {
        const int bf = ci & 1;
        const int base = chunk_base(ci);
        const bool diag = task.y + ci / kSymChunks == bi;
        if (wv < NR) {
            rec[bf][wv][lane] = nxt;
            rec[bf][wv][lane + kSymChunk] = nxt;
        }
        // rec[bf] complete; every wave has finished chunk ci - 1
        __syncthreads();
        if (ci > 0 && task.y + (ci - 1) / kSymChunks != bi) combine(bf ^ 1, chunk_base(ci - 1));
        if (wv < NR && ci + 1 < nchunks) nxt = load_record(chunk_base(ci + 1));
        if (diag) {
            // one-sided, every source of the block (self pair included)
#pragma unroll 2
            for (int q = 0; q < kSymChunk; ++q) {
                const R4 a = rec[bf][0][q];
                const R4 b = rec[bf][1][q];
                if constexpr (ANG) {
                    const R4 d = rec[bf][2][q];
                    const R4 e = rec[bf][3][q];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        interact_ang<Real>(xi[m], yi[m], zi[m], a, b, d, e, c, acc[m], acc[m] + 3);
                } else {
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        interact<Real, false>(xi[m], yi[m], zi[m], a, b, zero4, c, acc[m], nullptr);
                }
            }
        } else {
#pragma unroll 2
            for (int st = 0; st < kSymChunk; ++st) {
                const int q = lane + st;
                const R4 a = rec[bf][0][q];
                const R4 b = rec[bf][1][q];
                Real sj[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) sj[k] = Real(0);
                if constexpr (ANG) {
                    const R4 d = rec[bf][2][q];
                    const R4 e = rec[bf][3][q];
#pragma unroll
                    for (int m = 0; m < 2; ++m)
                        sym_ang<Real>(xi[m], yi[m], zi[m], a, b, d, e, fpx[m], fi[m], ti[m], hi[m], c, acc[m],
                                      acc[m] + 3, sj, sj + 3);
                } else {
#pragma unroll
                    for (int m = 0; m < 2; ++m) sym_lin<Real>(xi[m], yi[m], zi[m], a, b, fi[m], c, acc[m], sj);
                }
                // each lane owns column q of its wave's accumulator in this step,
                // and a wave's LDS operations complete in order: a plain
                // read-add-write is race-free (float64 uses the LDS add, which
                // is as fast; float32 LDS adds were about ten times slower)
                if constexpr (COMP) {
#pragma unroll
                    for (int k = 0; k < NC; ++k) jl[bf][wv][k][q] += sj[k];
                } else {
#pragma unroll
                    for (int k = 0; k < NC; ++k) atomicAdd(&jl[bf][wv][k][q], sj[k]);
                }
            }
        }
        if constexpr (COMP) {
            if (++chunks_since_fold == kSymFold) {
                chunks_since_fold = 0;
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        neumaier(sum[m][k], cmp[m][k], acc[m][k]);
                        acc[m][k] = Real(0);
                    }
            }
        }
    }
    __syncthreads();
    if (nchunks > 0 && task.y + (nchunks - 1) / kSymChunks != bi) combine((nchunks - 1) & 1, chunk_base(nchunks - 1));
    constexpr int PC = COMP ? 2 * NC : NC;
    Real *out = ipart + (size_t)task.w * PC * kSymBlock;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int t = m * kSymThreads + tid;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            if constexpr (COMP) {
                neumaier(sum[m][k], cmp[m][k], acc[m][k]);
                out[(size_t)k * kSymBlock + t] = sum[m][k];
                out[(size_t)(NC + k) * kSymBlock + t] = cmp[m][k];
            } else {
                out[(size_t)k * kSymBlock + t] = acc[m][k];
            }
        }
    }
}

// Per particle i (component blockIdx.y): the target-side partials of the
// tasks of its block (slots slot0[b] .. slot0[b + 1] - 1), then the
// source-side partials of blocks 0 .. b - 1, scaled by k.
template <typename Real, typename Tout, bool ANG>
__global__ void __launch_bounds__(256)
sym_reduce_kernel(const Real *__restrict__ ipart, const Real *__restrict__ jpart, const int *__restrict__ slot0,
                  int n, double k, Tout *__restrict__ lin, Tout *__restrict__ ang) {
    constexpr int NC = ANG ? 6 : 3;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int PC = COMP ? 2 * NC : NC;
    const int c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = i / kSymBlock, t = i % kSymBlock;
    const int s0 = slot0[b], s1 = slot0[b + 1];
    double v;
    if constexpr (COMP) {
        float s = 0.f, cp = 0.f, extra = 0.f;
        for (int q = s0; q < s1; ++q) {
            const Real *p = ipart + (size_t)q * PC * kSymBlock;
            neumaier(s, cp, p[(size_t)c * kSymBlock + t]);
            extra += p[(size_t)(NC + c) * kSymBlock + t];
        }
        for (int bb = 0; bb < b; ++bb) neumaier(s, cp, jpart[((size_t)bb * NC + c) * (size_t)n + i]);
        v = (double)s + ((double)cp + (double)extra);
    } else {
        double s = 0.0;
        for (int q = s0; q < s1; ++q) s += (double)ipart[((size_t)q * PC + c) * kSymBlock + t];
        for (int bb = 0; bb < b; ++bb) s += (double)jpart[((size_t)bb * NC + c) * (size_t)n + i];
        v = s;
    }
    const Tout out = (Tout)(k * v);
    if (c < 3)
        lin[3 * (size_t)i + c] = out;
    else
        ang[3 * (size_t)i + (c - 3)] = out;
}

}  // namespace

int64_t sym_max_n() { return (int64_t)1 << 18; }

// Task list for n particles and `span` source blocks per task (0 = automatic);
// cached on the solver.
rpy_status sym_tasks(rpy_solver *s, int span) {
    const int64_t n = s->n;
    const int nb = (int)((n + kSymBlock - 1) / kSymBlock);
    if (span <= 0) span = std::max(1, std::min(nb, 2));
    if (s->sym_n == n && s->sym_span == span) return RPY_OK;
    std::vector<int4> tasks;
    std::vector<int> slot0(nb + 1, 0);
    for (int bi = 0; bi < nb; ++bi) {
        slot0[bi] = (int)tasks.size();
        for (int j0 = bi; j0 < nb; j0 += span)
            tasks.push_back(make_int4(bi, j0, std::min(nb, j0 + span), (int)tasks.size()));
    }
    slot0[nb] = (int)tasks.size();
    HIP_TRY(s, s->sym_task_buf.ensure(sizeof(int4) * tasks.size()));
    HIP_TRY(s, s->sym_slot_buf.ensure(sizeof(int) * slot0.size()));
    HIP_TRY(s, hipMemcpy(s->sym_task_buf.p, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(s->sym_slot_buf.p, slot0.data(), sizeof(int) * slot0.size(), hipMemcpyHostToDevice));
    s->sym_n = n;
    s->sym_span = span;
    s->sym_ntasks = (int)tasks.size();
    return RPY_OK;
}

// M [F; T] for the stored positions with F (and T) staged in s->f (s->t), by
// the symmetric pair kernel; the tile configuration's n_split is the task's
// span in source blocks.
template <typename Real, typename Tout>
rpy_status apply_sym(rpy_solver *s, bool ang, int span, Tout *lin, Tout *ang_out, hipStream_t st, const void *pos_in) {
    const int64_t n = s->n;
    if (n > sym_max_n()) return fail(s, RPY_ERR_INVALID_ARG, "the symmetric pair mode is limited to N <= 2^18");
    rpy_status r = sym_tasks(s, span);
    if (r != RPY_OK) return r;
    const int nb = (int)((n + kSymBlock - 1) / kSymBlock);
    const int nc = ang ? 6 : 3;
    const int pc = nc * (std::is_same<Real, float>::value ? 2 : 1);
    HIP_TRY(s, s->part.ensure(sizeof(Real) * (size_t)s->sym_ntasks * pc * kSymBlock));
    HIP_TRY(s, s->sym_jpart.ensure(sizeof(Real) * (size_t)nb * nc * n));
    const PairConst<Real> c = make_pair_const<Real>(s->radius);
    const auto *pos = pos_in ? static_cast<const vec4_t<Real> *>(pos_in) : s->pos.as<vec4_t<Real>>();
    const auto *f = s->f.as<vec4_t<Real>>();
    const auto *t = ang ? s->t.as<vec4_t<Real>>() : nullptr;
    hipEvent_t e0 = timing_begin(s, RPY_KERNEL_PAIR, (double)n * (double)n);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    if (ang)
        hipLaunchKernelGGL((sym_pair_kernel<Real, true>), dim3((unsigned)s->sym_ntasks), dim3(kSymThreads), 0, st, pos,
                           f, t, (int)n, s->sym_task_buf.as<int4>(), c, s->part.as<Real>(), s->sym_jpart.as<Real>());
    else
        hipLaunchKernelGGL((sym_pair_kernel<Real, false>), dim3((unsigned)s->sym_ntasks), dim3(kSymThreads), 0, st,
                           pos, f, t, (int)n, s->sym_task_buf.as<int4>(), c, s->part.as<Real>(),
                           s->sym_jpart.as<Real>());
    HIP_TRY(s, hipGetLastError());
    if (hipEvent_t e1 = timing_end(s, RPY_KERNEL_PAIR)) HIP_TRY(s, hipEventRecord(e1, st));
    const dim3 rg((unsigned)((n + 255) / 256), (unsigned)nc);
    if (ang)
        hipLaunchKernelGGL((sym_reduce_kernel<Real, Tout, true>), rg, dim3(256), 0, st, s->part.as<Real>(),
                           s->sym_jpart.as<Real>(), s->sym_slot_buf.as<int>(), (int)n, k_factor(s), lin, ang_out);
    else
        hipLaunchKernelGGL((sym_reduce_kernel<Real, Tout, false>), rg, dim3(256), 0, st, s->part.as<Real>(),
                           s->sym_jpart.as<Real>(), s->sym_slot_buf.as<int>(), (int)n, k_factor(s), lin, ang_out);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

template rpy_status apply_sym<float, float>(rpy_solver *, bool, int, float *, float *, hipStream_t, const void *);
template rpy_status apply_sym<float, double>(rpy_solver *, bool, int, double *, double *, hipStream_t, const void *);
template rpy_status apply_sym<double, double>(rpy_solver *, bool, int, double *, double *, hipStream_t,
                                              const void *);

}  // namespace rpy

// The symmetric pair machinery (each unordered pair evaluated once and
// applied in both directions), shared by the single-system symmetric mode
// (rpy_sym.hip) and the batched solver (rpy_batch.hip).  The design notes
// are at the top of rpy_sym.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "rpy_adjoint.hpp"
#include "rpy_device.hpp"
#include "rpy_pair.hpp"

namespace rpy {
namespace {

constexpr int kSymThreads = 256;   // 4 wavefronts; blocks of 256 x (targets per lane) particles
constexpr int kSymChunk = 64;      // sources per LDS chunk
constexpr int kSymFold = 1;        // chunks between float32 folds (64 sources)

// The value lane (l + 1) mod 64 holds, for lane l: a DPP wavefront rotate
// by one lane (control 0x134, every row and bank enabled).  The caller runs
// with all 64 lanes active.
__device__ __forceinline__ float from_next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_next_lane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x134, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x134, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Coefficients of one angular pair in the direct form: with d = X_i - X_j
// and e = G d,
//   U_i += A F_j + f1 (d.F_j) e + T_j x e,   W_i += D T_j + f2 (d.T_j) e + F_j x e
// (eq. (block_mobility) in k-units: far field A = 1/r + (2a^2/3)/r^3,
// f1 = 1 - 2a^2/r^2, G = 1/r^3, D = -G/2, f2 = 3/(2r^2); the overlap branch
// r < 2a takes its own A, B/G, G, D, E/G; r = 0 gives the self blocks).
// The reversed direction (target j, source i) has d -> -d: the same A, D and
// (d.V) e terms, and the cross products change sign.
template <typename Real>
struct AngPair {
    Real dx, dy, dz, ex, ey, ez, A, f1, f2, D;
};

template <typename Real>
__device__ __forceinline__ AngPair<Real> ang_pair(Real xi, Real yi, Real zi, const vec4_t<Real> &p,
                                                  const PairConst<Real> &c) {
    AngPair<Real> q;
    q.dx = xi - p.x;
    q.dy = yi - p.y;
    q.dz = zi - p.z;
    const Real r2 = fma(q.dx, q.dx, fma(q.dy, q.dy, q.dz * q.dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    Real g = ri * ri2;
    q.A = fma(c.two_a2_3, g, ri);
    q.f1 = fma(c.m_two_a2, ri2, Real(1));
    q.f2 = Real(1.5) * ri2;
    q.D = Real(-0.5) * g;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        const Real rs = sel_pos(r2, ri);
        const Real r = r2 * rs;
        const Real Gn = fma(c.nG1, r, c.nG0);
        const Real inv = Real(1) / Gn;
        q.A = fma(c.nA1, r, c.nA0);
        q.f1 = c.nB * rs * inv;
        q.f2 = fma(c.nE_1, rs, c.nE1 * r) * inv;
        q.D = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
        g = Gn;
    }
    q.ex = g * q.dx;
    q.ey = g * q.dy;
    q.ez = g * q.dz;
    return q;
}

// Adds the contribution of force f and torque t at the other end of pair q
// to (u, w); SIGN = -1 for the reversed direction.
template <typename Real, int SIGN>
__device__ __forceinline__ void ang_apply(const AngPair<Real> &q, const vec4_t<Real> &f, const vec4_t<Real> &t,
                                          Real *u, Real *w) {
    const Real s1 = q.f1 * fma(q.dx, f.x, fma(q.dy, f.y, q.dz * f.z));
    const Real s2 = q.f2 * fma(q.dx, t.x, fma(q.dy, t.y, q.dz * t.z));
    const Real sg = Real(SIGN);
    u[0] = fma(sg * t.y, q.ez, fma(-sg * t.z, q.ey, fma(s1, q.ex, fma(q.A, f.x, u[0]))));
    u[1] = fma(sg * t.z, q.ex, fma(-sg * t.x, q.ez, fma(s1, q.ey, fma(q.A, f.y, u[1]))));
    u[2] = fma(sg * t.x, q.ey, fma(-sg * t.y, q.ex, fma(s1, q.ez, fma(q.A, f.z, u[2]))));
    w[0] = fma(sg * f.y, q.ez, fma(-sg * f.z, q.ey, fma(s2, q.ex, fma(q.D, t.x, w[0]))));
    w[1] = fma(sg * f.z, q.ex, fma(-sg * f.x, q.ez, fma(s2, q.ey, fma(q.D, t.y, w[1]))));
    w[2] = fma(sg * f.x, q.ey, fma(-sg * f.y, q.ex, fma(s2, q.ez, fma(q.D, t.z, w[2]))));
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

// ---------------------------------------------------------------------------
// pair policies: what a target holds, what a source record is, and the two
// pair evaluations (one-sided for the diagonal block, both directions
// elsewhere)
// ---------------------------------------------------------------------------
// Forward product M [F; T]: records position, force (, torque).
template <typename Real, bool ANG>
struct FwdPairs {
    using R4 = vec4_t<Real>;
    static constexpr int TM = 2;                 // targets per lane
    static constexpr int NC = ANG ? 6 : 3;       // output components
    static constexpr int NR = ANG ? 3 : 2;       // records per source
    // float32 angular: steps not unrolled and at most 128 VGPRs, so that
    // four waves share a SIMD (two unrolled steps retire as many
    // instructions per step and need 141 VGPRs, three waves); float64
    // translational likewise (116 VGPRs instead of 134); float64 angular
    // not unrolled and held to 168 VGPRs, three waves instead of two (six
    // values spilled; measured 5 % faster)
    static constexpr bool kFourWaves = ANG == std::is_same<Real, float>::value;
    static constexpr int kUnroll = (kFourWaves || ANG) ? 1 : 2;
    static constexpr int kMinWaves = kFourWaves ? 4 : (ANG ? 3 : 1);
    struct Args {
        const R4 *pos, *frc, *trq;
    };
    struct Tgt {
        Real x, y, z;
        R4 f, t;
    };
    __device__ static Tgt target(const Args &a, const PairConst<Real> &c, int idx, int n) {
        (void)c;
        const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
        const R4 p = a.pos[min(idx, n - 1)];
        Tgt k;
        k.x = p.x;
        k.y = p.y;
        k.z = p.z;
        k.f = idx < n ? a.frc[idx] : zero4;
        k.t = (ANG && idx < n) ? a.trq[idx] : zero4;
        return k;
    }
    // record r of source js (position, force (, torque)) as stored; a
    // padding source js >= n reads particle n - 1, and sym_block_task zeroes
    // its records r > 0 when it stores them.  One load from a base chosen per
    // record (r is uniform over the wavefront)
    __device__ static R4 record(const Args &a, const PairConst<Real> &c, int r, int js, int n) {
        (void)c;
        const R4 *src = r == 0 ? a.pos : (r == 1 ? a.frc : a.trq);
        return src[min(js, n - 1)];
    }
    __device__ static void one_sided(const Tgt &k, const R4 *q, const PairConst<Real> &c, Real *acc) {
        if constexpr (ANG) {
            const AngPair<Real> g = ang_pair<Real>(k.x, k.y, k.z, q[0], c);
            ang_apply<Real, 1>(g, q[1], q[2], acc, acc + 3);
        } else {
            const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
            interact<Real, false>(k.x, k.y, k.z, q[0], q[1], zero4, c, acc, nullptr);
        }
    }
    __device__ static void both(const Tgt &k, const R4 *q, const PairConst<Real> &c, Real *acc, Real *sj) {
        if constexpr (ANG) {
            const AngPair<Real> g = ang_pair<Real>(k.x, k.y, k.z, q[0], c);
            ang_apply<Real, 1>(g, q[1], q[2], acc, acc + 3);
            ang_apply<Real, -1>(g, k.f, k.t, sj, sj + 3);
        } else {
            sym_lin<Real>(k.x, k.y, k.z, q[0], q[1], k.f, c, acc, sj);
        }
    }
};

// Adjoint: records position, F, g_U (, T, g_W); outputs dX, (M g)_U (,
// (M g)_W), the pair term of rpy_adjoint.hpp.
template <typename Real, bool ANG>
struct AdjPairs {
    using R4 = vec4_t<Real>;
    static constexpr int TM = 1;
    static constexpr int NC = ANG ? 9 : 6;
    static constexpr int NR = ANG ? 5 : 3;
    // float32 angular: at most 128 VGPRs (four waves per SIMD instead of
    // three; the one value spilled is reloaded only on the overlap branch)
    static constexpr int kUnroll = 2;
    static constexpr int kMinWaves = (ANG && std::is_same<Real, float>::value) ? 4 : 1;
    struct Args {
        const R4 *pos, *frc, *gu, *trq, *gw;
    };
    using Tgt = rpy::Tgt<Real, ANG>;
    __device__ static Tgt target(const Args &a, const PairConst<Real> &c, int idx, int n) {
        (void)c;
        const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
        const bool ok = idx < n;
        const R4 p = a.pos[min(idx, n - 1)];
        const R4 f = ok ? a.frc[idx] : zero4, g = ok ? a.gu[idx] : zero4;
        Tgt k;
        k.x = p.x;
        k.y = p.y;
        k.z = p.z;
        k.fx = f.x;
        k.fy = f.y;
        k.fz = f.z;
        k.gx = g.x;
        k.gy = g.y;
        k.gz = g.z;
        if constexpr (ANG) {
            const R4 t = ok ? a.trq[idx] : zero4, h = ok ? a.gw[idx] : zero4;
            k.tx = t.x;
            k.ty = t.y;
            k.tz = t.z;
            k.hx = h.x;
            k.hy = h.y;
            k.hz = h.z;
        }
        return k;
    }
    // as FwdPairs::record: records r > 0 of padding sources are zeroed by
    // the caller
    __device__ static R4 record(const Args &a, const PairConst<Real> &c, int r, int js, int n) {
        (void)c;
        const R4 *src = r == 0 ? a.pos : r == 1 ? a.frc : r == 2 ? a.gu : r == 3 ? a.trq : a.gw;
        return src[min(js, n - 1)];
    }
    __device__ static void one_sided(const Tgt &k, const R4 *q, const PairConst<Real> &c, Real *acc) {
        const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
        adj_pair<Real, ANG, false>(k, q[0], q[1], q[2], ANG ? q[NR > 3 ? 3 : 0] : zero4,
                                   ANG ? q[NR > 4 ? 4 : 0] : zero4, c, acc, nullptr);
    }
    __device__ static void both(const Tgt &k, const R4 *q, const PairConst<Real> &c, Real *acc, Real *sj) {
        const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
        adj_pair<Real, ANG, true>(k, q[0], q[1], q[2], ANG ? q[NR > 3 ? 3 : 0] : zero4,
                                  ANG ? q[NR > 4 ? 4 : 0] : zero4, c, acc, sj);
    }
};

// The work of one workgroup: task = (target block I, first source block,
// end source block, target-side partial slot) of a system of n particles;
// blocks of BLK = 256 TM particles.  A launch covers the tasks of a slab of
// target blocks (jbase = its first block, slot_base = its first task's
// slot).
//   ipart: [slot - slot_base][PC][BLK]  target-side partials (float32: sums,
//          then compensations; PC = 2 NC, float64: NC)
//   jpart: [I - jbase][NC][n]           source-side partials
// s_waitcnt immediate of the GFX9 family: vmcnt(0), expcnt and lgkmcnt not
// waited for (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;

template <typename Real, typename P>
__device__ __forceinline__ void sym_block_task(const typename P::Args &args, int n, const int4 task, int slot_base,
                                               int jbase, const PairConst<Real> &c, Real *__restrict__ ipart,
                                               Real *__restrict__ jpart) {
    using R4 = vec4_t<Real>;
    constexpr int TM = P::TM, NC = P::NC, NR = P::NR;
    constexpr int BLK = kSymThreads * TM;
    constexpr int CHUNKS = BLK / kSymChunk;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int kWaves = kSymThreads / 64;
    constexpr int RPW = (NR + kWaves - 1) / kWaves;   // records staged per lane
    // double-buffered source records and source-side sums: one barrier per
    // chunk, the next chunk's records loaded during this one.  The records
    // are stored twice (columns q and q + 64), so a lane's source at step st
    // is column lane + st without a wrap: the addresses are the lane's base
    // plus a constant per step.  Source-side sums travel with their source
    // through the lanes (registers rotated by one lane per step) and land in
    // jl[bf][wave][k][q] at the end of the chunk
    // float64 records are kept as a 16-byte plane (x, y) and an 8-byte plane
    // z (w is never read): lanes reading consecutive 32-byte records would put
    // lanes l and l + 4 on the same LDS banks, and a (z, w) plane read for z
    // alone lanes l and l + 8; with these planes every read is consecutive
    constexpr int HP = std::is_same<Real, double>::value ? 2 : 1;
    using H = typename std::conditional<HP == 2, double2, R4>::type;
    constexpr int ZC = HP == 2 ? 2 * kSymChunk : 1;
    __shared__ H rec[2][NR][2 * kSymChunk];
    __shared__ Real recz[2][NR][ZC];
    __shared__ Real jl[2][kWaves][NC][kSymChunk];
    auto put_rec = [&](int bf, int r, int col, const R4 &v) {
        if constexpr (HP == 2) {
            rec[bf][r][col] = H{v.x, v.y};
            recz[bf][r][col] = v.z;
        } else {
            rec[bf][r][col] = v;
        }
    };
    auto get_rec = [&](int bf, int r, int col) -> R4 {
        if constexpr (HP == 2) {
            const H a = rec[bf][r][col];
            return R4{a.x, a.y, recz[bf][r][col], Real(0)};
        } else {
            return rec[bf][r][col];
        }
    };

    const int bi = task.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    // targets bi * BLK + m * 256 + tid; padding targets beyond n repeat the
    // last position with zero vectors, so their source-side terms vanish
    typename P::Tgt tg[TM];
#pragma unroll
    for (int m = 0; m < TM; ++m) tg[m] = P::target(args, c, bi * BLK + m * kSymThreads + tid, n);
    // the targets' loads complete here, before the first prefetch of source
    // records: the compiler then knows them complete inside the step loop,
    // which otherwise waits there for every outstanding load (the prefetch
    // included) at the first step of each chunk
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    Real acc[TM][NC];
    Real sum[TM][COMP ? NC : 1], cmp[TM][COMP ? NC : 1];
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            acc[m][k] = Real(0);
            if constexpr (COMP) {
                sum[m][k] = Real(0);
                cmp[m][k] = Real(0);
            }
        }

    // source-side sums of a finished chunk: the four waves in order, stored
    // as the partial of (bi, source)
    auto combine = [&](int bf, int base) {
        for (int e = tid; e < NC * kSymChunk; e += kSymThreads) {
            const int k = e / kSymChunk, q = e % kSymChunk;
            Real v = Real(0);
#pragma unroll
            for (int w2 = 0; w2 < kWaves; ++w2) v += jl[bf][w2][k][q];
            const int js = base + q;
            if (js < n) jpart[((size_t)(bi - jbase) * NC + k) * (size_t)n + js] = v;
        }
    };

    const int nchunks = (task.z - task.y) * CHUNKS;
    auto chunk_base = [&](int ci) { return (task.y + ci / CHUNKS) * BLK + (ci % CHUNKS) * kSymChunk; };
    R4 nxt[RPW];
#pragma unroll
    for (int u = 0; u < RPW; ++u)
        if (wv + u * kWaves < NR) nxt[u] = P::record(args, c, wv + u * kWaves, chunk_base(0) + lane, n);
    int chunks_since_fold = 0;
    for (int ci = 0; ci < nchunks; ++ci) {
        const int bf = ci & 1;
        const bool diag = task.y + ci / CHUNKS == bi;
        // the prefetched records have arrived (in every wavefront, also those
        // that load none: the compiler then knows the prefetch registers free
        // when the next prefetch is set up after the partials' stores)
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
#pragma unroll
        for (int u = 0; u < RPW; ++u) {
            const int r = wv + u * kWaves;
            if (r < NR) {
                // records r > 0 (vectors) of padding sources vanish
                const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
                const R4 v = (r > 0 && chunk_base(ci) + lane >= n) ? zero4 : nxt[u];
                put_rec(bf, r, lane, v);
                put_rec(bf, r, lane + kSymChunk, v);
            }
        }
        // rec[bf] complete; every wave has finished chunk ci - 1
        __syncthreads();
        if (ci > 0 && task.y + (ci - 1) / CHUNKS != bi) combine(bf ^ 1, chunk_base(ci - 1));
        if (ci + 1 < nchunks) {
#pragma unroll
            for (int u = 0; u < RPW; ++u)
                if (wv + u * kWaves < NR) nxt[u] = P::record(args, c, wv + u * kWaves, chunk_base(ci + 1) + lane, n);
        }
        if (diag) {
            // one-sided, every source of the block (self pair included)
#pragma unroll 2
            for (int q = 0; q < kSymChunk; ++q) {
                R4 rq[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) rq[r] = get_rec(bf, r, q);
#pragma unroll
                for (int m = 0; m < TM; ++m) P::one_sided(tg[m], rq, c, acc[m]);
            }
        } else {
            // sj holds the wave's sums for source (lane + st) mod 64; after
            // the step the next lane's register is the one for this lane's
            // next source.  64 rotations bring source l's sums back to lane l
            Real sj[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) sj[k] = Real(0);
#pragma unroll P::kUnroll
            for (int st = 0; st < kSymChunk; ++st) {
                const int q = lane + st;
                R4 rq[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) rq[r] = get_rec(bf, r, q);
#pragma unroll
                for (int m = 0; m < TM; ++m) P::both(tg[m], rq, c, acc[m], sj);
#pragma unroll
                for (int k = 0; k < NC; ++k) sj[k] = from_next_lane(sj[k]);
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) jl[bf][wv][k][lane] = sj[k];
        }
        if constexpr (COMP) {
            if (++chunks_since_fold == kSymFold) {
                chunks_since_fold = 0;
#pragma unroll
                for (int m = 0; m < TM; ++m)
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        neumaier(sum[m][k], cmp[m][k], acc[m][k]);
                        acc[m][k] = Real(0);
                    }
            }
        }
    }
    __syncthreads();
    if (nchunks > 0 && task.y + (nchunks - 1) / CHUNKS != bi) combine((nchunks - 1) & 1, chunk_base(nchunks - 1));
    constexpr int PC = COMP ? 2 * NC : NC;
    Real *out = ipart + (size_t)(task.w - slot_base) * PC * BLK;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int t = m * kSymThreads + tid;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            if constexpr (COMP) {
                neumaier(sum[m][k], cmp[m][k], acc[m][k]);
                out[(size_t)k * BLK + t] = sum[m][k];
                out[(size_t)(NC + k) * BLK + t] = cmp[m][k];
            } else {
                out[(size_t)k * BLK + t] = acc[m][k];
            }
        }
    }
}

}  // namespace
}  // namespace rpy

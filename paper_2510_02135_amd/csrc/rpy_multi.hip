// Several mobility products with one geometry (gfx950):
//   U_r = M(X) [F_r; T_r],  r = 0 .. nrhs-1,
// the blocks of eq. (block_mobility) applied to nrhs force (and torque)
// sets at the same positions.  Everything about a pair that does not depend
// on the vectors (separation, 1/r, the coefficient functions, the overlap
// branch) is computed once and applied to NV vectors, so the rsqrt and the
// geometry are shared.
//
// Work decomposition (as the single-vector pair kernel, one grid dimension
// more)
//   grid.x : target blocks of 256*TM targets (TM per lane, strided by 256);
//   grid.y : source splits (those of the single-vector product);
//   grid.z : groups of NV vectors.
//   A tile stages up to 256 source positions and, per vector, the force (and
//   torque) records.
// The order of the sum over sources and the Neumaier folding after every 256
// sources are those of the single-vector kernel.  The translational pair
// arithmetic is too, so translational results are bit-identical to single
// products of the same vectors; the angular pair uses a form that is
// cheaper per vector (ang_apply), so angular results agree with single
// products to rounding.
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <type_traits>

namespace rpy {
namespace {

constexpr int kBlockM = 256;   // threads per workgroup
constexpr int kFold = 256;     // sources between Neumaier folds: the single-vector kernel's tile
constexpr int kTileBytes = 32768;

// Sources per LDS tile: the largest of 256, 128, 64 whose records fit in
// 32 KiB (position plus NR records per vector), so that several workgroups
// share a CU.  kFold is a multiple of it, so the fold points do not move.
template <typename Real, int NV, int NR>
constexpr int tile_sources() {
    constexpr int per = (int)sizeof(vec4_t<Real>) * (1 + NR * NV);
    return per * 256 <= kTileBytes ? 256 : (per * 128 <= kTileBytes ? 128 : 64);
}

// ---------------------------------------------------------------------------
// pair geometry and its application to one vector
// ---------------------------------------------------------------------------
// The angular pair in the direct form of the blocks, with the separation
// prescaled by G (e = G d) so that the coupling terms G (T x d) and
// G (F x d) are plain cross products with e:
//   U += A F + B (d.F) d + T x e,   W += D T + E (d.T) d + F x e.
// Per vector that is 32 instructions (two dot products, two scalings, four
// multiply-adds per output component) against 35 for the regrouped form of
// the single-vector kernel, whose savings are per pair (the coefficients
// B, D, E, A and e cost 6 more per pair here); from two vectors on, this form
// is the cheaper one.  The overlap branch only changes the coefficients.
template <typename Real>
struct AngGeom {
    Real dx, dy, dz;   // d = X_i - X_j
    Real ex, ey, ez;   // e = G d
    Real A, B, D, E;
};

template <typename Real>
__device__ __forceinline__ AngGeom<Real> ang_geom(Real xi, Real yi, Real zi, const vec4_t<Real> &p,
                                                  const PairConst<Real> &c) {
    AngGeom<Real> q;
    q.dx = xi - p.x;
    q.dy = yi - p.y;
    q.dz = zi - p.z;
    const Real r2 = fma(q.dx, q.dx, fma(q.dy, q.dy, q.dz * q.dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    Real G = ri * ri2;
    const Real ri5 = G * ri2;
    q.A = fma(c.two_a2_3, G, ri);
    q.B = fma(c.m_two_a2, ri5, G);
    q.D = Real(-0.5) * G;
    q.E = Real(1.5) * ri5;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        // overlap branch; at r = 0 (self pair) it gives the Stokes drag
        const Real rs = sel_pos(r2, ri);
        const Real r = r2 * rs;
        q.A = fma(c.nA1, r, c.nA0);
        q.B = c.nB * rs;
        G = fma(c.nG1, r, c.nG0);
        q.D = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
        q.E = fma(c.nE_1, rs, c.nE1 * r);
    }
    q.ex = G * q.dx;
    q.ey = G * q.dy;
    q.ez = G * q.dz;
    return q;
}

// One vector's force f and torque t (the .w slots unused).
template <typename Real>
__device__ __forceinline__ void ang_apply(const AngGeom<Real> &q, const vec4_t<Real> &f, const vec4_t<Real> &t,
                                          Real *u, Real *w) {
    const Real dF = fma(q.dx, f.x, fma(q.dy, f.y, q.dz * f.z));
    const Real dT = fma(q.dx, t.x, fma(q.dy, t.y, q.dz * t.z));
    const Real sB = q.B * dF;
    const Real sE = q.E * dT;
    // U += A F + B (d.F) d + T x e
    u[0] = fma(q.A, f.x, fma(sB, q.dx, fma(t.y, q.ez, fma(-t.z, q.ey, u[0]))));
    u[1] = fma(q.A, f.y, fma(sB, q.dy, fma(t.z, q.ex, fma(-t.x, q.ez, u[1]))));
    u[2] = fma(q.A, f.z, fma(sB, q.dz, fma(t.x, q.ey, fma(-t.y, q.ex, u[2]))));
    // W += D T + E (d.T) d + F x e
    w[0] = fma(q.D, t.x, fma(sE, q.dx, fma(f.y, q.ez, fma(-f.z, q.ey, w[0]))));
    w[1] = fma(q.D, t.y, fma(sE, q.dy, fma(f.z, q.ex, fma(-f.x, q.ez, w[1]))));
    w[2] = fma(q.D, t.z, fma(sE, q.dz, fma(f.x, q.ey, fma(-f.y, q.ex, w[2]))));
}

template <typename Real>
struct LinGeom {
    Real dx, dy, dz, A, B;   // U += A F + B (d.F) d
};

template <typename Real>
__device__ __forceinline__ LinGeom<Real> lin_geom(Real xi, Real yi, Real zi, const vec4_t<Real> &p,
                                                  const PairConst<Real> &c) {
    LinGeom<Real> q;
    q.dx = xi - p.x;
    q.dy = yi - p.y;
    q.dz = zi - p.z;
    const Real r2 = fma(q.dx, q.dx, fma(q.dy, q.dy, q.dz * q.dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    const Real ri3 = ri * ri2;
    q.A = fma(c.two_a2_3, ri3, ri);
    q.B = fma(c.m_two_a2, ri3 * ri2, ri3);
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        const Real rs = sel_pos(r2, ri);
        q.A = fma(c.nA1, r2 * rs, c.nA0);
        q.B = c.nB * rs;
    }
    return q;
}

template <typename Real>
__device__ __forceinline__ void lin_apply(const LinGeom<Real> &q, const vec4_t<Real> &f, Real *u) {
    const Real dF = fma(q.dx, f.x, fma(q.dy, f.y, q.dz * f.z));
    const Real s = q.B * dF;
    u[0] = fma(q.A, f.x, fma(s, q.dx, u[0]));
    u[1] = fma(q.A, f.y, fma(s, q.dy, u[1]));
    u[2] = fma(q.A, f.z, fma(s, q.dz, u[2]));
}

// ---------------------------------------------------------------------------
// pair kernel over NV vectors
// ---------------------------------------------------------------------------
// frc / trq: staged vectors, vector v at frc + v * n.  Vectors of this
// launch: v0 + blockIdx.z * NV + j, j < NV (all exist).
// part layout: [split][vector][component][n], FP32 with 2*NC components per
// vector (sums, then compensations), FP64 with NC.
template <typename Real, bool ANG, int NV, int TM>
__global__ void __launch_bounds__(kBlockM)
multi_pair_kernel(const vec4_t<Real> *__restrict__ pos, const vec4_t<Real> *__restrict__ frc,
                  const vec4_t<Real> *__restrict__ trq, int n, int nrhs, int v0, int split_len, PairConst<Real> c,
                  Real *__restrict__ part) {
    using R4 = vec4_t<Real>;
    constexpr int NC = ANG ? 6 : 3;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int NR = ANG ? 2 : 1;          // records per vector and source (F, T or F)
    constexpr int TS = tile_sources<Real, NV, NR>();
    static_assert(kFold % TS == 0, "fold points must fall on tile ends");
    __shared__ R4 sp[TS];
    __shared__ R4 sv[NV][NR][TS];

    const int tid = threadIdx.x;
    const int tbase = blockIdx.x * (kBlockM * TM);
    const int vb = v0 + blockIdx.z * NV;
    Real xi[TM], yi[TM], zi[TM];
    Real acc[TM][NV][NC];
    Real sum[TM][NV][COMP ? NC : 1], cmp[TM][NV][COMP ? NC : 1];
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int idx = min(tbase + m * kBlockM + tid, n - 1);
        const R4 p = pos[idx];
        xi[m] = p.x;
        yi[m] = p.y;
        zi[m] = p.z;
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                acc[m][j][k] = Real(0);
                if constexpr (COMP) {
                    sum[m][j][k] = Real(0);
                    cmp[m][j][k] = Real(0);
                }
            }
    }

    const int s_begin = blockIdx.y * split_len;
    const int s_end = min(n, s_begin + split_len);
    const size_t nn = (size_t)n;
    for (int t0 = s_begin; t0 < s_end; t0 += TS) {
        const int src = t0 + tid;
        if (tid < TS && src < s_end) {
            sp[tid] = pos[src];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                sv[j][0][tid] = frc[(size_t)(vb + j) * nn + src];
                if constexpr (ANG) sv[j][1][tid] = trq[(size_t)(vb + j) * nn + src];
            }
        }
        __syncthreads();
        const int cnt = min(TS, s_end - t0);
        for (int q = 0; q < cnt; ++q) {
            const R4 p = sp[q];
            if constexpr (ANG) {
                AngGeom<Real> g[TM];
#pragma unroll
                for (int m = 0; m < TM; ++m) g[m] = ang_geom<Real>(xi[m], yi[m], zi[m], p, c);
#pragma unroll
                for (int j = 0; j < NV; ++j) {
                    const R4 f = sv[j][0][q], t = sv[j][1][q];
#pragma unroll
                    for (int m = 0; m < TM; ++m) ang_apply<Real>(g[m], f, t, acc[m][j], acc[m][j] + 3);
                }
            } else {
                LinGeom<Real> g[TM];
#pragma unroll
                for (int m = 0; m < TM; ++m) g[m] = lin_geom<Real>(xi[m], yi[m], zi[m], p, c);
#pragma unroll
                for (int j = 0; j < NV; ++j) {
                    const R4 f = sv[j][0][q];
#pragma unroll
                    for (int m = 0; m < TM; ++m) lin_apply<Real>(g[m], f, acc[m][j]);
                }
            }
        }
        __syncthreads();
        // fold every kFold sources from the split's start, and at its end
        if constexpr (COMP) {
            if ((t0 + TS - s_begin) % kFold == 0 || t0 + TS >= s_end) {
#pragma unroll
                for (int m = 0; m < TM; ++m)
#pragma unroll
                    for (int j = 0; j < NV; ++j)
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            neumaier(sum[m][j][k], cmp[m][j][k], acc[m][j][k]);
                            acc[m][j][k] = Real(0);
                        }
            }
        }
    }

    constexpr int PC = COMP ? 2 * NC : NC;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int idx = tbase + m * kBlockM + tid;
        if (idx < n) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                Real *base = part + ((size_t)blockIdx.y * nrhs + (vb + j)) * PC * nn;
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    if constexpr (COMP) {
                        base[(size_t)k * nn + idx] = sum[m][j][k];
                        base[(size_t)(NC + k) * nn + idx] = cmp[m][j][k];
                    } else {
                        base[(size_t)k * nn + idx] = acc[m][j][k];
                    }
                }
            }
        }
    }
}

// Sum over splits of vector blockIdx.z, component blockIdx.y, target i, in
// the order and arithmetic of the single-vector reduction; writes
// lin[v * ostride + 3 i + c] (ang likewise for c >= 3).
template <typename Real, typename Tout, bool ANG>
__global__ void __launch_bounds__(256)
multi_reduce_kernel(const Real *__restrict__ part, int n_split, int n, int nrhs, double k, int64_t ostride,
                    Tout *__restrict__ lin, Tout *__restrict__ ang) {
    constexpr int NC = ANG ? 6 : 3;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int PC = COMP ? 2 * NC : NC;
    constexpr int U = 4;
    const int c = blockIdx.y;
    const int v = blockIdx.z;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (c >= 3 && !ang)) return;
    const size_t nn = (size_t)n;
    const size_t stride = (size_t)nrhs * PC * nn;   // between splits
    const Real *p0 = part + ((size_t)v * PC + c) * nn + i;
    Tout val;
    if constexpr (COMP) {
        const Real *p1 = p0 + (size_t)NC * nn;
        float s = 0.f, cp = 0.f, extra = 0.f;
        int q = 0;
        for (; q + U <= n_split; q += U) {
            float x[U], e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x[u] = p0[(size_t)(q + u) * stride];
                e[u] = p1[(size_t)(q + u) * stride];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                neumaier(s, cp, x[u]);
                extra += e[u];
            }
        }
        for (; q < n_split; ++q) {
            neumaier(s, cp, (float)p0[(size_t)q * stride]);
            extra += (float)p1[(size_t)q * stride];
        }
        val = (Tout)(k * ((double)s + ((double)cp + (double)extra)));
    } else {
        double s = 0.0;
        int q = 0;
        for (; q + U <= n_split; q += U) {
            double x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = (double)p0[(size_t)(q + u) * stride];
#pragma unroll
            for (int u = 0; u < U; ++u) s += x[u];
        }
        for (; q < n_split; ++q) s += (double)p0[(size_t)q * stride];
        val = (Tout)(k * s);
    }
    const size_t o = (size_t)v * (size_t)ostride + 3 * (size_t)i;
    if (c < 3)
        lin[o + c] = val;
    else
        ang[o + (c - 3)] = val;
}

// AoS nrhs x n x 3 (or NULL = zeros) -> vec4 [vector][n]
template <typename Real>
__global__ void multi_stage_kernel(const Real *__restrict__ in, int64_t total, vec4_t<Real> *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    vec4_t<Real> v;
    if (in) {
        v.x = in[3 * e];
        v.y = in[3 * e + 1];
        v.z = in[3 * e + 2];
    } else {
        v.x = v.y = v.z = Real(0);
    }
    v.w = Real(0);
    out[e] = v;
}

template <typename Real, bool ANG, int NV>
hipError_t launch_multi_nv(const vec4_t<Real> *pos, const vec4_t<Real> *f, const vec4_t<Real> *t, int64_t n,
                           int nrhs, int v0, int groups, int tm, int n_split, int split_len,
                           const PairConst<Real> &pc, Real *part, hipStream_t st) {
    const int64_t tpb = (int64_t)kBlockM * tm;
    dim3 grid((unsigned)((n + tpb - 1) / tpb), (unsigned)n_split, (unsigned)groups);
    if (tm == 1)
        hipLaunchKernelGGL((multi_pair_kernel<Real, ANG, NV, 1>), grid, dim3(kBlockM), 0, st, pos, f, t, (int)n,
                           nrhs, v0, split_len, pc, part);
    else
        hipLaunchKernelGGL((multi_pair_kernel<Real, ANG, NV, 2>), grid, dim3(kBlockM), 0, st, pos, f, t, (int)n,
                           nrhs, v0, split_len, pc, part);
    return hipGetLastError();
}

// Vectors per group: 4 with the angular blocks, 4 without.
template <bool ANG>
constexpr int nv_max() {
    return 4;
}

template <typename Real, bool ANG>
hipError_t launch_multi(const vec4_t<Real> *pos, const vec4_t<Real> *f, const vec4_t<Real> *t, int64_t n, int nrhs,
                        int tm, int n_split, const PairConst<Real> &pc, Real *part, hipStream_t st) {
    constexpr int NVM = nv_max<ANG>();
    int64_t split_len = (n + n_split - 1) / n_split;
    split_len = (split_len + kFold - 1) / kFold * kFold;
    const int full = nrhs / NVM, rest = nrhs % NVM;
    hipError_t e = hipSuccess;
    if (full > 0) e = launch_multi_nv<Real, ANG, NVM>(pos, f, t, n, nrhs, 0, full, tm, n_split, (int)split_len, pc,
                                                      part, st);
    if (e != hipSuccess || rest == 0) return e;
    const int v0 = full * NVM;
    switch (rest) {
        case 1: return launch_multi_nv<Real, ANG, 1>(pos, f, t, n, nrhs, v0, 1, tm, n_split, (int)split_len, pc, part, st);
        case 2: return launch_multi_nv<Real, ANG, 2>(pos, f, t, n, nrhs, v0, 1, tm, n_split, (int)split_len, pc, part, st);
        default: return launch_multi_nv<Real, ANG, 3>(pos, f, t, n, nrhs, v0, 1, tm, n_split, (int)split_len, pc, part, st);
    }
}

}  // namespace

int multi_targets_per_lane(const rpy_solver *s, bool ang) {
    if (s->multi_tm > 0) return s->multi_tm;
    // measured at N = 65,536: one target per lane for the float32 angular
    // product (two would need 208 VGPRs), two elsewhere
    return (ang && s->dtype == RPY_F32) ? 1 : 2;
}

// nrhs products M [F_r; T_r] with the vectors already staged in s->f (and
// s->t) as [vector][n] vec4 arrays, with the source splits of the
// single-vector product.
template <typename Real, typename Tout>
rpy_status apply_staged_multi(rpy_solver *s, bool ang, int nrhs, Tout *lin, Tout *ang_out, int64_t ostride,
                              hipStream_t st) {
    const int64_t n = s->n;
    if (s->pse) {
        for (int r = 0; r < nrhs; ++r) {
            rpy_status rs = apply_pse<Real, Tout>(s, s->f.as<vec4_t<Real>>() + (size_t)r * n, lin + (size_t)r * ostride, st);
            if (rs != RPY_OK) return rs;
        }
        return RPY_OK;
    }
    if (s->wall) {
        // one wall product per vector
        for (int r = 0; r < nrhs; ++r) {
            rpy_status rs = apply_wall<Real, Tout>(s, ang, s->f.as<vec4_t<Real>>() + (size_t)r * n,
                                                   ang ? s->t.as<vec4_t<Real>>() + (size_t)r * n : nullptr,
                                                   lin + (size_t)r * ostride,
                                                   ang_out ? ang_out + (size_t)r * ostride : nullptr, st);
            if (rs != RPY_OK) return rs;
        }
        return RPY_OK;
    }
    const int splits = splits_for(s, ang);
    const int pc_count = (ang ? 6 : 3) * (std::is_same<Real, float>::value ? 2 : 1);
    HIP_TRY(s, s->part.ensure((size_t)splits * nrhs * pc_count * n * sizeof(Real)));
    const PairConst<Real> pc = make_pair_const<Real>(s->radius);
    const auto *pos = s->pos.as<vec4_t<Real>>();
    const auto *f = s->f.as<vec4_t<Real>>();
    const auto *t = s->t.as<vec4_t<Real>>();
    const int tm = multi_targets_per_lane(s, ang);
    hipEvent_t e0 = timing_begin(s, RPY_KERNEL_PAIR_MULTI, (double)n * (double)n * nrhs);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    if (ang)
        HIP_TRY(s, (launch_multi<Real, true>(pos, f, t, n, nrhs, tm, splits, pc, s->part.as<Real>(), st)));
    else
        HIP_TRY(s, (launch_multi<Real, false>(pos, f, nullptr, n, nrhs, tm, splits, pc, s->part.as<Real>(), st)));
    if (hipEvent_t e1 = timing_end(s, RPY_KERNEL_PAIR_MULTI)) HIP_TRY(s, hipEventRecord(e1, st));
    dim3 rgrid((unsigned)((n + 255) / 256), ang ? 6 : 3, (unsigned)nrhs);
    if (ang)
        hipLaunchKernelGGL((multi_reduce_kernel<Real, Tout, true>), rgrid, dim3(256), 0, st, s->part.as<Real>(),
                           splits, (int)n, nrhs, k_factor(s), ostride, lin, ang_out);
    else
        hipLaunchKernelGGL((multi_reduce_kernel<Real, Tout, false>), rgrid, dim3(256), 0, st, s->part.as<Real>(),
                           splits, (int)n, nrhs, k_factor(s), ostride, lin, ang_out);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

template <typename Real>
rpy_status stage_multi(rpy_solver *s, const Real *F, const Real *T, int nrhs, bool ang, hipStream_t st) {
    const size_t elt = sizeof(vec4_t<Real>);
    const int64_t total = (int64_t)nrhs * s->n;
    HIP_TRY(s, s->f.ensure(elt * total));
    hipLaunchKernelGGL((multi_stage_kernel<Real>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, F, total,
                       s->f.as<vec4_t<Real>>());
    HIP_TRY(s, hipGetLastError());
    if (ang) {
        HIP_TRY(s, s->t.ensure(elt * total));
        hipLaunchKernelGGL((multi_stage_kernel<Real>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, T,
                           total, s->t.as<vec4_t<Real>>());
        HIP_TRY(s, hipGetLastError());
    }
    return RPY_OK;
}

template rpy_status apply_staged_multi<float, float>(rpy_solver *, bool, int, float *, float *, int64_t,
                                                     hipStream_t);
template rpy_status apply_staged_multi<float, double>(rpy_solver *, bool, int, double *, double *, int64_t,
                                                      hipStream_t);
template rpy_status apply_staged_multi<double, double>(rpy_solver *, bool, int, double *, double *, int64_t,
                                                       hipStream_t);
template rpy_status stage_multi<float>(rpy_solver *, const float *, const float *, int, bool, hipStream_t);
template rpy_status stage_multi<double>(rpy_solver *, const double *, const double *, int, bool, hipStream_t);

}  // namespace rpy

using namespace rpy;

extern "C" {

rpy_status rpy_mdot_multi(rpy_solver *s, const void *forces, const void *torques, int nrhs, void *lin_out,
                          void *ang_out, void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(s, RPY_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    if (!forces && !torques) return fail(s, RPY_ERR_INVALID_ARG, "need forces, torques or both");
    if (!lin_out) return fail(s, RPY_ERR_INVALID_ARG, "linear output pointer is NULL");
    if ((torques || ang_out) && !s->angular)
        return fail(s, RPY_ERR_ANGULAR_DISABLED, "torques / angular output need include_angular");
    if ((int64_t)nrhs * s->n > (int64_t)INT32_MAX)
        return fail(s, RPY_ERR_INVALID_ARG, "nrhs * n must stay below 2^31");
    const bool am = torques != nullptr || ang_out != nullptr;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64) {
        r = stage_multi<double>(s, static_cast<const double *>(forces), static_cast<const double *>(torques), nrhs, am,
                                st);
        if (r != RPY_OK) return r;
        return apply_staged_multi<double, double>(s, am, nrhs, static_cast<double *>(lin_out),
                                                  static_cast<double *>(ang_out), 3 * s->n, st);
    }
    r = stage_multi<float>(s, static_cast<const float *>(forces), static_cast<const float *>(torques), nrhs, am, st);
    if (r != RPY_OK) return r;
    return apply_staged_multi<float, float>(s, am, nrhs, static_cast<float *>(lin_out), static_cast<float *>(ang_out),
                                            3 * s->n, st);
}

rpy_status rpy_set_multi_config(rpy_solver *s, int targets_per_lane) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if (targets_per_lane < 0 || targets_per_lane > 2)
        return fail(s, RPY_ERR_INVALID_ARG, "targets_per_lane must be 0 (automatic), 1 or 2");
    s->multi_tm = targets_per_lane;
    return RPY_OK;
}

}  // extern "C"

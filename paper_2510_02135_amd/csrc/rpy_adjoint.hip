// Adjoint of the RPY mobility product (an addition beside the paper's
// method; forward operator: eq. (block_mobility) with the generalised RPY
// pair tensors of the open-boundary N-body solver, Sec. 3.5).
//
// For cotangents g = (g_U, g_W) of a scalar loss L with respect to the Mdot
// outputs, and inputs s = (F, T):
//   dL/dF, dL/dT = M g                  (the grand mobility is symmetric)
//   dL/dX_k      = sum_j [ grad Phi(g_k, s_j; d) - grad Phi(g_j, s_k; -d) ],
//                  d = X_k - X_j,  Phi(g, s; r) = g^T M(r) s.
// With the k-unit scalar functions of rpy_pair.hpp (A, B, G, D, E and
// X_r := X'(r)/r, so that X'(r) rhat = X_r d) the pair term is
//   dX += d [ A_r (gUk.Fj + gUj.Fk) + B_r ((d.gUk)(d.Fj) + (d.gUj)(d.Fk))
//            + G_r (gUk.(Tj x d) + gWk.(Fj x d) - gUj.(Tk x d) - gWj.(Fk x d))
//            + D_r (gWk.Tj + gWj.Tk) + E_r ((d.gWk)(d.Tj) + (d.gWj)(d.Tk)) ]
//       + B [ (d.Fj) gUk + (d.gUk) Fj + (d.Fk) gUj + (d.gUj) Fk ]
//       + G [ gUk x Tj + gWk x Fj - gUj x Tk - gWj x Fk ]
//       + E [ (d.Tj) gWk + (d.gWk) Tj + (d.Tk) gWj + (d.gWj) Tk ]
// A zero-distance pair (the self pair, or coincident particles where M is
// not differentiable) contributes nothing to dX.
//
// Same decomposition as the forward pair kernel: target blocks x source
// splits, LDS source tiles (position, F, g_U [, T, g_W]), fp32 in-tile sums
// folded into Neumaier pairs per tile, fp64 plain sums.
#include "rpy_adjoint.hpp"
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <cmath>

namespace rpy {
namespace {

constexpr int kBlock = 256;
constexpr int kTile = 256;
// automatic choice of the symmetric mode: from this N on (large N runs in
// slabs whose partials fit a fixed workspace)
constexpr int64_t kSymAdjointMinN = 4096;

template <typename Real, bool ANG>
__global__ void __launch_bounds__(kBlock)
adjoint_kernel(const vec4_t<Real> *__restrict__ pos, const vec4_t<Real> *__restrict__ frc,
               const vec4_t<Real> *__restrict__ gu, const vec4_t<Real> *__restrict__ trq,
               const vec4_t<Real> *__restrict__ gw, int n, int split_len, PairConst<Real> c, Real *__restrict__ part) {
    using R4 = vec4_t<Real>;
    constexpr int NC = ANG ? 9 : 6;
    constexpr bool COMP = std::is_same<Real, float>::value;
    __shared__ R4 sp[kTile], sf[kTile], sg[kTile];
    __shared__ R4 st[ANG ? kTile : 1], sh[ANG ? kTile : 1];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kBlock + tid;
    const int ic = min(i, n - 1);
    Tgt<Real, ANG> k;
    {
        const R4 p = pos[ic], f = frc[ic], g = gu[ic];
        k.x = p.x; k.y = p.y; k.z = p.z;
        k.fx = f.x; k.fy = f.y; k.fz = f.z;
        k.gx = g.x; k.gy = g.y; k.gz = g.z;
        if constexpr (ANG) {
            const R4 t = trq[ic], h = gw[ic];
            k.tx = t.x; k.ty = t.y; k.tz = t.z;
            k.hx = h.x; k.hy = h.y; k.hz = h.z;
        }
    }
    Real acc[NC], sum[COMP ? NC : 1], cmp[COMP ? NC : 1];
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = Real(0);
    if constexpr (COMP) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            sum[q] = Real(0);
            cmp[q] = Real(0);
        }
    }
    const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
    const int s_begin = blockIdx.y * split_len;
    const int s_end = min(n, s_begin + split_len);
    for (int t0 = s_begin; t0 < s_end; t0 += kTile) {
        const int j = t0 + tid;
        if (j < s_end) {
            sp[tid] = pos[j];
            sf[tid] = frc[j];
            sg[tid] = gu[j];
            if constexpr (ANG) {
                st[tid] = trq[j];
                sh[tid] = gw[j];
            }
        }
        __syncthreads();
        const int cnt = min(kTile, s_end - t0);
        for (int q = 0; q < cnt; ++q) {
            R4 a4 = zero4, b4 = zero4;
            if constexpr (ANG) {
                a4 = st[q];
                b4 = sh[q];
            }
            adj_interact<Real, ANG>(k, sp[q], sf[q], sg[q], a4, b4, c, acc);
        }
        __syncthreads();
        if constexpr (COMP) {
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                neumaier(sum[q], cmp[q], acc[q]);
                acc[q] = Real(0);
            }
        }
    }
    if (i < n) {
        const size_t nn = (size_t)n;
        Real *base = part + (size_t)blockIdx.y * (COMP ? 2 * NC : NC) * nn;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if constexpr (COMP) {
                base[(size_t)q * nn + i] = sum[q];
                base[(size_t)(NC + q) * nn + i] = cmp[q];
            } else {
                base[(size_t)q * nn + i] = acc[q];
            }
        }
    }
}

template <typename Real, int NV>
__global__ void reduce3_kernel(const Real *__restrict__ part, int n_split, int n, double k, Real *o0, Real *o1,
                               Real *o2) {
    constexpr int NC = 3 * NV;
    constexpr bool COMP = std::is_same<Real, float>::value;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t nn = (size_t)n;
    const size_t stride = (size_t)(COMP ? 2 * NC : NC) * nn;
    Real *outs[3] = {o0, o1, o2};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Real *o = outs[c / 3];
        if (!o) continue;
        double v;
        if constexpr (COMP) {
            float s = 0.f, cp = 0.f, extra = 0.f;
            for (int q = 0; q < n_split; ++q) {
                neumaier(s, cp, (float)part[q * stride + (size_t)c * nn + i]);
                extra += (float)part[q * stride + (size_t)(NC + c) * nn + i];
            }
            v = (double)s + ((double)cp + (double)extra);
        } else {
            v = 0.0;
            for (int q = 0; q < n_split; ++q) v += (double)part[q * stride + (size_t)c * nn + i];
        }
        o[3 * (size_t)i + (c % 3)] = (Real)(k * v);
    }
}

template <typename Real>
rpy_status backward_typed(rpy_solver *s, const Real *F, const Real *T, const Real *gl, const Real *ga, Real *gp,
                          Real *gf, Real *gt, hipStream_t st) {
    const int64_t n = s->n;
    const bool ang = s->angular && (T || ga || gt);
    const size_t elt = sizeof(vec4_t<Real>);
    // staging: F, g_U (+ T, g_W) as vec4 arrays in one buffer
    const int nvec = ang ? 4 : 2;
    HIP_TRY(s, s->lz_vec.ensure(elt * n * nvec));
    auto *v4 = s->lz_vec.as<vec4_t<Real>>();
    vec4_t<Real> *f4 = v4, *g4 = v4 + n, *t4 = ang ? v4 + 2 * n : nullptr, *h4 = ang ? v4 + 3 * n : nullptr;
    HIP_TRY(s, (launch_stage_vec<Real, Real>(F, n, f4, st)));
    HIP_TRY(s, (launch_stage_vec<Real, Real>(gl, n, g4, st)));
    if (ang) {
        HIP_TRY(s, (launch_stage_vec<Real, Real>(T, n, t4, st)));
        HIP_TRY(s, (launch_stage_vec<Real, Real>(ga, n, h4, st)));
    }
    // the symmetric mode evaluates each unordered pair once (rpy_sym.hip)
    const bool sym = s->adjoint_mode == 2 || (s->adjoint_mode == 0 && n >= kSymAdjointMinN);
    if (sym) return adjoint_sym<Real>(s, ang, f4, g4, t4, h4, gp, gf, gt, st);
    const int nc = (ang ? 9 : 6) * (std::is_same<Real, float>::value ? 2 : 1);
    const int64_t tblocks = (n + kBlock - 1) / kBlock;
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + tblocks - 1) / tblocks,
                                                                   (n + kTile - 1) / kTile));
    HIP_TRY(s, s->part.ensure((size_t)splits * nc * n * sizeof(Real)));
    int64_t split_len = (n + splits - 1) / splits;
    split_len = (split_len + kTile - 1) / kTile * kTile;
    const PairConst<Real> pc = make_pair_const<Real>(s->radius);
    dim3 grid((unsigned)tblocks, (unsigned)splits);
    hipEvent_t e0 = timing_begin(s, RPY_KERNEL_ADJOINT, (double)n * (double)n);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    if (ang)
        hipLaunchKernelGGL((adjoint_kernel<Real, true>), grid, dim3(kBlock), 0, st, s->pos.as<vec4_t<Real>>(), f4, g4,
                           t4, h4, (int)n, (int)split_len, pc, s->part.as<Real>());
    else
        hipLaunchKernelGGL((adjoint_kernel<Real, false>), grid, dim3(kBlock), 0, st, s->pos.as<vec4_t<Real>>(), f4, g4,
                           nullptr, nullptr, (int)n, (int)split_len, pc, s->part.as<Real>());
    HIP_TRY(s, hipGetLastError());
    if (hipEvent_t e1 = timing_end(s, RPY_KERNEL_ADJOINT)) HIP_TRY(s, hipEventRecord(e1, st));
    const dim3 rg((unsigned)((n + 255) / 256));
    if (ang)
        hipLaunchKernelGGL((reduce3_kernel<Real, 3>), rg, dim3(256), 0, st, s->part.as<Real>(), splits, (int)n,
                           k_factor(s), gp, gf, gt);
    else
        hipLaunchKernelGGL((reduce3_kernel<Real, 2>), rg, dim3(256), 0, st, s->part.as<Real>(), splits, (int)n,
                           k_factor(s), gp, gf, (Real *)nullptr);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

}  // namespace
}  // namespace rpy

extern "C" rpy_status rpy_mdot_backward(rpy_solver *s, const void *forces, const void *torques, const void *grad_lin,
                                        const void *grad_ang, void *grad_pos, void *grad_forces, void *grad_torques,
                                        void *hip_stream) {
    using namespace rpy;
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!forces && !torques) return fail(s, RPY_ERR_INVALID_ARG, "need forces, torques or both");
    if (!grad_lin && !grad_ang) return fail(s, RPY_ERR_INVALID_ARG, "need at least one cotangent");
    if (!grad_pos && !grad_forces && !grad_torques) return fail(s, RPY_ERR_INVALID_ARG, "no gradient requested");
    if ((torques || grad_ang || grad_torques) && !s->angular)
        return fail(s, RPY_ERR_ANGULAR_DISABLED, "torques / angular cotangents need include_angular");
    if (s->wall || s->pse)
        return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY, "the adjoint is built for open boundaries only");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (s->dtype == RPY_F64)
        return backward_typed<double>(s, static_cast<const double *>(forces), static_cast<const double *>(torques),
                                      static_cast<const double *>(grad_lin), static_cast<const double *>(grad_ang),
                                      static_cast<double *>(grad_pos), static_cast<double *>(grad_forces),
                                      static_cast<double *>(grad_torques), st);
    return backward_typed<float>(s, static_cast<const float *>(forces), static_cast<const float *>(torques),
                                 static_cast<const float *>(grad_lin), static_cast<const float *>(grad_ang),
                                 static_cast<float *>(grad_pos), static_cast<float *>(grad_forces),
                                 static_cast<float *>(grad_torques), st);
}

extern "C" rpy_status rpy_set_adjoint_mode(rpy_solver *s, int mode) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if (mode < 0 || mode > 2) return rpy::fail(s, RPY_ERR_INVALID_ARG, "adjoint mode must be 0, 1 or 2");
    s->adjoint_mode = mode;
    return RPY_OK;
}

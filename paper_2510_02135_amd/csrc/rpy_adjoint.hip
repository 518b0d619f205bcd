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
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <algorithm>
#include <cmath>

namespace rpy {
namespace {

constexpr int kBlock = 256;
constexpr int kTile = 256;

template <typename Real>
__device__ __forceinline__ Real dot3(Real ax, Real ay, Real az, Real bx, Real by, Real bz) {
    return fma(ax, bx, fma(ay, by, az * bz));
}

// Target-side data of one lane.
template <typename Real, bool ANG>
struct Tgt {
    Real x, y, z;
    Real fx, fy, fz;
    Real gx, gy, gz;          // g_U
    Real tx, ty, tz;          // T      (ANG)
    Real hx, hy, hz;          // g_W    (ANG)
};

// Output accumulator layout: [0..2] dX, [3..5] dF (= (M g)_U), [6..8] dT.
template <typename Real, bool ANG>
__device__ __forceinline__ void adj_interact(const Tgt<Real, ANG> &k, const vec4_t<Real> &sp, const vec4_t<Real> &sf,
                                             const vec4_t<Real> &sg, const vec4_t<Real> &st, const vec4_t<Real> &sh,
                                             const PairConst<Real> &c, Real *acc) {
    const Real dx = k.x - sp.x, dy = k.y - sp.y, dz = k.z - sp.z;
    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const Real ri = rsq(r2);
    const Real ri2 = ri * ri;
    const Real ri3 = ri * ri2;
    const Real ri5 = ri3 * ri2;
    const Real ri7 = ri5 * ri2;
    // far branch; c.m_two_a2 = -2a^2, c.two_a2_3 = 2a^2/3
    Real A = fma(c.two_a2_3, ri3, ri);
    Real B = fma(c.m_two_a2, ri5, ri3);
    Real Ar = fma(c.m_two_a2, ri5, -ri3);                    // -1/r^3 - 2a^2/r^5
    Real Br = fma(Real(-5) * c.m_two_a2, ri7, Real(-3) * ri5);  // -3/r^5 + 10a^2/r^7
    Real G = ri3, Gg = ri3, Gr = Real(-3) * ri5;
    Real D = Real(-0.5) * ri3, Dr = Real(1.5) * ri5;
    Real E = Real(1.5) * ri5, Er = Real(-7.5) * ri7;
    if (__builtin_expect(r2 < c.four_a2, 0)) {
        const Real rs = r2 > Real(0) ? ri : Real(0);
        const Real r = r2 * rs;
        const Real rs3 = rs * rs * rs;
        A = fma(c.nA1, r, c.nA0);
        Ar = c.nA1 * rs;
        B = c.nB * rs;
        Br = -c.nB * rs3;
        if constexpr (ANG) {
            G = fma(c.nG1, r, c.nG0);
            Gg = r2 > Real(0) ? G : Real(0);
            Gr = c.nG1 * rs;
            D = fma(fma(c.nD3, r * r, c.nD1), r, c.nD0);
            Dr = fma(c.nD1, rs, Real(3) * c.nD3 * r);
            E = fma(c.nE_1, rs, c.nE1 * r);
            Er = fma(-c.nE_1, rs3, c.nE1 * rs);
        }
    }
    // dot products shared by the terms
    const Real dFj = dot3(dx, dy, dz, sf.x, sf.y, sf.z);
    const Real dgj = dot3(dx, dy, dz, sg.x, sg.y, sg.z);
    const Real dFk = dot3(dx, dy, dz, k.fx, k.fy, k.fz);
    const Real dgk = dot3(dx, dy, dz, k.gx, k.gy, k.gz);
    const Real gkFj = dot3(k.gx, k.gy, k.gz, sf.x, sf.y, sf.z);
    const Real gjFk = dot3(sg.x, sg.y, sg.z, k.fx, k.fy, k.fz);
    Real S = fma(Ar, gkFj + gjFk, Br * fma(dgk, dFj, dgj * dFk));
    const Real b1 = B * dFj, b2 = B * dgk, b3 = B * dFk, b4 = B * dgj;
    Real ox = fma(b1, k.gx, fma(b2, sf.x, fma(b3, sg.x, b4 * k.fx)));
    Real oy = fma(b1, k.gy, fma(b2, sf.y, fma(b3, sg.y, b4 * k.fy)));
    Real oz = fma(b1, k.gz, fma(b2, sf.z, fma(b3, sg.z, b4 * k.fz)));
    // (M g)_U += A gUj + B (d.gUj) d
    acc[3] = fma(A, sg.x, fma(b4, dx, acc[3]));
    acc[4] = fma(A, sg.y, fma(b4, dy, acc[4]));
    acc[5] = fma(A, sg.z, fma(b4, dz, acc[5]));
    if constexpr (ANG) {
        // C = gUk x Tj + gWk x Fj - gUj x Tk - gWj x Fk, one fused chain per component
        const Real cx = fma(k.gy, st.z, fma(-k.gz, st.y, fma(k.hy, sf.z, fma(-k.hz, sf.y,
                        fma(-sg.y, k.tz, fma(sg.z, k.ty, fma(-sh.y, k.fz, sh.z * k.fy)))))));
        const Real cy = fma(k.gz, st.x, fma(-k.gx, st.z, fma(k.hz, sf.x, fma(-k.hx, sf.z,
                        fma(-sg.z, k.tx, fma(sg.x, k.tz, fma(-sh.z, k.fx, sh.x * k.fz)))))));
        const Real cz = fma(k.gx, st.y, fma(-k.gy, st.x, fma(k.hx, sf.y, fma(-k.hy, sf.x,
                        fma(-sg.x, k.ty, fma(sg.y, k.tx, fma(-sh.x, k.fy, sh.y * k.fx)))))));
        // gUk.(Tj x d) + gWk.(Fj x d) - gUj.(Tk x d) - gWj.(Fk x d) = d.C (cyclic triple products)
        const Real gsum = dot3(dx, dy, dz, cx, cy, cz);
        const Real dTj = dot3(dx, dy, dz, st.x, st.y, st.z);
        const Real dhj = dot3(dx, dy, dz, sh.x, sh.y, sh.z);
        const Real dTk = dot3(dx, dy, dz, k.tx, k.ty, k.tz);
        const Real dhk = dot3(dx, dy, dz, k.hx, k.hy, k.hz);
        const Real hkTj = dot3(k.hx, k.hy, k.hz, st.x, st.y, st.z);
        const Real hjTk = dot3(sh.x, sh.y, sh.z, k.tx, k.ty, k.tz);
        S = fma(Gr, gsum, fma(Dr, hkTj + hjTk, fma(Er, fma(dhk, dTj, dhj * dTk), S)));
        // G C
        const Real e1 = E * dTj, e2 = E * dhk, e3 = E * dTk, e4 = E * dhj;
        ox = fma(Gg, cx, fma(e1, k.hx, fma(e2, st.x, fma(e3, sh.x, fma(e4, k.tx, ox)))));
        oy = fma(Gg, cy, fma(e1, k.hy, fma(e2, st.y, fma(e3, sh.y, fma(e4, k.ty, oy)))));
        oz = fma(Gg, cz, fma(e1, k.hz, fma(e2, st.z, fma(e3, sh.z, fma(e4, k.tz, oz)))));
        // (M g)_U += G (gWj x d);  (M g)_W += G (gUj x d) + D gWj + E (d.gWj) d
        const Real hjx = sh.y * dz - sh.z * dy, hjy = sh.z * dx - sh.x * dz, hjz = sh.x * dy - sh.y * dx;
        const Real gjx = sg.y * dz - sg.z * dy, gjy = sg.z * dx - sg.x * dz, gjz = sg.x * dy - sg.y * dx;
        acc[3] = fma(G, hjx, acc[3]);
        acc[4] = fma(G, hjy, acc[4]);
        acc[5] = fma(G, hjz, acc[5]);
        acc[6] = fma(G, gjx, fma(D, sh.x, fma(e4, dx, acc[6])));
        acc[7] = fma(G, gjy, fma(D, sh.y, fma(e4, dy, acc[7])));
        acc[8] = fma(G, gjz, fma(D, sh.z, fma(e4, dz, acc[8])));
    }
    acc[0] = fma(S, dx, acc[0] + ox);
    acc[1] = fma(S, dy, acc[1] + oy);
    acc[2] = fma(S, dz, acc[2] + oz);
}

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

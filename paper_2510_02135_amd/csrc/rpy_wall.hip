// Pair kernel of the single-wall geometry (gfx950).
//
// With `single_wall` along z the N-body solver replaces the free-space RPY
// blocks by the Swan-Brady kernel (Sec. 3.5, "RPY kernels (NBody)"): the
// RPY construction applied to the Stokeslet plus Blake's image system for a
// no-slip plane at z = wallHeight.  Each block is the open-boundary block
// (overlap branch and self block included) plus an image part that depends
// on the in-plane separation (dx, dy), the two heights above the wall h_i,
// h_j and the radius.  Particles that overlap the wall are handled by the
// damping of the cited rollers paper (its Appendix A, as read here): every
// height is raised to max(h, a) and the matrix is multiplied on both sides
// by D = diag(d), d = min(max(h / a, 0), 1), linear and angular rows alike.
//
// Image part in units of k = 1/(8 pi eta), with R = (dx, dy, h_i + h_j),
// rho = |R|, e = R / rho, H_i = h_i / rho, H_j = h_j / rho, s = a / rho,
// z the wall normal and w = e x z:
//   U += (1/rho) [f1 F + (f2 (e.F) + f3 F_z) e + (f4 (e.F) + f5 F_z) z]
//     f1 = -1 - 2 H_i H_j - (2/3) s^2 (1 - 3 e_z^2) + (2/3) s^4 (1 - 5 e_z^2)
//     f2 = -1 + 6 H_i H_j + 2 s^2 (1 - 5 e_z^2) - (10/3) s^4 (1 - 7 e_z^2)
//     f3 = 2 H_j - 12 e_z H_i H_j - 4 s^2 e_z (1 - 5 e_z^2) + (20/3) s^4 e_z (2 - 7 e_z^2)
//     f4 = 2 H_j - (20/3) s^4 e_z
//     f5 = -4 H_j^2 - 4 s^2 e_z^2 - (4/3) s^4 (2 - 15 e_z^2)
//   W += (1/rho^2) [e x F + c2 (z x F) + (c3 (e.F) + c4 F_z) w]
//     c2 = 2 s^2 e_z - 2 H_j,  c3 = 10 s^2 e_z - 6 H_j,  c4 = 2 s^2 + 12 H_j e_z - 20 s^2 e_z^2
//   U += (torque) the transpose of the force -> rotation block of the
//        reversed pair (e' = (-e_x, -e_y, e_z), w' = -w, H_i in place of H_j)
//   W += (1/rho^3) [(7/2 - 6 e_z^2) T - (9/2)(e.T) e - 3 T_z z + 3 e_z T_z e + 6 e_z (e.T) z]
// The self pair is the same expression at R = (0, 0, 2 h_i).
//
// Work decomposition as in the ordinary pair kernel: target blocks of
// 256 x TM (TM targets per lane), source splits along grid.y, 256-source
// LDS tiles read by broadcast; the float32 mode folds per-tile sums into
// Neumaier pairs.  Source records carry (x, y, h, -) and the damped
// force (and torque); the epilogue multiplies a target's partials by d_i.
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"
#include "rpy_wall.hpp"

#include <algorithm>
#include <type_traits>

namespace rpy {
namespace {

constexpr int kWallBlock = 256;
constexpr int kWallTile = 256;

template <typename Real, bool ANG, int TM>
__global__ void __launch_bounds__(kWallBlock)
wall_pair_kernel(const vec4_t<Real> *__restrict__ pos, const vec4_t<Real> *__restrict__ frc,
                 const vec4_t<Real> *__restrict__ trq, int n, int split_len, PairConst<Real> c, WallConst<Real> wc,
                 Real *__restrict__ part) {
    using R4 = vec4_t<Real>;
    constexpr int NC = ANG ? 6 : 3;
    constexpr bool COMP = std::is_same<Real, float>::value;
    __shared__ R4 sp[kWallTile];
    __shared__ R4 sf[kWallTile];
    __shared__ R4 st[ANG ? kWallTile : 1];

    const int tid = threadIdx.x;
    const int tbase = blockIdx.x * (kWallBlock * TM);
    Real xi[TM], yi[TM], hi[TM], di[TM];
    Real acc[TM][NC];
    Real sum[TM][COMP ? NC : 1], cmp[TM][COMP ? NC : 1];
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const R4 p = pos[min(tbase + m * kWallBlock + tid, n - 1)];
        xi[m] = p.x;
        yi[m] = p.y;
        wall_height<Real>(p.z, wc, hi[m], di[m]);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            acc[m][k] = Real(0);
            if constexpr (COMP) {
                sum[m][k] = Real(0);
                cmp[m][k] = Real(0);
            }
        }
    }
    const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
    const int s_begin = blockIdx.y * split_len;
    const int s_end = min(n, s_begin + split_len);
    for (int t0 = s_begin; t0 < s_end; t0 += kWallTile) {
        const int j = t0 + tid;
        if (j < s_end) {
            R4 p = pos[j];
            Real h, d;
            wall_height<Real>(p.z, wc, h, d);
            p.z = h;
            R4 f = frc[j];
            f.x *= d;
            f.y *= d;
            f.z *= d;
            sp[tid] = p;
            sf[tid] = f;
            if constexpr (ANG) {
                R4 t = trq[j];
                t.x *= d;
                t.y *= d;
                t.z *= d;
                st[tid] = t;
            }
        }
        __syncthreads();
        const int cnt = min(kWallTile, s_end - t0);
#pragma unroll 2
        for (int q = 0; q < cnt; ++q) {
            const R4 a = sp[q];
            const R4 b = sf[q];
            R4 tq = zero4;
            if constexpr (ANG) tq = st[q];
#pragma unroll
            for (int m = 0; m < TM; ++m) {
                interact<Real, ANG>(xi[m], yi[m], hi[m], a, b, tq, c, acc[m], ANG ? acc[m] + 3 : nullptr);
                wall_image<Real, ANG>(xi[m] - a.x, yi[m] - a.y, hi[m], a.z, b, tq, wc.a2, acc[m],
                                      ANG ? acc[m] + 3 : nullptr);
            }
        }
        __syncthreads();
        if constexpr (COMP) {
#pragma unroll
            for (int m = 0; m < TM; ++m)
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    neumaier(sum[m][k], cmp[m][k], acc[m][k]);
                    acc[m][k] = Real(0);
                }
        }
    }
    // partial outputs of this split, scaled by the target's damping: [split][component][n]
    const size_t nn = (size_t)n;
    Real *base = part + (size_t)blockIdx.y * (COMP ? 2 * NC : NC) * nn;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int idx = tbase + m * kWallBlock + tid;
        if (idx < n) {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                if constexpr (COMP) {
                    base[(size_t)k * nn + idx] = di[m] * sum[m][k];
                    base[(size_t)(NC + k) * nn + idx] = di[m] * cmp[m][k];
                } else {
                    base[(size_t)k * nn + idx] = di[m] * acc[m][k];
                }
            }
        }
    }
}

template <typename Real, bool ANG>
hipError_t launch_wall(const vec4_t<Real> *pos, const vec4_t<Real> *f, const vec4_t<Real> *t, int64_t n,
                       const PairConst<Real> &pc, const WallConst<Real> &wc, int tm, int n_split, Real *part,
                       hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t split_len = (n + n_split - 1) / n_split;
    split_len = (split_len + kWallTile - 1) / kWallTile * kWallTile;
    const int64_t tpb = (int64_t)kWallBlock * tm;
    dim3 grid((unsigned)((n + tpb - 1) / tpb), (unsigned)n_split);
    if (tm == 1)
        hipLaunchKernelGGL((wall_pair_kernel<Real, ANG, 1>), grid, dim3(kWallBlock), 0, st, pos, f, t, (int)n,
                           (int)split_len, pc, wc, part);
    else
        hipLaunchKernelGGL((wall_pair_kernel<Real, ANG, 2>), grid, dim3(kWallBlock), 0, st, pos, f, t, (int)n,
                           (int)split_len, pc, wc, part);
    return hipGetLastError();
}

}  // namespace

// Targets per lane of the wall kernel: the tile configuration's 1 or 2,
// else one with the angular blocks and two without.
int wall_targets_per_lane(const rpy_solver *s, bool ang) {
    const int tm = s->cfg[ang ? 1 : 0].tm;
    if (tm == 1 || tm == 2) return tm;
    return ang ? 1 : 2;
}

template <typename Real, typename Tout>
rpy_status apply_wall(rpy_solver *s, bool ang, const vec4_t<Real> *f, const vec4_t<Real> *t, Tout *lin,
                      Tout *ang_out, hipStream_t st, const void *pos_in) {
    const int64_t n = s->n;
    const int tm = wall_targets_per_lane(s, ang);
    const TileConfig &cfg = s->cfg[ang ? 1 : 0];
    const int splits = (cfg.tm == 1 || cfg.tm == 2) && cfg.n_split > 0
                           ? std::min(cfg.n_split, max_splits(n))
                           : choose_splits(n, tm, s->dtype == RPY_F64, ang);
    const int nc = (ang ? 6 : 3) * (std::is_same<Real, float>::value ? 2 : 1);
    HIP_TRY(s, s->part.ensure((size_t)splits * nc * n * sizeof(Real)));
    const PairConst<Real> pc = make_pair_const<Real>(s->radius);
    const WallConst<Real> wc = make_wall_const<Real>(s->wall_height, s->radius);
    const auto *pos = pos_in ? static_cast<const vec4_t<Real> *>(pos_in) : s->pos.as<vec4_t<Real>>();
    hipEvent_t e0 = timing_begin(s, RPY_KERNEL_PAIR, (double)n * (double)n);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    if (ang)
        HIP_TRY(s, (launch_wall<Real, true>(pos, f, t, n, pc, wc, tm, splits, s->part.as<Real>(), st)));
    else
        HIP_TRY(s, (launch_wall<Real, false>(pos, f, nullptr, n, pc, wc, tm, splits, s->part.as<Real>(), st)));
    if (hipEvent_t e1 = timing_end(s, RPY_KERNEL_PAIR)) HIP_TRY(s, hipEventRecord(e1, st));
    if (ang)
        HIP_TRY(s, (launch_reduce<Real, Tout, true>(s->part.as<Real>(), splits, n, k_factor(s), lin, ang_out, st)));
    else
        HIP_TRY(s, (launch_reduce<Real, Tout, false>(s->part.as<Real>(), splits, n, k_factor(s), lin, ang_out, st)));
    return RPY_OK;
}

template rpy_status apply_wall<float, float>(rpy_solver *, bool, const float4 *, const float4 *, float *, float *,
                                             hipStream_t, const void *);
template rpy_status apply_wall<float, double>(rpy_solver *, bool, const float4 *, const float4 *, double *, double *,
                                              hipStream_t, const void *);
template rpy_status apply_wall<double, double>(rpy_solver *, bool, const double4 *, const double4 *, double *,
                                               double *, hipStream_t, const void *);

}  // namespace rpy

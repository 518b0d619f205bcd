// Pair kernels of the open-boundary RPY mobility product (gfx950).
//
// U = M(X) [F; T] summed over all ordered pairs, self pair included (the
// N-body solver of Sec. 3.5, blocks of eq. (block_mobility) with the
// generalised Rotne-Prager-Yamakawa tensors; the coefficient functions are
// listed with PairConst in rpy_pair.hpp).
//
// Work decomposition
//   grid.x : target blocks of 256*TM targets (TM targets per lane, strided
//            by 256 so global loads/stores stay coalesced);
//   grid.y : source splits, contiguous ranges of the source list.
//   Each workgroup streams its source range through LDS in tiles of 256
//   records (one coalesced 16 B (fp32) or 32 B (fp64) load per field per
//   thread), then every lane walks the tile reading each record by LDS
//   broadcast and updates its TM targets.  The overlap branch r < 2a, which
//   also covers the self pair, sits behind a divergent `if` that the wave
//   skips whenever none of its lanes has such a partner (the common case).
// Precision
//   fp32: in-tile plain float sums, folded into per-target (sum, comp)
//         Neumaier pairs after every tile; the partial pairs of the splits
//         are combined by the reduce kernel.
//   fp64: plain double sums; 1/sqrt from the hardware estimate refined by
//         one Newton step (relative error below 4.2e-15).
#include "rpy_device.hpp"
#include "rpy_internal.hpp"

#include <algorithm>
#include <cmath>

namespace rpy {

constexpr int kBlock = 256;   // threads per workgroup of the pair kernel
constexpr int kTile = 256;    // sources per LDS tile (one per thread)

int targets_per_block(int tm) { return kBlock * tm; }
int source_tile() { return kTile; }

int max_splits(int64_t n) { return (int)std::max<int64_t>(1, (n + kTile - 1) / kTile); }

int choose_splits(int64_t n, int tm, bool fp64, bool ang) {
    (void)fp64;
    (void)ang;
    const int64_t tblocks = (n + targets_per_block(tm) - 1) / targets_per_block(tm);
    const int64_t max_split = std::max<int64_t>(1, (n + kTile - 1) / kTile);
    // ~32 workgroups per CU: the split count the autotuner picks at
    // N = 65,536, and at larger N it keeps the grid's tail short
    const int64_t want = (8192 + tblocks - 1) / tblocks;
    return (int)std::max<int64_t>(1, std::min(want, max_split));
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
hipError_t DevBuf::ensure(size_t want) {
    if (want <= bytes && p) return hipSuccess;
    release();
    size_t b = std::max<size_t>(want, 256);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        bytes = 0;
        return e;
    }
    bytes = b;
    return hipSuccess;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

template <typename Real, bool ANG, int TM>
__global__ void __launch_bounds__(kBlock)
pair_kernel(const vec4_t<Real> *__restrict__ pos, const vec4_t<Real> *__restrict__ frc,
            const vec4_t<Real> *__restrict__ trq, int n, int split_len, PairConst<Real> c,
            Real *__restrict__ part) {
    using R4 = vec4_t<Real>;
    constexpr int NC = ANG ? 6 : 3;                       // output components
    constexpr bool COMP = std::is_same<Real, float>::value;  // compensated sums
    __shared__ R4 sp[kTile];
    __shared__ R4 sf[kTile];
    __shared__ R4 st[ANG ? kTile : 1];
    __shared__ R4 sh[ANG ? kTile : 1];

    const int tid = threadIdx.x;
    const int tbase = blockIdx.x * (kBlock * TM);
    Real xi[TM], yi[TM], zi[TM];
    Real acc[TM][NC];
    Real sum[TM][COMP ? NC : 1], cmp[TM][COMP ? NC : 1];
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int idx = min(tbase + m * kBlock + tid, n - 1);
        const R4 p = pos[idx];
        xi[m] = p.x;
        yi[m] = p.y;
        zi[m] = p.z;
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[m][k] = Real(0);
        if constexpr (COMP) {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                sum[m][k] = Real(0);
                cmp[m][k] = Real(0);
            }
        }
    }

    const int s_begin = blockIdx.y * split_len;
    const int s_end = min(n, s_begin + split_len);
    const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
    for (int t0 = s_begin; t0 < s_end; t0 += kTile) {
        const int j = t0 + tid;
        if (j < s_end) {
            R4 p = pos[j], f = frc[j];
            if constexpr (ANG) {
                // per-source vectors of the regrouped angular pair (interact_ang)
                R4 t = trq[j];
                p.w = c.two_a2_3 * f.x;
                f.w = c.two_a2_3 * f.y;
                t.w = c.two_a2_3 * f.z;
                R4 h;
                h.x = Real(-0.5) * t.x;
                h.y = Real(-0.5) * t.y;
                h.z = Real(-0.5) * t.z;
                h.w = Real(0);
                st[tid] = t;
                sh[tid] = h;
            }
            sp[tid] = p;
            sf[tid] = f;
        }
        __syncthreads();
        const int cnt = min(kTile, s_end - t0);
#pragma unroll 2
        for (int q = 0; q < cnt; ++q) {
            const R4 a = sp[q];
            const R4 b = sf[q];
            if constexpr (ANG) {
                const R4 d = st[q];
                const R4 e = sh[q];
#pragma unroll
                for (int m = 0; m < TM; ++m)
                    interact_ang<Real>(xi[m], yi[m], zi[m], a, b, d, e, c, acc[m], acc[m] + 3);
            } else {
#pragma unroll
                for (int m = 0; m < TM; ++m)
                    interact<Real, false>(xi[m], yi[m], zi[m], a, b, zero4, c, acc[m], nullptr);
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

    // partial outputs of this split: [split][component][n]
    const size_t nn = (size_t)n;
    Real *base = part + (size_t)blockIdx.y * (COMP ? 2 * NC : NC) * nn;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int idx = tbase + m * kBlock + tid;
        if (idx < n) {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                if constexpr (COMP) {
                    base[(size_t)k * nn + idx] = sum[m][k];
                    base[(size_t)(NC + k) * nn + idx] = cmp[m][k];
                } else {
                    base[(size_t)k * nn + idx] = acc[m][k];
                }
            }
        }
    }
}

template <typename Real, bool ANG>
hipError_t launch_pair(const vec4_t<Real> *pos, const vec4_t<Real> *f, const vec4_t<Real> *t,
                       int64_t n, const PairConst<Real> &pc, const TileConfig &cfg, int n_split,
                       Real *part, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int tm = (cfg.tm == 1 || cfg.tm == 4) ? cfg.tm : 2;
    const int64_t tpb = targets_per_block(tm);
    int64_t split_len = (n + n_split - 1) / n_split;
    split_len = (split_len + kTile - 1) / kTile * kTile;
    dim3 grid((unsigned)((n + tpb - 1) / tpb), (unsigned)n_split);
    if (tm == 1)
        hipLaunchKernelGGL((pair_kernel<Real, ANG, 1>), grid, dim3(kBlock), 0, st, pos, f, t, (int)n,
                           (int)split_len, pc, part);
    else if (tm == 4)
        hipLaunchKernelGGL((pair_kernel<Real, ANG, 4>), grid, dim3(kBlock), 0, st, pos, f, t, (int)n,
                           (int)split_len, pc, part);
    else
        hipLaunchKernelGGL((pair_kernel<Real, ANG, 2>), grid, dim3(kBlock), 0, st, pos, f, t, (int)n,
                           (int)split_len, pc, part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduction over source splits + epilogue (x k, AoS store)
// ---------------------------------------------------------------------------
// One thread per (target i, component c = blockIdx.y); the loads of four
// splits are issued ahead of the (sequential, fixed-order) compensated sum.
template <typename Real, typename Tout, bool ANG>
__global__ void __launch_bounds__(256)
reduce_kernel(const Real *__restrict__ part, int n_split, int n, double k, Tout *__restrict__ lin,
              Tout *__restrict__ ang) {
    constexpr int NC = ANG ? 6 : 3;
    constexpr bool COMP = std::is_same<Real, float>::value;
    constexpr int U = 4;
    const int c = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (c >= 3 && !ang)) return;
    const size_t nn = (size_t)n;
    const size_t stride = (size_t)(COMP ? 2 * NC : NC) * nn;
    const Real *p0 = part + (size_t)c * nn + i;
    Tout v;
    if constexpr (COMP) {
        const Real *p1 = part + (size_t)(NC + c) * nn + i;
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
        // combine in double, then round once to the output type
        v = (Tout)(k * ((double)s + ((double)cp + (double)extra)));
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
        v = (Tout)(k * s);
    }
    if (c < 3)
        lin[3 * (size_t)i + c] = v;
    else
        ang[3 * (size_t)i + (c - 3)] = v;
}

template <typename Real, typename Tout, bool ANG>
hipError_t launch_reduce(const Real *part, int n_split, int64_t n, double k, Tout *lin, Tout *ang,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((reduce_kernel<Real, Tout, ANG>), dim3((unsigned)((n + 255) / 256), ANG ? 6 : 3), dim3(256),
                       0, st, part, n_split, (int)n, k, lin, ang);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// staging
// ---------------------------------------------------------------------------
template <typename Tin, typename Real>
__global__ void stage_positions_kernel(const Tin *__restrict__ in, int n, vec4_t<Real> *__restrict__ out,
                                       unsigned *__restrict__ nonfinite) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Tin x = in[3 * (size_t)i], y = in[3 * (size_t)i + 1], z = in[3 * (size_t)i + 2];
    if (!(isfinite((double)x) && isfinite((double)y) && isfinite((double)z))) atomicAdd(nonfinite, 1u);
    vec4_t<Real> v;
    v.x = (Real)x;
    v.y = (Real)y;
    v.z = (Real)z;
    v.w = Real(0);
    out[i] = v;
}

template <typename Tin, typename Real>
__global__ void stage_vec_kernel(const Tin *__restrict__ in, int n, vec4_t<Real> *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    vec4_t<Real> v;
    if (in) {
        v.x = (Real)in[3 * (size_t)i];
        v.y = (Real)in[3 * (size_t)i + 1];
        v.z = (Real)in[3 * (size_t)i + 2];
    } else {
        v.x = v.y = v.z = Real(0);
    }
    v.w = Real(0);
    out[i] = v;
}

template <typename Tin, typename Real>
hipError_t launch_stage_positions(const Tin *pos, int64_t n, vec4_t<Real> *out, unsigned *nonfinite,
                                  hipStream_t st) {
    hipLaunchKernelGGL((stage_positions_kernel<Tin, Real>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       st, pos, (int)n, out, nonfinite);
    return hipGetLastError();
}

template <typename Tin, typename Real>
hipError_t launch_stage_vec(const Tin *v, int64_t n, vec4_t<Real> *out, hipStream_t st) {
    hipLaunchKernelGGL((stage_vec_kernel<Tin, Real>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       v, (int)n, out);
    return hipGetLastError();
}

template <typename T>
__global__ void fill_zero_kernel(T *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = T(0);
}

template <typename T>
hipError_t launch_fill_zero(T *p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((fill_zero_kernel<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p,
                       count);
    return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_stage_positions<float, float>(const float *, int64_t, float4 *, unsigned *, hipStream_t);
template hipError_t launch_stage_positions<double, double>(const double *, int64_t, double4 *, unsigned *, hipStream_t);
template hipError_t launch_stage_vec<float, float>(const float *, int64_t, float4 *, hipStream_t);
template hipError_t launch_stage_vec<double, double>(const double *, int64_t, double4 *, hipStream_t);
template hipError_t launch_stage_vec<double, float>(const double *, int64_t, float4 *, hipStream_t);
template hipError_t launch_pair<float, false>(const float4 *, const float4 *, const float4 *, int64_t,
                                              const PairConst<float> &, const TileConfig &, int, float *,
                                              hipStream_t);
template hipError_t launch_pair<float, true>(const float4 *, const float4 *, const float4 *, int64_t,
                                             const PairConst<float> &, const TileConfig &, int, float *,
                                             hipStream_t);
template hipError_t launch_pair<double, false>(const double4 *, const double4 *, const double4 *, int64_t,
                                               const PairConst<double> &, const TileConfig &, int, double *,
                                               hipStream_t);
template hipError_t launch_pair<double, true>(const double4 *, const double4 *, const double4 *, int64_t,
                                              const PairConst<double> &, const TileConfig &, int, double *,
                                              hipStream_t);
template hipError_t launch_reduce<float, float, false>(const float *, int, int64_t, double, float *, float *, hipStream_t);
template hipError_t launch_reduce<float, float, true>(const float *, int, int64_t, double, float *, float *, hipStream_t);
template hipError_t launch_reduce<float, double, false>(const float *, int, int64_t, double, double *, double *, hipStream_t);
template hipError_t launch_reduce<float, double, true>(const float *, int, int64_t, double, double *, double *, hipStream_t);
template hipError_t launch_reduce<double, double, false>(const double *, int, int64_t, double, double *, double *, hipStream_t);
template hipError_t launch_reduce<double, double, true>(const double *, int, int64_t, double, double *, double *, hipStream_t);
template hipError_t launch_fill_zero<float>(float *, int64_t, hipStream_t);
template hipError_t launch_fill_zero<double>(double *, int64_t, hipStream_t);
template hipError_t launch_fill_zero<unsigned>(unsigned *, int64_t, hipStream_t);

}  // namespace rpy

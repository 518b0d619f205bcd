// Fused pair kernel for small N (tile mode 3): the whole product M [F; T]
// in one launch, for sizes where launch latency and the few workgroups of
// the tiled kernels, not pair arithmetic, set the time (the open-boundary
// N-body product of Sec. 3.5).
//
// A workgroup of 16 wavefronts owns TG targets (4, 8 or 16: enough
// workgroups for every CU).  Sources pass through LDS in chunks (1024 in
// float32, 512 in float64): every thread loads one source's position and
// force (and torque) straight from the caller's arrays (N x 3 with stride 3,
// or staged vec4 records with stride 4), so a chunk costs one memory latency
// and no staging launch is needed.  In every wavefront lane (t, p) =
// (lane % TG, lane / TG) holds target t and walks source phase p of the
// wavefront's sixteenth of the chunk.  float32 sums fold into Neumaier pairs
// once per chunk.  The 1024 / TG partial sums of a target (16 wavefronts x
// 64 / TG phases) are added in a fixed order in two levels (groups of 16,
// then the groups; compensated in float32), scaled by k = 1/(8 pi eta) and
// written in the output type: no reduction launch.
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <type_traits>

namespace rpy {
namespace {

constexpr int kFusedWaves = 16;
constexpr int kFusedThreads = kFusedWaves * 64;

template <typename Real>
__device__ __forceinline__ vec4_t<Real> load3(const Real *__restrict__ v, int stride, int j) {
    vec4_t<Real> r;
    if (v) {
        r.x = v[(size_t)j * stride];
        r.y = v[(size_t)j * stride + 1];
        r.z = v[(size_t)j * stride + 2];
    } else {
        r.x = r.y = r.z = Real(0);
    }
    r.w = Real(0);
    return r;
}

template <typename Real, bool ANG>
struct FusedShape {
    static constexpr bool COMP = std::is_same<Real, float>::value;
    static constexpr int NC = ANG ? 6 : 3;
    static constexpr int PC = COMP ? 2 * NC : NC;
    static constexpr int CHUNK = COMP ? 1024 : 512;                    // sources per LDS chunk
    static constexpr int NR = ANG ? 3 : 2;                             // records per source
    static constexpr size_t kStage = sizeof(vec4_t<Real>) * NR * CHUNK;
    static constexpr size_t kPart = sizeof(Real) * kFusedThreads * PC;   // one partial set per lane
    static constexpr size_t kBytes = kStage > kPart ? kStage : kPart;   // the two uses alias
};

template <typename Real, typename Tout, bool ANG, int TG>
__global__ void __launch_bounds__(kFusedThreads)
fused_kernel(const vec4_t<Real> *__restrict__ pos, const Real *__restrict__ f, const Real *__restrict__ t,
             int stride, int n, PairConst<Real> c, double k, Tout *__restrict__ lin, Tout *__restrict__ ang) {
    using Sh = FusedShape<Real, ANG>;
    using R4 = vec4_t<Real>;
    constexpr int NC = Sh::NC, PC = Sh::PC, CHUNK = Sh::CHUNK;
    constexpr bool COMP = Sh::COMP;
    constexpr int PH = 64 / TG;                      // source phases per wavefront
    constexpr int NP = kFusedWaves * PH;             // partials per target
    constexpr int G = NP / 16;                       // groups of 16 partials
    constexpr int PER_WAVE = CHUNK / kFusedWaves;
    __shared__ __align__(16) unsigned char smem[Sh::kBytes];
    __shared__ Real gsum[NC * TG * G][COMP ? 2 : 1];
    R4 *rec = reinterpret_cast<R4 *>(smem);                              // [NR][CHUNK]
    Real (*part)[PC][TG] = reinterpret_cast<Real (*)[PC][TG]>(smem);      // [NP][PC][TG]

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int tl = lane % TG, ph = lane / TG;
    const int i = blockIdx.x * TG + tl;
    const R4 pi = pos[min(i, n - 1)];
    Real acc[NC], sum[COMP ? NC : 1], cmp[COMP ? NC : 1];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        acc[q] = Real(0);
        if constexpr (COMP) {
            sum[q] = Real(0);
            cmp[q] = Real(0);
        }
    }
    const R4 zero4 = {Real(0), Real(0), Real(0), Real(0)};
    for (int cb = 0; cb < n; cb += CHUNK) {
        for (int e = tid; e < CHUNK; e += kFusedThreads) {
            const int j = cb + e;
            const bool ok = j < n;
            rec[e] = pos[ok ? j : n - 1];
            rec[CHUNK + e] = ok ? load3(f, stride, j) : zero4;
            if constexpr (ANG) rec[2 * CHUNK + e] = ok ? load3(t, stride, j) : zero4;
        }
        __syncthreads();
        // this wavefront's slice of the chunk, phase ph
        const int q0 = wv * PER_WAVE, q1 = min(q0 + PER_WAVE, n - cb);
        for (int q = q0 + ph; q < q1; q += PH) {
            const R4 pj = rec[q];
            const R4 fj = rec[CHUNK + q];
            const R4 tj = ANG ? rec[2 * CHUNK + q] : zero4;
            interact<Real, ANG>(pi.x, pi.y, pi.z, pj, fj, tj, c, acc, ANG ? acc + 3 : nullptr);
        }
        if constexpr (COMP) {
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                neumaier(sum[q], cmp[q], acc[q]);
                acc[q] = Real(0);
            }
        }
        __syncthreads();   // the chunk's records are read before they are overwritten
    }
    const int slot = wv * PH + ph;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        if constexpr (COMP) {
            part[slot][q][tl] = sum[q];
            part[slot][NC + q][tl] = cmp[q];
        } else {
            part[slot][q][tl] = acc[q];
        }
    }
    __syncthreads();
    // level 1: thread (component q, target l, group g) sums partials
    // 16 g .. 16 g + 15 in order
    if (tid < NC * TG * G) {
        const int g = tid % G, ql = tid / G;
        const int q = ql / TG, l = ql % TG;
        if constexpr (COMP) {
            float s = 0.f, cp = 0.f, extra = 0.f;
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                neumaier(s, cp, part[16 * g + w][q][l]);
                extra += part[16 * g + w][NC + q][l];
            }
            gsum[tid][0] = s;
            gsum[tid][1] = cp + extra;
        } else {
            Real v = Real(0);
#pragma unroll
            for (int w = 0; w < 16; ++w) v += part[16 * g + w][q][l];
            gsum[tid][0] = v;
        }
    }
    __syncthreads();
    // level 2: thread (q, l) sums its G groups in order
    if (tid < NC * TG) {
        const int q = tid / TG, l = tid % TG;
        const int ti = blockIdx.x * TG + l;
        Tout *o = q < 3 ? lin : ang;
        if (ti < n && o) {
            double v;
            if constexpr (COMP) {
                float s = 0.f, cp = 0.f, extra = 0.f;
                for (int g = 0; g < G; ++g) {
                    neumaier(s, cp, gsum[tid * G + g][0]);
                    extra += gsum[tid * G + g][1];
                }
                v = (double)s + ((double)cp + (double)extra);
            } else {
                v = 0.0;
                for (int g = 0; g < G; ++g) v += (double)gsum[tid * G + g][0];
            }
            o[(size_t)ti * 3 + (q % 3)] = (Tout)(k * v);
        }
    }
}

template <typename Real, typename Tout, bool ANG>
void launch_fused(int tg, const vec4_t<Real> *pos, const Real *f, const Real *t, int stride, int n,
                  const PairConst<Real> &c, double k, Tout *lin, Tout *ang, hipStream_t st) {
    const dim3 grid((unsigned)((n + tg - 1) / tg)), block(kFusedThreads);
    if (tg == 4)
        hipLaunchKernelGGL((fused_kernel<Real, Tout, ANG, 4>), grid, block, 0, st, pos, f, t, stride, n, c, k, lin, ang);
    else if (tg == 8)
        hipLaunchKernelGGL((fused_kernel<Real, Tout, ANG, 8>), grid, block, 0, st, pos, f, t, stride, n, c, k, lin, ang);
    else
        hipLaunchKernelGGL((fused_kernel<Real, Tout, ANG, 16>), grid, block, 0, st, pos, f, t, stride, n, c, k, lin,
                           ang);
}

}  // namespace

template <typename Real, typename Tout>
rpy_status apply_fused(rpy_solver *s, bool ang, const Real *f, const Real *t, int stride, Tout *lin, Tout *ang_out,
                       hipStream_t st, const void *pos_in) {
    const int64_t n = s->n;
    if (n <= 0) return RPY_OK;
    const PairConst<Real> pc = make_pair_const<Real>(s->radius);
    const auto *pos = pos_in ? static_cast<const vec4_t<Real> *>(pos_in) : s->pos.as<vec4_t<Real>>();
    // targets per workgroup: at least 256 workgroups where N allows
    const int tg = n <= 1024 ? 4 : (n <= 2048 ? 8 : 16);
    hipEvent_t e0 = timing_begin(s, RPY_KERNEL_PAIR, (double)n * (double)n);
    if (e0) HIP_TRY(s, hipEventRecord(e0, st));
    if (ang)
        launch_fused<Real, Tout, true>(tg, pos, f, t, stride, (int)n, pc, k_factor(s), lin, ang_out, st);
    else
        launch_fused<Real, Tout, false>(tg, pos, f, t, stride, (int)n, pc, k_factor(s), lin, ang_out, st);
    HIP_TRY(s, hipGetLastError());
    if (hipEvent_t e1 = timing_end(s, RPY_KERNEL_PAIR)) HIP_TRY(s, hipEventRecord(e1, st));
    return RPY_OK;
}

template rpy_status apply_fused<float, float>(rpy_solver *, bool, const float *, const float *, int, float *, float *,
                                              hipStream_t, const void *);
template rpy_status apply_fused<float, double>(rpy_solver *, bool, const float *, const float *, int, double *,
                                               double *, hipStream_t, const void *);
template rpy_status apply_fused<double, double>(rpy_solver *, bool, const double *, const double *, int, double *,
                                                double *, hipStream_t, const void *);

}  // namespace rpy

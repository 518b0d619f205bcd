// Preconditioned Lanczos square root (Sec. 3.3 notes that a preconditioner
// can speed up the Krylov iteration; the paper's release does not use one).
//
// With a lower-triangular L, the noise y = L (L^{-1} M L^{-T})^{1/2} W has
// covariance L L^{-1} M L^{-T} L^T = M, so it satisfies the fluctuation-
// dissipation balance of eq. (fdt) like M^{1/2} W, and Lanczos on the
// preconditioned operator A = L^{-1} M L^{-T} converges in fewer iterations
// when L L^T captures the stiff part of M.  L here is block diagonal: the
// particles form groups of G consecutive particles (a chain, a rigid body,
// a cluster), and for every group L holds the Cholesky factor of M
// restricted to the group's 3G linear rows and, with angular blocks,
// separately of its 3G angular rows.  Every block is a dense D x D float64
// matrix (D = 3G, column-major); the last group is padded with identity
// rows.
//
// Setup (once per positions and group size): one kernel assembles every
// block from the pair formulas (open or single-wall geometry, in float64
// from the stored positions), then the batched Cholesky factorisation of
// the library solver (rocSOLVER potrf, strided batched) factors them in
// place.  Per Lanczos iteration: t = L^{-T} v (blocked backward
// substitution), the product M t, and w = L^{-1} (M t) (blocked forward
// substitution); at the end y = L z.  Each block is handled by one
// workgroup, with its vector segment in LDS: panels of 64 columns are
// solved sequentially by one wave on a copy of the diagonal panel in LDS,
// and the coupling to the other panels is a matrix-vector update by all
// threads with coalesced column reads.
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"
#include "rpy_wall.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace rpy {
namespace {

constexpr int kTriThreads = 256;
constexpr int kPanel = 64;
constexpr int kMaxBlockDim = 1536;   // D = 3G, G <= 512 particles per group

// Block b of the preconditioner: group g = b / parts, part p = b % parts
// (0 linear rows, 1 angular rows); entries of the vector it covers: the
// part's offset (0 or 3N) + 3 g G + r for r < 3 min(G, N - g G).
struct BlockMap {
    int64_t np;      // particles
    int group;       // G
    int parts;       // 1 or 2
    int dim;         // D = 3G
    __device__ int64_t first(int b) const { return (int64_t)(b % parts) * 3 * np + (int64_t)3 * (b / parts) * group; }
    __device__ int rows(int b) const {
        const int64_t left = np - (int64_t)(b / parts) * group;
        return 3 * (int)(left < group ? left : group);
    }
};

// Assembly: thread (i, j) of block b writes the 3 x 3 entries coupling
// particles i and j of the group (columns 3j + c, rows 3i + a).  Entries of
// padding particles form an identity.
template <typename Real, bool WALL>
__global__ void assemble_blocks(const vec4_t<Real> *__restrict__ pos, BlockMap m, PairConst<double> pc,
                                WallConst<double> wc, double k, double *__restrict__ L) {
    const int b = blockIdx.x;
    const int i = blockIdx.y * 16 + threadIdx.y, j = blockIdx.z * 16 + threadIdx.x;
    if (i >= m.group || j >= m.group) return;
    const bool ang = (b % m.parts) == 1;
    const int64_t g0 = (int64_t)(b / m.parts) * m.group;
    const int64_t pi = g0 + i, pj = g0 + j;
    double blk[3][3];
    if (pi < m.np && pj < m.np) {
        const vec4_t<Real> qi = pos[pi], qj = pos[pj];
        double xi = qi.x, yi = qi.y, zi = qi.z, di = 1.0;
        double4 sp = {(double)qj.x, (double)qj.y, (double)qj.z, 0.0};
        double dj = 1.0;
        if constexpr (WALL) {
            wall_height<double>(zi, wc, zi, di);
            wall_height<double>(sp.z, wc, sp.z, dj);
        }
        for (int c = 0; c < 3; ++c) {
            double4 e = {0.0, 0.0, 0.0, 0.0};
            const double4 zero4 = {0.0, 0.0, 0.0, 0.0};
            (c == 0 ? e.x : (c == 1 ? e.y : e.z)) = 1.0;
            double u[3] = {0.0, 0.0, 0.0}, w[3] = {0.0, 0.0, 0.0};
            if (!ang) {
                interact<double, false>(xi, yi, zi, sp, e, zero4, pc, u, nullptr);
                if constexpr (WALL) wall_image<double, false>(xi - sp.x, yi - sp.y, zi, sp.z, e, zero4, wc.a2, u, nullptr);
            } else {
                interact<double, true>(xi, yi, zi, sp, zero4, e, pc, u, w);
                if constexpr (WALL) wall_image<double, true>(xi - sp.x, yi - sp.y, zi, sp.z, zero4, e, wc.a2, u, w);
            }
            const double *col = ang ? w : u;
            for (int a = 0; a < 3; ++a) blk[a][c] = k * di * dj * col[a];
        }
    } else {
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) blk[a][c] = (i == j && a == c) ? 1.0 : 0.0;
    }
    double *Lb = L + (size_t)b * m.dim * m.dim;
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a) Lb[(size_t)(3 * j + c) * m.dim + 3 * i + a] = blk[a][c];
}

// Loads the diagonal panel L[p0 .. p0 + pn, p0 .. p0 + pn] into dg (column
// c at dg[c][.]).
__device__ __forceinline__ void load_panel(const double *Lb, int dim, int p0, int pn, double (*dg)[kPanel + 1]) {
    for (int e = threadIdx.x; e < pn * pn; e += blockDim.x) {
        const int c = e / pn, r = e % pn;
        dg[c][r] = Lb[(size_t)(p0 + c) * dim + p0 + r];
    }
}

// x = L^{-1} x (forward substitution) or x = L^{-T} x (backward), for the
// vector segment of every block; in and out may alias.
template <bool TRANS>
__global__ void __launch_bounds__(kTriThreads)
tri_solve(const double *__restrict__ L, BlockMap m, const double *in, double *out) {
    __shared__ double x[kMaxBlockDim];
    __shared__ double dg[kPanel][kPanel + 1];
    const int b = blockIdx.x;
    const int dim = m.dim, nr = m.rows(b);
    const int64_t f = m.first(b);
    const double *Lb = L + (size_t)b * dim * dim;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int r = threadIdx.x; r < dim; r += blockDim.x) x[r] = r < nr ? in[f + r] : 0.0;
    __syncthreads();
    const int npanel = (dim + kPanel - 1) / kPanel;
    for (int q = 0; q < npanel; ++q) {
        const int p = TRANS ? npanel - 1 - q : q;
        const int p0 = p * kPanel, pn = min(kPanel, dim - p0);
        if (TRANS) {
            // x_r -= sum_{c >= p0 + pn} L[c][r] x_c for the panel's rows: one
            // wave per row, lanes along the column (contiguous)
            for (int r = wv; r < pn; r += kTriThreads / 64) {
                const double *col = Lb + (size_t)(p0 + r) * dim;
                double acc = 0.0;
                for (int c = p0 + pn + lane; c < dim; c += 64) acc = fma(col[c], x[c], acc);
                acc = wave_sum(acc);
                if (lane == 0) x[p0 + r] -= acc;
            }
        }
        load_panel(Lb, dim, p0, pn, dg);
        __syncthreads();
        if (wv == 0) {
            double xr = lane < pn ? x[p0 + lane] : 0.0;
            if (!TRANS) {
                for (int c = 0; c < pn; ++c) {
                    const double xc = __shfl(xr, c, 64) / dg[c][c];
                    if (lane == c) xr = xc;
                    else if (lane > c) xr = fma(-dg[c][lane], xc, xr);
                }
            } else {
                for (int c = pn - 1; c >= 0; --c) {
                    const double xc = __shfl(xr, c, 64) / dg[c][c];
                    if (lane == c) xr = xc;
                    else if (lane < c) xr = fma(-dg[lane][c], xc, xr);
                }
            }
            if (lane < pn) x[p0 + lane] = xr;
        }
        __syncthreads();
        if (!TRANS) {
            // rows below the panel: x_r -= sum_{c in panel} L[r][p0 + c] x_{p0 + c}
            for (int r = p0 + pn + threadIdx.x; r < dim; r += blockDim.x) {
                double acc = 0.0;
                for (int c = 0; c < pn; ++c) acc = fma(Lb[(size_t)(p0 + c) * dim + r], x[p0 + c], acc);
                x[r] -= acc;
            }
            __syncthreads();
        }
    }
    for (int r = threadIdx.x; r < nr; r += blockDim.x) out[f + r] = x[r];
}

// out = prefactor * L z (+ out when accumulating), written into the caller's
// linear and angular outputs (vector entries below 3N are linear rows).
template <typename Tout>
__global__ void __launch_bounds__(kTriThreads)
tri_mul(const double *__restrict__ L, BlockMap m, const double *__restrict__ z, double prefactor, int accumulate,
        Tout *__restrict__ lin, Tout *__restrict__ ang) {
    __shared__ double x[kMaxBlockDim];
    const int b = blockIdx.x;
    const int dim = m.dim, nr = m.rows(b);
    const int64_t f = m.first(b);
    const double *Lb = L + (size_t)b * dim * dim;
    for (int r = threadIdx.x; r < dim; r += blockDim.x) x[r] = r < nr ? z[f + r] : 0.0;
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c <= r; ++c) acc = fma(Lb[(size_t)c * dim + r], x[c], acc);
        const int64_t e = f + r;
        Tout *dst = e < 3 * m.np ? lin + e : ang + (e - 3 * m.np);
        const double base = accumulate ? (double)*dst : 0.0;
        *dst = (Tout)(base + prefactor * acc);
    }
}

BlockMap block_map(const rpy_solver *s) {
    BlockMap m;
    m.np = s->n;
    m.group = s->pc_group;
    m.parts = s->pc_parts;
    m.dim = 3 * s->pc_group;
    return m;
}

int block_count(const rpy_solver *s) {
    return (int)((s->n + s->pc_group - 1) / s->pc_group) * s->pc_parts;
}

}  // namespace

rpy_status precond_setup(rpy_solver *s, int64_t group, hipStream_t st) {
    if (s->pse) return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY, "the preconditioner is built for open boundaries and the wall");
    if (group < 1 || group > kMaxBlockDim / 3)
        return fail(s, RPY_ERR_INVALID_ARG, "group size must be in [1, 512] particles");
    const int parts = s->angular ? 2 : 1;
    if (s->pc_valid && s->pc_version == s->pos_version && s->pc_group == group && s->pc_parts == parts)
        return RPY_OK;
    s->pc_valid = false;
    s->pc_group = (int)group;
    s->pc_parts = parts;
    const BlockMap m = block_map(s);
    const int nb = block_count(s);
    const size_t bytes = sizeof(double) * (size_t)nb * m.dim * m.dim;
    HIP_TRY(s, s->pc_L.ensure(bytes));
    HIP_TRY(s, s->pc_tmp.ensure(sizeof(double) * (size_t)(parts * 3) * s->n));
    HIP_TRY(s, s->pc_info.ensure(sizeof(int) * (size_t)nb));
    const dim3 grid((unsigned)nb, (unsigned)((group + 15) / 16), (unsigned)((group + 15) / 16)), block(16, 16);
    const PairConst<double> pc = make_pair_const<double>(s->radius);
    const WallConst<double> wc = make_wall_const<double>(s->wall_height, s->radius);
    const double k = k_factor(s);
    if (s->dtype == RPY_F64) {
        if (s->wall)
            hipLaunchKernelGGL((assemble_blocks<double, true>), grid, block, 0, st, s->pos.as<double4>(), m, pc, wc, k,
                               s->pc_L.as<double>());
        else
            hipLaunchKernelGGL((assemble_blocks<double, false>), grid, block, 0, st, s->pos.as<double4>(), m, pc, wc, k,
                               s->pc_L.as<double>());
    } else {
        if (s->wall)
            hipLaunchKernelGGL((assemble_blocks<float, true>), grid, block, 0, st, s->pos.as<float4>(), m, pc, wc, k,
                               s->pc_L.as<double>());
        else
            hipLaunchKernelGGL((assemble_blocks<float, false>), grid, block, 0, st, s->pos.as<float4>(), m, pc, wc, k,
                               s->pc_L.as<double>());
    }
    HIP_TRY(s, hipGetLastError());
    if (!s->blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success)
            return fail(s, RPY_ERR_HIP, "rocblas_create_handle failed");
        s->blas = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(s->blas);
    if (rocblas_set_stream(h, st) != rocblas_status_success) return fail(s, RPY_ERR_HIP, "rocblas_set_stream failed");
    if (rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, m.dim, s->pc_L.as<double>(), m.dim,
                                         (rocblas_stride)m.dim * m.dim, s->pc_info.as<rocblas_int>(),
                                         nb) != rocblas_status_success)
        return fail(s, RPY_ERR_HIP, "batched Cholesky factorisation (rocsolver_dpotrf_strided_batched) failed");
    std::vector<int> info(nb);
    HIP_TRY(s, hipMemcpyAsync(info.data(), s->pc_info.p, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    HIP_TRY(s, hipStreamSynchronize(st));
    for (int b = 0; b < nb; ++b)
        if (info[b] != 0)
            return fail(s, RPY_ERR_NOT_SPD,
                        "a preconditioner block is not positive definite (group " + std::to_string(b / parts) + ")");
    s->pc_version = s->pos_version;
    s->pc_valid = true;
    return RPY_OK;
}

rpy_status precond_solve_lt(rpy_solver *s, const double *v, double *out, hipStream_t st) {
    hipLaunchKernelGGL((tri_solve<true>), dim3((unsigned)block_count(s)), dim3(kTriThreads), 0, st,
                       s->pc_L.as<double>(), block_map(s), v, out);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

rpy_status precond_solve_l(rpy_solver *s, double *w, hipStream_t st) {
    hipLaunchKernelGGL((tri_solve<false>), dim3((unsigned)block_count(s)), dim3(kTriThreads), 0, st,
                       s->pc_L.as<double>(), block_map(s), w, w);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

template <typename Tout>
rpy_status precond_mul_l(rpy_solver *s, const double *z, double prefactor, bool accumulate, Tout *lin, Tout *ang,
                         hipStream_t st) {
    hipLaunchKernelGGL((tri_mul<Tout>), dim3((unsigned)block_count(s)), dim3(kTriThreads), 0, st,
                       s->pc_L.as<double>(), block_map(s), z, prefactor, accumulate ? 1 : 0, lin, ang);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

template rpy_status precond_mul_l<float>(rpy_solver *, const double *, double, bool, float *, float *, hipStream_t);
template rpy_status precond_mul_l<double>(rpy_solver *, const double *, double, bool, double *, double *, hipStream_t);

void precond_release(rpy_solver *s) {
    s->pc_L.release();
    s->pc_tmp.release();
    s->pc_info.release();
    if (s->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(s->blas));
    s->blas = nullptr;
    s->pc_valid = false;
}

}  // namespace rpy

using namespace rpy;

extern "C" rpy_status rpy_sqrt_mdot_w_precond(rpy_solver *s, const void *w, int64_t group_size, double prefactor,
                                             double tol, int max_iter, void *lin_out, void *ang_out, int *iters_out,
                                             double *incr_out, void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!w || !lin_out) return fail(s, RPY_ERR_INVALID_ARG, "W and the linear output must not be NULL");
    if (s->angular && !ang_out) return fail(s, RPY_ERR_INVALID_ARG, "include_angular needs the angular output");
    if (!s->angular && ang_out) return fail(s, RPY_ERR_ANGULAR_DISABLED, "angular output needs include_angular");
    if (!(tol > 0.0 && tol < 1.0)) return fail(s, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(s, RPY_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!std::isfinite(prefactor)) return fail(s, RPY_ERR_INVALID_ARG, "prefactor must be finite");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    r = precond_setup(s, group_size, st);
    if (r != RPY_OK) return r;
    if (s->dtype == RPY_F64)
        return lanczos_run_multi<double>(s, static_cast<const double *>(w), 1, 0, prefactor, tol, max_iter,
                                         static_cast<double *>(lin_out), static_cast<double *>(ang_out), 0, iters_out,
                                         incr_out, st, false, true);
    return lanczos_run_multi<float>(s, static_cast<const float *>(w), 1, 0, prefactor, tol, max_iter,
                                    static_cast<float *>(lin_out), static_cast<float *>(ang_out), 0, iters_out,
                                    incr_out, st, false, true);
}

// Internal declarations shared by the HIP translation units of librpy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "rpy.h"

namespace rpy {

// ---------------------------------------------------------------------------
// Device vector types: one particle's 3-vector padded to 4 lanes.
// ---------------------------------------------------------------------------
template <typename Real> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };
template <typename Real> using vec4_t = typename V4<Real>::type;

// Pair-kernel constants, all in units of k = 1/(8 pi eta) so that the pair
// loop never multiplies by k; the epilogue does it once per output.
//   far  (r >= 2a):  A = 1/r + (2a^2/3)/r^3      B = 1/r^3 - 2a^2/r^5
//                    G = 1/r^3  D = -1/(2r^3)    E = 3/(2r^5)
//   near (r <  2a):  A = 4/(3a) - 3r/(8a^2)      B = 1/(8a^2 r)
//                    G = 1/(2a^3) - 3r/(16a^4)
//                    D = 1/a^3 - 27r/(32a^4) + 5r^3/(64a^6)
//                    E = 9/(32a^4 r) - 3r/(64a^6)
// contribution of source j to target i, d = X_i - X_j:
//   U_i += A F + B (d.F) d + G (T x d)
//   W_i += G (F x d) + D T + E (d.T) d
template <typename Real>
struct PairConst {
    Real two_a2_3;   // 2a^2/3
    Real m_two_a2;   // -2a^2
    Real four_a2;    // (2a)^2, near-branch threshold on r^2
    Real nA0, nA1;   // 4/(3a), -3/(8a^2)
    Real nB;         // 1/(8a^2)
    Real nG0, nG1;   // 1/(2a^3), -3/(16a^4)
    Real nD0, nD1, nD3;  // 1/a^3, -27/(32a^4), 5/(64a^6)
    Real nE_1, nE1;  // 9/(32a^4), -3/(64a^6)
};

template <typename Real>
inline PairConst<Real> make_pair_const(double a) {
    PairConst<Real> c;
    const double a2 = a * a, a3 = a2 * a, a4 = a2 * a2, a6 = a3 * a3;
    c.two_a2_3 = Real(2.0 * a2 / 3.0);
    c.m_two_a2 = Real(-2.0 * a2);
    c.four_a2 = Real(4.0 * a2);
    c.nA0 = Real(4.0 / (3.0 * a));
    c.nA1 = Real(-3.0 / (8.0 * a2));
    c.nB = Real(1.0 / (8.0 * a2));
    c.nG0 = Real(1.0 / (2.0 * a3));
    c.nG1 = Real(-3.0 / (16.0 * a4));
    c.nD0 = Real(1.0 / a3);
    c.nD1 = Real(-27.0 / (32.0 * a4));
    c.nD3 = Real(5.0 / (64.0 * a6));
    c.nE_1 = Real(9.0 / (32.0 * a4));
    c.nE1 = Real(-3.0 / (64.0 * a6));
    return c;
}

// Tile configuration of the pair kernels.
struct TileConfig {
    int tm = 2;          // targets per lane (1, 2 or 4)
    int n_split = 0;     // source splits (0 = choose from N)
};

// Plain device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want);
    void release();
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Launchers (defined in rpy_kernels.hip).  All take the caller's stream.
// stage_positions: AoS n x 3 (float or double) -> vec4 of Real, counts non-finite entries.
template <typename Tin, typename Real>
hipError_t launch_stage_positions(const Tin *pos, int64_t n, vec4_t<Real> *out,
                                  unsigned *nonfinite, hipStream_t st);
// stage_vec: AoS n x 3 (or NULL = zeros) -> vec4 of Real.
template <typename Tin, typename Real>
hipError_t launch_stage_vec(const Tin *v, int64_t n, vec4_t<Real> *out, hipStream_t st);

// Pair sum: partial sums over source splits.
//   part layout: [split][component][n]  (FP32: 2*ncomp components: sums then
//   Neumaier compensations; FP64: ncomp components).
template <typename Real, bool ANG>
hipError_t launch_pair(const vec4_t<Real> *pos, const vec4_t<Real> *f, const vec4_t<Real> *t,
                       int64_t n, const PairConst<Real> &pc, const TileConfig &cfg,
                       int n_split, Real *part, hipStream_t st);

// Reduce partials over splits, scale by k = 1/(8 pi eta), write AoS n x 3 outputs.
template <typename Real, typename Tout, bool ANG>
hipError_t launch_reduce(const Real *part, int n_split, int64_t n, double k,
                         Tout *lin, Tout *ang, hipStream_t st);

template <typename T>
hipError_t launch_fill_zero(T *p, int64_t count, hipStream_t st);

// Choice of source splits for n particles; largest useful split count.
int choose_splits(int64_t n, int tm, bool fp64, bool ang);
int max_splits(int64_t n);
int targets_per_block(int tm);
int source_tile();

}  // namespace rpy

// Opaque solver object behind the C interface.
struct rpy_solver {
    rpy_periodicity per[3] = {RPY_OPEN, RPY_OPEN, RPY_OPEN};
    bool initialized = false;
    double eta = 0.0, radius = 0.0;
    bool angular = false;
    bool have_pos = false;
    int64_t n = 0;
    rpy_dtype dtype = RPY_F32;
    rpy::TileConfig cfg[2];   // pair-kernel tiles for products without / with the angular blocks
    rpy::DevBuf pos, f, t, part, flag;
    // Lanczos workspace (float64): basis, scratch vectors, tridiagonal data
    rpy::DevBuf lz_basis, lz_w, lz_scal, lz_red, lz_q, lz_vec, lz_mon;
    // launch timing (rpy_enable_timing): event pairs and pair counts per kernel class
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
    size_t ev_used[2] = {0, 0};
    double ev_pairs[2] = {0.0, 0.0};
    unsigned *host_flag = nullptr;   // pinned host word for flags
    double *host_scal = nullptr;     // pinned host scalars for Lanczos polling
    std::string err;
};

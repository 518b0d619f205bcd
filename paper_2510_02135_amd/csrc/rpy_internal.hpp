// Internal declarations shared by the HIP translation units of librpy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "rpy.h"
#include "rpy_pair.hpp"

namespace rpy {

struct PseState;   // triply periodic solver state (rpy_pse.hip)

constexpr int kKernelClasses = 4;   // rpy_kernel values
constexpr int kMaxRhs = 1024;       // vectors per multi-vector product

// Tile configuration of the pair kernels.
struct TileConfig {
    int tm = 2;          // targets per lane (1, 2 or 4), 0: symmetric pair mode (rpy_sym.hip), 3: fused small-N kernel
    int n_split = 0;     // source splits (0 = choose from N); symmetric mode: source blocks per task
    bool automatic = true;   // neither set nor tuned: the symmetric mode from kAutoSymN particles on
};
constexpr int64_t kAutoSymN = 32768;

// Plain device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want);
    void release();
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Task list of the symmetric pair mode (rpy_sym.hip), cached for (n, span, block).
struct SymTasks {
    DevBuf task, slot;
    DevBuf order;                 // the same tasks, those holding a diagonal block last
    std::vector<int> slot_host;   // first task of each target block, and the total
    int64_t n = -1;
    int span = 0, blk = 0, ntasks = 0;
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
    bool wall = false;          // (open, open, single_wall): Swan-Brady kernel with damping
    double wall_height = 0.0;   // z of the wall (rpy_set_parameter "wallHeight")
    rpy::PseState *pse = nullptr;   // (periodic, periodic, periodic): positively split Ewald
    bool initialized = false;
    double eta = 0.0, radius = 0.0;
    bool angular = false;
    bool have_pos = false;
    int64_t n = 0;
    rpy_dtype dtype = RPY_F32;
    rpy::TileConfig cfg[2];   // pair-kernel tiles for products without / with the angular blocks
    int multi_tm = 0;         // targets per lane of the multi-vector pair kernel (0 = automatic, 1, 2)
    rpy::DevBuf pos, f, t, part, flag;
    // Lanczos workspace (float64): basis, scratch vectors, tridiagonal data
    rpy::DevBuf lz_basis, lz_w, lz_scal, lz_red, lz_q, lz_vec, lz_mon, drift;
    // conjugate-gradient workspace (float64): x, r, p and a product slot per right-hand side; scalars
    rpy::DevBuf cg_vec, cg_scal;
    // symmetric pair mode: task lists of the forward and adjoint kernels, source-side partials
    rpy::SymTasks sym_fwd, sym_adj;
    rpy::DevBuf sym_jpart, sym_state;
    // preconditioned Lanczos: Cholesky blocks of groups of pc_group particles
    // (pc_parts = 1, or 2 with angular rows), valid for positions pc_version
    rpy::DevBuf pc_L, pc_tmp, pc_info;
    int pc_group = 0, pc_parts = 0;
    bool pc_valid = false;
    uint64_t pos_version = 0, pc_version = 0;
    void *blas = nullptr;   // library handle of the batched Cholesky
    int adjoint_mode = 0;     // rpy_set_adjoint_mode: 0 automatic, 1 one-sided, 2 symmetric
    // launch timing (rpy_enable_timing): event pairs and pair counts per kernel class
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[rpy::kKernelClasses];
    size_t ev_used[rpy::kKernelClasses] = {};
    double ev_pairs[rpy::kKernelClasses] = {};
    unsigned *host_flag = nullptr;   // pinned host word for flags
    double *host_stat = nullptr;     // pinned host copy of the Lanczos status blocks
    size_t host_stat_cap = 0;        // doubles in host_stat
    hipEvent_t lz_event = nullptr;   // Lanczos: end of an iteration's stopping test (host waits on it)
    std::string err;
};

// Triply periodic RPY mobility by the positively split Ewald method (gfx950).
//
// With periodic boundaries on all three axes (Sec. 3.5, "Positively Split
// Ewald (PSE)") the mobility is the lattice sum over wave vectors k != 0 of
// sinc^2(k a) (I - khat khat^T) / (eta k^2) e^{i k.(x_i - x_j)} / V, split
// with Hasimoto's function H(k, xi) = (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)}
// into two positive parts:
//   real space  sum over near pairs (minimum image, r < rc) of RPY(r) - Wr(r),
//               Wr the free-space transform of the H-weighted kernel, read
//               from a table built on the host by Gauss-Legendre quadrature;
//   wave space  Gaussian spreading of the forces to a grid, a forward FFT,
//               the scaling D(k) (I - khat khat^T) on the half spectrum, an
//               inverse FFT and Gaussian interpolation back (spectral Ewald:
//               the Gaussian's two factors are undone inside D(k)).
// Fluctuations with covariance M use the split: Lanczos on the real part
// plus a wave part drawn from independent Fourier-space normals (one
// inverse FFT).  Parameters: tolerance tol sets the real cutoff rc (|RPY -
// Wr| < tol mu0 beyond it, and the neglected pairs' root-mean-square sum at
// the suspension's density below tol mu0 / 2), the wave cutoff kc ((1 + q) e^{-q} = tol,
// q = kc^2/(4 xi^2)), the grid (Nyquist at 2 kc), the Gaussian width
// (aliasing of kc below tol) and its support P (truncation below tol).
//
// Data layout: particles are binned by tiles of 8^3 grid points (a counting
// sort; deterministic order: by tile, then by index).  The tiles serve both
// parts: the real-space sum scans the tiles within rc of a target's tile;
// spreading runs one workgroup per tile that gathers the particles whose
// Gaussian support reaches it (every grid point written once, no atomics);
// interpolation runs one wavefront per particle in tile order, lanes over
// the (y, z) support points so that neighbouring lanes read neighbouring
// grid words.  The grid is three real Nx x Ny x Nz arrays (z fastest), the
// spectrum three Nx x Ny x (Nz/2 + 1) complex arrays.  With these fixed
// orders a product is reproducible bit for bit.
#include "rpy_device.hpp"
#include "rpy_internal.hpp"
#include "rpy_solver_ops.hpp"

#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

namespace rpy {

namespace {

constexpr int kTable = 4096;         // table intervals on [0, rc]
constexpr int kMaxSupport = 32;      // Gaussian support points per axis
constexpr int kMaxGridAxis = 4096;   // grid points per axis
constexpr int kScanBlock = 1024;     // threads of the scan kernels (4 items each)
constexpr int kTile = 8;             // grid points per tile side (tiles bin the particles)
constexpr int kMaxTileNbr = 343;     // neighbour tiles scanned by a tile (reach <= 3)

template <typename Real> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };
template <typename Real> using vec2_t = typename V2<Real>::type;

template <typename Real> struct FftTypes;
template <> struct FftTypes<float> { using complex_t = hipfftComplex; };
template <> struct FftTypes<double> { using complex_t = hipfftDoubleComplex; };

}  // namespace

// Device constants of one PSE configuration.
template <typename Real>
struct PseConst {
    Real L[3], invL[3];
    int ncell[3];               // tiles of kTile^3 grid points per axis (the last may be partial)
    Real cell_scale[3];         // 1 / (kTile h): position -> tile
    int nbr_lo[3], nbr_cnt[3];  // tiles within rc of a tile: offsets lo .. lo + cnt - 1 per axis
    int sp_lo[3], sp_cnt[3];    // tiles whose particles' supports can reach a tile
    Real rc2, inv_dr;
    int grid[3];
    Real h[3], invh[3];
    int P;
    Real inv_2s2;             // 1 / (2 sigma^2)
    Real gnorm3;              // (2 pi sigma^2)^{-3/2}
    Real xi, a, eta;
    Real two_pi_invL[3];
    Real sig2;
};

struct PseState {
    // parameters (rpy_set_parameter)
    double box[3] = {0.0, 0.0, 0.0};
    double psi = 0.0;   // splitting parameter xi; 0 = automatic
    double tol = 1e-4;
    // derived configuration, valid for key = (box, psi, tol, a, eta, n)
    bool ready = false;
    double key[8] = {};
    double xi = 0.0, rc = 0.0, sigma = 0.0, dr = 0.0;
    double h[3] = {}, qc = 0.0;
    int P = 0, grid[3] = {}, ncell[3] = {}, reach_real[3] = {}, reach_spread = 0;
    std::vector<double> table;   // (f, g) pairs, kTable + 4 entries, in units of 1/(8 pi eta)
    DevBuf tab32, tab64;
    // cell list and sorted particles
    DevBuf count, start, scan_tmp, cell_of, order, wrapped, spos, sfrc;
    // grids
    DevBuf rgrid, cgrid;
    hipfftHandle plan_r2c[2] = {0, 0}, plan_c2r[2] = {0, 0};
    int plan_grid[2][3] = {};
    bool real_only = false;
};

namespace {

// ---------------------------------------------------------------------------
// Host: quadrature of the wave-space kernel's free-space transform
// ---------------------------------------------------------------------------

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_m).
void gauss_legendre(int m, std::vector<double> &x, std::vector<double> &w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// j0(x) - j1(x)/x and j2(x) (spherical Bessel functions), series below 0.5.
inline void bessel_pair(double x, double &a, double &b) {
    if (x < 0.5) {
        const double t = -0.5 * x * x;
        double pw = 1.0, dfa = 3.0;   // (2m+3)!!
        double sa = 0.0, sb = 0.0;
        double fact = 1.0, df5 = 15.0;   // m!, (2m+5)!!
        for (int m = 0; m < 9; ++m) {
            if (m > 0) {
                fact *= m;
                dfa *= (2.0 * m + 3.0);
                df5 *= (2.0 * m + 5.0);
            }
            sa += pw / fact * (2.0 * m + 2.0) / dfa;
            sb += pw / (fact * df5);
            pw *= t;
        }
        a = sa;
        b = x * x * sb;
        return;
    }
    const double s = std::sin(x), c = std::cos(x);
    const double ix = 1.0 / x, ix2 = ix * ix;
    a = s * ix - s * ix2 * ix + c * ix2;
    b = (3.0 * ix2 - 1.0) * s * ix - 3.0 * c * ix2;
}

struct WaveQuad {
    std::vector<double> q, w;   // nodes on [0, qtop] and weights times sinc^2 H (4/pi)
};

// Nodes for r up to rmax: panels of 16 Gauss points, at most 1.5 rad of
// q r per panel; the integrand sinc^2(q a) H(q, xi) is below 1e-19 past qtop.
WaveQuad make_quad(double xi, double a, double rmax) {
    const double qtop = 2.0 * xi * std::sqrt(48.0);
    const int panels = std::max(32, (int)std::ceil(qtop * std::max(rmax, a) / 1.5));
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
    WaveQuad wq;
    const double hp = qtop / panels;
    for (int p = 0; p < panels; ++p)
        for (int i = 0; i < 16; ++i) {
            const double q = hp * (p + 0.5 * (gx[i] + 1.0));
            const double qa = q * a;
            const double sinc = qa < 1e-8 ? 1.0 : std::sin(qa) / qa;
            const double t = q * q / (4.0 * xi * xi);
            wq.q.push_back(q);
            wq.w.push_back(0.5 * hp * gw[i] * sinc * sinc * (1.0 + t) * std::exp(-t) * 4.0 / M_PI);
        }
    return wq;
}

// Wr(r) = f I + g rhat rhat^T in units of 1/(8 pi eta).
inline void wave_kernel(const WaveQuad &wq, double r, double &f, double &g) {
    double sf = 0.0, sg = 0.0;
    for (size_t i = 0; i < wq.q.size(); ++i) {
        double a, b;
        bessel_pair(wq.q[i] * r, a, b);
        sf += wq.w[i] * a;
        sg += wq.w[i] * b;
    }
    f = sf;
    g = sg;
}

// Open RPY coefficients (units of 1/(8 pi eta)): A I + B r^2 rhat rhat^T.
inline void rpy_coeffs(double r, double a, double &A, double &Br2) {
    if (r < 2.0 * a) {
        A = 4.0 / (3.0 * a) - 3.0 * r / (8.0 * a * a);
        Br2 = r / (8.0 * a * a);
    } else {
        A = 1.0 / r + 2.0 * a * a / (3.0 * r * r * r);
        Br2 = 1.0 / r - 2.0 * a * a / (r * r * r);
    }
}

// Smallest grid size >= n that is a multiple of the tile (so that every tile
// is whole and the tile reaches below hold) with prime factors 2, 3, 5, 7.
int nice_fft_size(int n) {
    if (n < 8) n = 8;
    for (;; ++n) {
        if (n % kTile) continue;
        int m = n;
        for (int p : {2, 3, 5, 7})
            while (m % p == 0) m /= p;
        if (m == 1) return n;
    }
}

// Real-space cutoff: the smallest r >= 2a beyond which both the kernel
// K(r) = max(|A - f|, |A + B r^2 - f - g|) stays below tol mu0 (one close
// neighbour) and the root-mean-square sum of the neglected pairs at number
// density rho, sqrt(rho int_r^inf 4 pi s^2 K(s)^2 ds) (unit random forces),
// stays below tol mu0 / 2.  Scan of a grid of step 0.02/xi up to 2a + 12/xi.
double real_cutoff(double xi, double a, double tol, double rho) {
    const double step = 0.02 / xi, rmax = 2.0 * a + 12.0 / xi;
    const WaveQuad wq = make_quad(xi, a, rmax);
    const double mu0 = 4.0 / (3.0 * a);
    double tail = 0.0;
    for (double r = rmax; r >= 2.0 * a; r -= step) {
        double f, g, A, Br2;
        wave_kernel(wq, r, f, g);
        rpy_coeffs(r, a, A, Br2);
        const double k = std::max(std::fabs(A - f), std::fabs(A + Br2 - f - g));
        tail += 4.0 * M_PI * r * r * k * k * step;
        if (k > tol * mu0 || std::sqrt(rho * tail) > 0.5 * tol * mu0) return r + step;
    }
    return 2.0 * a;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device kernels
// ---------------------------------------------------------------------------
namespace {

template <typename Real>
__device__ __forceinline__ Real wrap_coord(Real x, Real L, Real invL) {
    Real w = x - L * floor(x * invL);
    if (w >= L) w -= L;
    if (w < Real(0)) w = Real(0);
    return w;
}

template <typename Real>
__device__ __forceinline__ int cell_coord(Real w, Real scale, int nc) {
    return min((int)(w * scale), nc - 1);
}

template <typename Real>
__global__ void __launch_bounds__(256) pse_bin(const vec4_t<Real> *__restrict__ pos, int n, PseConst<Real> c,
                                               int *__restrict__ count, int *__restrict__ cell_of,
                                               vec4_t<Real> *__restrict__ wrapped) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const vec4_t<Real> p = pos[i];
    vec4_t<Real> w;
    w.x = wrap_coord(p.x, c.L[0], c.invL[0]);
    w.y = wrap_coord(p.y, c.L[1], c.invL[1]);
    w.z = wrap_coord(p.z, c.L[2], c.invL[2]);
    w.w = Real(0);
    const int cx = cell_coord(w.x, c.cell_scale[0], c.ncell[0]);
    const int cy = cell_coord(w.y, c.cell_scale[1], c.ncell[1]);
    const int cz = cell_coord(w.z, c.cell_scale[2], c.ncell[2]);
    const int cell = (cx * c.ncell[1] + cy) * c.ncell[2] + cz;
    cell_of[i] = cell;
    wrapped[i] = w;
    atomicAdd(count + cell, 1);
}

// Exclusive scan, three passes: per-block scans of 4096 items with block
// totals, a scan of the totals (one block), then the offsets added.
__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const int t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    total = sh[kScanBlock - 1];
    const int incl = sh[tid];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanBlock) scan_blocks(const int *__restrict__ in, int count,
                                                          int *__restrict__ out, int *__restrict__ totals) {
    __shared__ int sh[kScanBlock];
    const int base = blockIdx.x * kScanBlock * 4 + threadIdx.x * 4;
    int v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < count ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < count) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) scan_totals(int *__restrict__ totals, int nblocks, int *__restrict__ out,
                                                          int count) {
    __shared__ int sh[kScanBlock];
    int carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += kScanBlock) {
        const int b = b0 + (int)threadIdx.x;
        const int v = b < nblocks ? totals[b] : 0;
        int total;
        const int ex = block_exclusive_scan(v, sh, total);
        if (b < nblocks) totals[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) out[count] = carry;
}

__global__ void __launch_bounds__(256) scan_add(int *__restrict__ out, int count, const int *__restrict__ totals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] += totals[i / (kScanBlock * 4)];
}

// Slot of each particle: start of its cell plus a rank taken by counting
// the cell down (which leaves count zeroed).
__global__ void __launch_bounds__(256) pse_place(int n, const int *__restrict__ cell_of, const int *__restrict__ start,
                                                 int *__restrict__ count, int *__restrict__ order) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int r = atomicSub(count + c, 1) - 1;
    order[start[c] + r] = i;
}

// Sort each cell's slots by particle index (a deterministic order):
// insertion sort for short cells, Shell sort (Ciura's gaps) otherwise.
__global__ void __launch_bounds__(256) pse_sort_cells(int ncells, const int *__restrict__ start,
                                                      int *__restrict__ order) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int *o = order + start[c];
    const int m = start[c + 1] - start[c];
    // Ciura's gaps, extended by factors of 2.25 for very full cells
    const int gaps[17] = {1149241, 510774, 227011, 100894, 44842, 19930, 8858, 3937,
                          1750, 701, 301, 132, 57, 23, 10, 4, 1};
    for (int gi = 0; gi < 17; ++gi) {
        const int g = gaps[gi];
        if (g >= m) continue;
        for (int i = g; i < m; ++i) {
            const int v = o[i];
            int j = i;
            while (j >= g && o[j - g] > v) {
                o[j] = o[j - g];
                j -= g;
            }
            o[j] = v;
        }
    }
}

template <typename Real>
__global__ void __launch_bounds__(256) pse_gather(int n, const int *__restrict__ order,
                                                  const vec4_t<Real> *__restrict__ wrapped,
                                                  const vec4_t<Real> *__restrict__ f, vec4_t<Real> *__restrict__ spos,
                                                  vec4_t<Real> *__restrict__ sfrc) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = order[s];
    spos[s] = wrapped[i];
    if (f) sfrc[s] = f[i];
}

// Cubic Lagrange interpolation of the (f, g) table at t = r / dr: nodes
// m-1 .. m+2 stored at m .. m+3 (entry 0 is r = -dr, the even mirror).
template <typename Real>
__device__ __forceinline__ void table_lookup(const vec2_t<Real> *__restrict__ tab, Real t, Real &f, Real &g) {
    int m = (int)t;
    m = min(m, kTable);
    const Real u = t - Real(m);
    const Real um1 = u - Real(1), um2 = u - Real(2), up1 = u + Real(1);
    const Real w0 = -u * um1 * um2 * Real(1.0 / 6.0);
    const Real w1 = up1 * um1 * um2 * Real(0.5);
    const Real w2 = -up1 * u * um2 * Real(0.5);
    const Real w3 = up1 * u * um1 * Real(1.0 / 6.0);
    const vec2_t<Real> a = tab[m], b = tab[m + 1], c = tab[m + 2], d = tab[m + 3];
    f = w0 * a.x + w1 * b.x + w2 * c.x + w3 * d.x;
    g = w0 * a.y + w1 * b.y + w2 * c.y + w3 * d.y;
}

template <typename Real>
__device__ __forceinline__ Real wave_reduce(Real v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Real part of one pair in k-units: (A - f) F + (B - g / r^2)(d.F) d, with
// the RPY coefficients A, B (overlap branch and r = 0 included) and Wr's
// (f, g) from the table.
template <typename Real>
__device__ __forceinline__ void real_pair(Real dx, Real dy, Real dz, Real r2, const vec4_t<Real> &F,
                                          const PairConst<Real> &pc, const vec2_t<Real> *__restrict__ tab,
                                          Real inv_dr, Real &u0, Real &u1, Real &u2) {
    Real A, B, r;
    if (r2 < pc.four_a2) {
        const Real rs = r2 > Real(0) ? rsq(r2) : Real(0);
        r = r2 * rs;
        A = fma(pc.nA1, r, pc.nA0);
        B = pc.nB * rs;
    } else {
        const Real ri = rsq(r2);
        const Real ri2 = ri * ri, ri3 = ri * ri2;
        r = r2 * ri;
        A = fma(pc.two_a2_3, ri3, ri);
        B = fma(pc.m_two_a2, ri3 * ri2, ri3);
    }
    Real f, g;
    table_lookup<Real>(tab, r * inv_dr, f, g);
    A -= f;
    if (r2 > Real(0)) B -= g / r2;
    const Real sdf = B * fma(dx, F.x, fma(dy, F.y, dz * F.z));
    u0 = fma(A, F.x, fma(sdf, dx, u0));
    u1 = fma(A, F.y, fma(sdf, dy, u1));
    u2 = fma(A, F.z, fma(sdf, dz, u2));
}

// Real-space part, one wavefront per tile.  The wavefront loads the particle
// ranges of the tiles within rc (at most kRealNbr of them) into LDS at once
// and scans their counts; the particles of those tiles then form one virtual
// list that the lanes take 64 at a time (virtual index -> tile by binary
// search), every loop uniform over the wavefront.  Each lane evaluates its
// source against the tile's targets, kRealTargets at a time held in
// registers (nearest image, pairs closer than rc); the per-target sums are
// reduced over the lanes in a fixed order and lane 0 writes (ADD = false) or
// adds k * sum into out[original index].
constexpr int kRealTargets = 8;
constexpr int kRealNbr = 343;                        // tiles within rc (reach <= 3)
constexpr int kRealPer = (kRealNbr + 63) / 64;       // neighbour entries per lane in the scan

template <typename Real, typename Tout, bool ADD>
__global__ void __launch_bounds__(256) pse_real_tiles(int ntiles, const vec4_t<Real> *__restrict__ spos,
                                                      const vec4_t<Real> *__restrict__ sfrc,
                                                      const int *__restrict__ order, const int *__restrict__ start,
                                                      PseConst<Real> c, PairConst<Real> pc,
                                                      const vec2_t<Real> *__restrict__ tab, Real kf,
                                                      Tout *__restrict__ out) {
    __shared__ int nb_first[4][kRealNbr], nb_pref[4][kRealNbr + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tile = blockIdx.x * 4 + wv;
    if (tile >= ntiles) return;   // whole wavefront; no workgroup barrier below
    const int ts = start[tile], te = start[tile + 1];
    if (ts == te) return;
    const int t2 = tile % c.ncell[2];
    const int t1 = (tile / c.ncell[2]) % c.ncell[1];
    const int t0 = tile / (c.ncell[2] * c.ncell[1]);
    int *nf = nb_first[wv], *np = nb_pref[wv];
    const int nnb = c.nbr_cnt[0] * c.nbr_cnt[1] * c.nbr_cnt[2];
    // lane l owns neighbour entries kRealPer l .. kRealPer l + kRealPer - 1
    int cnt[kRealPer], run = 0;
#pragma unroll
    for (int u = 0; u < kRealPer; ++u) {
        const int k = lane * kRealPer + u;
        cnt[u] = 0;
        if (k < nnb) {
            const int oz = k % c.nbr_cnt[2], oy = (k / c.nbr_cnt[2]) % c.nbr_cnt[1];
            const int ox = k / (c.nbr_cnt[2] * c.nbr_cnt[1]);
            int a = t0 + c.nbr_lo[0] + ox, b = t1 + c.nbr_lo[1] + oy, e = t2 + c.nbr_lo[2] + oz;
            a += a < 0 ? c.ncell[0] : (a >= c.ncell[0] ? -c.ncell[0] : 0);
            b += b < 0 ? c.ncell[1] : (b >= c.ncell[1] ? -c.ncell[1] : 0);
            e += e < 0 ? c.ncell[2] : (e >= c.ncell[2] ? -c.ncell[2] : 0);
            const int cell = (a * c.ncell[1] + b) * c.ncell[2] + e;
            const int s0 = start[cell];
            nf[k] = s0;
            cnt[u] = start[cell + 1] - s0;
        }
        run += cnt[u];
    }
    // exclusive scan of the lanes' totals, then each lane's entries
    int incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    int pre = incl - run;
#pragma unroll
    for (int u = 0; u < kRealPer; ++u) {
        const int k = lane * kRealPer + u;
        if (k < nnb) np[k] = pre;
        pre += cnt[u];
    }
    const int total = __shfl(incl, 63, 64);
    if (lane == 0) np[nnb] = total;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int tb = ts; tb < te; tb += kRealTargets) {
        const int nt = min(kRealTargets, te - tb);
        Real tx[kRealTargets], ty[kRealTargets], tz[kRealTargets];
        Real a0[kRealTargets], a1[kRealTargets], a2[kRealTargets];
#pragma unroll
        for (int t = 0; t < kRealTargets; ++t) {
            const vec4_t<Real> p = spos[tb + min(t, nt - 1)];
            tx[t] = p.x;
            ty[t] = p.y;
            tz[t] = p.z;
            a0[t] = a1[t] = a2[t] = Real(0);
        }
        for (int base = 0; base < total; base += 64) {
            const int v = base + lane;
            if (v < total) {
                int lo = 0, hi = nnb - 1;   // last k with np[k] <= v
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (np[mid] <= v) lo = mid; else hi = mid - 1;
                }
                const int j = nf[lo] + (v - np[lo]);
                const vec4_t<Real> sp = spos[j];
                const vec4_t<Real> F = sfrc[j];
#pragma unroll
                for (int t = 0; t < kRealTargets; ++t) {
                    if (t < nt) {
                        Real dx = tx[t] - sp.x, dy = ty[t] - sp.y, dz = tz[t] - sp.z;
                        dx -= c.L[0] * rint(dx * c.invL[0]);
                        dy -= c.L[1] * rint(dy * c.invL[1]);
                        dz -= c.L[2] * rint(dz * c.invL[2]);
                        const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                        if (r2 < c.rc2) real_pair<Real>(dx, dy, dz, r2, F, pc, tab, c.inv_dr, a0[t], a1[t], a2[t]);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kRealTargets; ++t) {
            if (t < nt) {
                const Real s0 = wave_reduce(a0[t]), s1 = wave_reduce(a1[t]), s2 = wave_reduce(a2[t]);
                if (lane == 0) {
                    const size_t o = (size_t)order[tb + t] * 3;
                    if (ADD) {
                        out[o + 0] = (Tout)((Tout)out[o + 0] + (Tout)(kf * s0));
                        out[o + 1] = (Tout)((Tout)out[o + 1] + (Tout)(kf * s1));
                        out[o + 2] = (Tout)((Tout)out[o + 2] + (Tout)(kf * s2));
                    } else {
                        out[o + 0] = (Tout)(kf * s0);
                        out[o + 1] = (Tout)(kf * s1);
                        out[o + 2] = (Tout)(kf * s2);
                    }
                }
            }
        }
    }
}

// Real-space part, fallback for cutoffs spanning more than kRealNbr tiles:
// one thread per target slot, the minimum image, pairs closer than rc.  Writes (ADD =
// false) or adds k * sum into out[original index].
template <typename Real, typename Tout, bool ADD>
__global__ void __launch_bounds__(256) pse_real_threads(int n, const vec4_t<Real> *__restrict__ spos,
                                                const vec4_t<Real> *__restrict__ sfrc, const int *__restrict__ order,
                                                const int *__restrict__ start, PseConst<Real> c, PairConst<Real> pc,
                                                const vec2_t<Real> *__restrict__ tab, Real kf, Tout *__restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const vec4_t<Real> pi = spos[s];
    const int cx = cell_coord(pi.x, c.cell_scale[0], c.ncell[0]);
    const int cy = cell_coord(pi.y, c.cell_scale[1], c.ncell[1]);
    const int cz = cell_coord(pi.z, c.cell_scale[2], c.ncell[2]);
    Real u0 = Real(0), u1 = Real(0), u2 = Real(0);
    for (int ox = 0; ox < c.nbr_cnt[0]; ++ox) {
        int gx = cx + c.nbr_lo[0] + ox;
        gx += gx < 0 ? c.ncell[0] : (gx >= c.ncell[0] ? -c.ncell[0] : 0);
        for (int oy = 0; oy < c.nbr_cnt[1]; ++oy) {
            int gy = cy + c.nbr_lo[1] + oy;
            gy += gy < 0 ? c.ncell[1] : (gy >= c.ncell[1] ? -c.ncell[1] : 0);
            for (int oz = 0; oz < c.nbr_cnt[2]; ++oz) {
                int gz = cz + c.nbr_lo[2] + oz;
                gz += gz < 0 ? c.ncell[2] : (gz >= c.ncell[2] ? -c.ncell[2] : 0);
                const int cell = (gx * c.ncell[1] + gy) * c.ncell[2] + gz;
                const int j1 = start[cell + 1];
                for (int j = start[cell]; j < j1; ++j) {
                    const vec4_t<Real> q = spos[j];
                    Real dx = pi.x - q.x, dy = pi.y - q.y, dz = pi.z - q.z;
                    dx -= c.L[0] * rint(dx * c.invL[0]);
                    dy -= c.L[1] * rint(dy * c.invL[1]);
                    dz -= c.L[2] * rint(dz * c.invL[2]);
                    const Real r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    if (r2 >= c.rc2) continue;
                    Real A, B, r;
                    if (r2 < pc.four_a2) {
                        const Real rs = r2 > Real(0) ? rsq(r2) : Real(0);
                        r = r2 * rs;
                        A = fma(pc.nA1, r, pc.nA0);
                        B = pc.nB * rs;
                    } else {
                        const Real ri = rsq(r2);
                        const Real ri2 = ri * ri, ri3 = ri * ri2;
                        r = r2 * ri;
                        A = fma(pc.two_a2_3, ri3, ri);
                        B = fma(pc.m_two_a2, ri3 * ri2, ri3);
                    }
                    Real f, g;
                    table_lookup<Real>(tab, r * c.inv_dr, f, g);
                    A -= f;
                    if (r2 > Real(0)) B -= g / r2;
                    const vec4_t<Real> F = sfrc[j];
                    const Real sdf = B * fma(dx, F.x, fma(dy, F.y, dz * F.z));
                    u0 = fma(A, F.x, fma(sdf, dx, u0));
                    u1 = fma(A, F.y, fma(sdf, dy, u1));
                    u2 = fma(A, F.z, fma(sdf, dz, u2));
                }
            }
        }
    }
    const size_t o = (size_t)order[s] * 3;
    if (ADD) {
        out[o + 0] = (Tout)((Tout)out[o + 0] + (Tout)(kf * u0));
        out[o + 1] = (Tout)((Tout)out[o + 1] + (Tout)(kf * u1));
        out[o + 2] = (Tout)((Tout)out[o + 2] + (Tout)(kf * u2));
    } else {
        out[o + 0] = (Tout)(kf * u0);
        out[o + 1] = (Tout)(kf * u1);
        out[o + 2] = (Tout)(kf * u2);
    }
}

// Support of a particle on one axis: first grid index and its offset
// (in grid units) from the particle, for P points centred on it.
template <typename Real>
__device__ __forceinline__ void support_axis(Real x, Real invh, int P, int &i0, Real &u0) {
    const Real u = x * invh;
    i0 = (P & 1) ? (int)rint(u) - (P - 1) / 2 : (int)floor(u) - P / 2 + 1;
    u0 = Real(i0) - u;
}

__device__ __forceinline__ int wrap_index(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// The 1-D Gaussian weights of one particle in LDS, w[axis][p] (lanes 0 ..
// P-1 of its wavefront write them; the caller synchronises the block).
template <typename Real>
__device__ __forceinline__ void support_weights(const vec4_t<Real> &p, const PseConst<Real> &c, Real *w, int *i0) {
    const int lane = threadIdx.x & 63;
    const Real xs[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Real u0;
        support_axis(xs[d], c.invh[d], c.P, i0[d], u0);
        if (lane < c.P) {
            const Real dd = (u0 + Real(lane)) * c.h[d];
            w[d * kMaxSupport + lane] = exp(-dd * dd * c.inv_2s2);
        }
    }
}

// Spreading by gathering: one workgroup per tile of kTile^3 grid points
// writes every point of its tile once (no atomics, no prior clearing, a
// fixed order of terms).  The particles of the tiles whose supports can
// reach it are scanned in rounds of 256; those whose P-point window
// (periodic) meets the tile on all three axes are compacted into LDS in a
// fixed order with their Gaussian weights at the tile's 8 points per axis
// (zero outside the window) and their force; each thread then sums its two
// points' terms, grid[m] = gnorm3 sum_j wx wy wz F_j.
template <typename Real>
__device__ __forceinline__ bool window_meets_tile(Real u, int P, int g0, int npts, int N, int &i0) {
    Real u0;
    support_axis(u, Real(1), P, i0, u0);
    int d0 = (g0 - i0) % N;
    if (d0 < 0) d0 += N;
    // points g0 .. g0 + npts - 1 meet the window [i0, i0 + P) mod N
    return d0 < P || d0 + npts > N;
}

template <typename Real>
__global__ void __launch_bounds__(256) pse_spread_tiles(const vec4_t<Real> *__restrict__ spos,
                                                        const vec4_t<Real> *__restrict__ sfrc,
                                                        const int *__restrict__ start, PseConst<Real> c,
                                                        Real *__restrict__ grid) {
    __shared__ Real sw[3][kTile][256];
    __shared__ vec4_t<Real> sf[256];
    __shared__ int nb_first[kMaxTileNbr], nb_pref[kMaxTileNbr + 1];
    __shared__ int wave_hits[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int tile = blockIdx.x;
    const int t2 = tile % c.ncell[2];
    const int t1 = (tile / c.ncell[2]) % c.ncell[1];
    const int t0 = tile / (c.ncell[2] * c.ncell[1]);
    const int g0[3] = {t0 * kTile, t1 * kTile, t2 * kTile};
    int npts[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) npts[d] = min(kTile, c.grid[d] - g0[d]);
    // neighbour tiles and the prefix sums of their particle counts
    const int nnb = c.sp_cnt[0] * c.sp_cnt[1] * c.sp_cnt[2];
    for (int k = tid; k < nnb; k += 256) {
        const int oz = k % c.sp_cnt[2], oy = (k / c.sp_cnt[2]) % c.sp_cnt[1], ox = k / (c.sp_cnt[2] * c.sp_cnt[1]);
        int a = t0 + c.sp_lo[0] + ox, b = t1 + c.sp_lo[1] + oy, e = t2 + c.sp_lo[2] + oz;
        a += a < 0 ? c.ncell[0] : (a >= c.ncell[0] ? -c.ncell[0] : 0);
        b += b < 0 ? c.ncell[1] : (b >= c.ncell[1] ? -c.ncell[1] : 0);
        e += e < 0 ? c.ncell[2] : (e >= c.ncell[2] ? -c.ncell[2] : 0);
        const int cell = (a * c.ncell[1] + b) * c.ncell[2] + e;
        nb_first[k] = start[cell];
        nb_pref[k + 1] = start[cell + 1] - start[cell];
    }
    __syncthreads();
    if (tid == 0) {
        nb_pref[0] = 0;
        for (int k = 0; k < nnb; ++k) nb_pref[k + 1] += nb_pref[k];
    }
    __syncthreads();
    const int total = nb_pref[nnb];
    // this thread's points: (lx, ly, lz) and (lx + 4, ly, lz)
    const int lz = tid & 7, ly = (tid >> 3) & 7, lx = tid >> 6;
    Real a0 = Real(0), a1 = Real(0), a2 = Real(0), b0 = Real(0), b1 = Real(0), b2 = Real(0);
    for (int base = 0; base < total; base += 256) {
        const int v = base + tid;
        bool hit = false;
        int j = 0, i0[3] = {0, 0, 0};
        Real u[3] = {Real(0), Real(0), Real(0)};
        if (v < total) {
            int lo = 0, hi = nnb - 1;   // last k with nb_pref[k] <= v
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (nb_pref[mid] <= v) lo = mid; else hi = mid - 1;
            }
            j = nb_first[lo] + (v - nb_pref[lo]);
            const vec4_t<Real> p = spos[j];
            u[0] = p.x * c.invh[0];
            u[1] = p.y * c.invh[1];
            u[2] = p.z * c.invh[2];
            hit = window_meets_tile(u[0], c.P, g0[0], npts[0], c.grid[0], i0[0]) &&
                  window_meets_tile(u[1], c.P, g0[1], npts[1], c.grid[1], i0[1]) &&
                  window_meets_tile(u[2], c.P, g0[2], npts[2], c.grid[2], i0[2]);
        }
        // fixed-order compaction: wave prefix by ballot, waves in order
        const unsigned long long mask = __ballot(hit);
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wave_hits[wv] = __popcll(mask);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wv; ++w) off += wave_hits[w];
        const int m = wave_hits[0] + wave_hits[1] + wave_hits[2] + wave_hits[3];
        if (hit) {
            const int slot = off + rank;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int l = 0; l < kTile; ++l) {
                    Real w = Real(0);
                    const int g = g0[d] + l;
                    if (l < npts[d]) {
                        int dd = (g - i0[d]) % c.grid[d];
                        if (dd < 0) dd += c.grid[d];
                        if (dd < c.P) {
                            const Real x = (Real(i0[d] + dd) - u[d]) * c.h[d];
                            w = exp(-x * x * c.inv_2s2);
                        }
                    }
                    sw[d][l][slot] = w;
                }
            }
            sf[slot] = sfrc[j];
        }
        __syncthreads();
        for (int k = 0; k < m; ++k) {
            const Real wyz = sw[1][ly][k] * sw[2][lz][k];
            const Real p0 = sw[0][lx][k] * wyz, p1 = sw[0][lx + 4][k] * wyz;
            const vec4_t<Real> F = sf[k];
            a0 = fma(p0, F.x, a0);
            a1 = fma(p0, F.y, a1);
            a2 = fma(p0, F.z, a2);
            b0 = fma(p1, F.x, b0);
            b1 = fma(p1, F.y, b1);
            b2 = fma(p1, F.z, b2);
        }
        __syncthreads();
    }
    const size_t ng = (size_t)c.grid[0] * c.grid[1] * c.grid[2];
    if (ly < npts[1] && lz < npts[2]) {
        const size_t gyz = (size_t)(g0[1] + ly) * c.grid[2] + (g0[2] + lz);
        if (lx < npts[0]) {
            const size_t idx = (size_t)(g0[0] + lx) * c.grid[1] * c.grid[2] + gyz;
            grid[idx] = c.gnorm3 * a0;
            grid[ng + idx] = c.gnorm3 * a1;
            grid[2 * ng + idx] = c.gnorm3 * a2;
        }
        if (lx + 4 < npts[0]) {
            const size_t idx = (size_t)(g0[0] + lx + 4) * c.grid[1] * c.grid[2] + gyz;
            grid[idx] = c.gnorm3 * b0;
            grid[ng + idx] = c.gnorm3 * b1;
            grid[2 * ng + idx] = c.gnorm3 * b2;
        }
    }
}

// Interpolation: one wavefront per particle, out[i] (+)= scale * sum_m
// u(x_m) g(x_m - x_i) over the support.
template <typename Real, typename Tout, bool ADD>
__global__ void __launch_bounds__(256) pse_interp(int n, const vec4_t<Real> *__restrict__ spos,
                                                  const int *__restrict__ order, PseConst<Real> c,
                                                  const Real *__restrict__ grid, Real scale, Tout *__restrict__ out) {
    __shared__ Real wsh[4][3 * kMaxSupport];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * 4 + wv;
    const bool active = s < n;   // uniform over the wavefront
    const vec4_t<Real> p = spos[active ? s : 0];
    int i0[3];
    Real *w = wsh[wv];
    support_weights(p, c, w, i0);
    __syncthreads();
    if (!active) return;
    const int P = c.P, P2 = P * P;
    const size_t ng = (size_t)c.grid[0] * c.grid[1] * c.grid[2];
    Real a0 = Real(0), a1 = Real(0), a2 = Real(0);
    for (int e = lane; e < P2; e += 64) {
        const int iy = e / P, iz = e - iy * P;
        const int gy = wrap_index(i0[1] + iy, c.grid[1]);
        const int gz = wrap_index(i0[2] + iz, c.grid[2]);
        const Real wyz = w[kMaxSupport + iy] * w[2 * kMaxSupport + iz];
        Real s0 = Real(0), s1 = Real(0), s2 = Real(0);
        for (int ix = 0; ix < P; ++ix) {
            const int gx = wrap_index(i0[0] + ix, c.grid[0]);
            const size_t idx = ((size_t)gx * c.grid[1] + gy) * c.grid[2] + gz;
            const Real wx = w[ix];
            s0 = fma(wx, grid[idx], s0);
            s1 = fma(wx, grid[ng + idx], s1);
            s2 = fma(wx, grid[2 * ng + idx], s2);
        }
        a0 = fma(wyz, s0, a0);
        a1 = fma(wyz, s1, a1);
        a2 = fma(wyz, s2, a2);
    }
    a0 = wave_reduce(a0);
    a1 = wave_reduce(a1);
    a2 = wave_reduce(a2);
    if (lane == 0) {
        const Real f = scale * c.gnorm3;
        const size_t o = (size_t)order[s] * 3;
        if (ADD) {
            out[o + 0] = (Tout)((Tout)out[o + 0] + (Tout)(f * a0));
            out[o + 1] = (Tout)((Tout)out[o + 1] + (Tout)(f * a1));
            out[o + 2] = (Tout)((Tout)out[o + 2] + (Tout)(f * a2));
        } else {
            out[o + 0] = (Tout)(f * a0);
            out[o + 1] = (Tout)(f * a1);
            out[o + 2] = (Tout)(f * a2);
        }
    }
}

// Wave vector of half-spectrum entry e; false for k = 0 and Nyquist entries.
template <typename Real>
__device__ __forceinline__ bool wave_vector(int64_t e, const PseConst<Real> &c, int nzh, int &ix, int &iy, int &iz,
                                            Real &kx, Real &ky, Real &kz) {
    iz = (int)(e % nzh);
    const int64_t t = e / nzh;
    iy = (int)(t % c.grid[1]);
    ix = (int)(t / c.grid[1]);
    const int mx = ix <= c.grid[0] / 2 ? ix : ix - c.grid[0];
    const int my = iy <= c.grid[1] / 2 ? iy : iy - c.grid[1];
    const int mz = iz;
    const bool nyq = (c.grid[0] % 2 == 0 && ix == c.grid[0] / 2) || (c.grid[1] % 2 == 0 && iy == c.grid[1] / 2) ||
                     (c.grid[2] % 2 == 0 && iz == c.grid[2] / 2);
    kx = c.two_pi_invL[0] * Real(mx);
    ky = c.two_pi_invL[1] * Real(my);
    kz = c.two_pi_invL[2] * Real(mz);
    return !nyq && (mx | my | mz) != 0;
}

// sinc^2(k a) H(k, xi) e^{sigma^2 k^2} / (eta k^2): the wave kernel with the
// two Gaussian factors of spreading and interpolation undone.
template <typename Real>
__device__ __forceinline__ Real wave_scale(Real k2, const PseConst<Real> &c) {
    const Real k = sqrt(k2);
    const Real ka = k * c.a;
    const Real sinc = ka < Real(1e-4) ? Real(1) - ka * ka * Real(1.0 / 6.0) : sin(ka) / ka;
    const Real q = k2 / (Real(4) * c.xi * c.xi);
    return sinc * sinc * (Real(1) + q) * exp(c.sig2 * k2 - q) / (c.eta * k2);
}

template <typename Real>
__global__ void __launch_bounds__(256) pse_scale(typename FftTypes<Real>::complex_t *__restrict__ spec, int64_t nh,
                                                 int nzh, PseConst<Real> c, Real inv_ng) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nh) return;
    int ix, iy, iz;
    Real kx, ky, kz;
    auto *v0 = spec + e;
    auto *v1 = spec + nh + e;
    auto *v2 = spec + 2 * nh + e;
    if (!wave_vector(e, c, nzh, ix, iy, iz, kx, ky, kz)) {
        v0->x = v0->y = v1->x = v1->y = v2->x = v2->y = Real(0);
        return;
    }
    const Real k2 = fma(kx, kx, fma(ky, ky, kz * kz));
    const Real D = wave_scale(k2, c) * inv_ng;
    const Real ik = rsq(k2);
    const Real hx = kx * ik, hy = ky * ik, hz = kz * ik;
    const Real re = hx * v0->x + hy * v1->x + hz * v2->x;
    const Real im = hx * v0->y + hy * v1->y + hz * v2->y;
    v0->x = D * (v0->x - hx * re);
    v0->y = D * (v0->y - hx * im);
    v1->x = D * (v1->x - hy * re);
    v1->y = D * (v1->y - hy * im);
    v2->x = D * (v2->x - hz * re);
    v2->y = D * (v2->y - hz * im);
}

// Fourier-space fluctuations: entry e of the half spectrum gets
// sqrt(D(k) / Ng) (I - khat khat^T) zeta_k, zeta_k complex unit normals from
// the noise array (3 x Nx x Ny x nzh x 2 reals) with zeta_{-k} =
// conj(zeta_k) on the planes kz = 0 and kz = Nz/2 that hold both: there the
// entry with (ix, iy) after its partner's (-ix, -iy) lexicographically
// takes the conjugate of the partner's numbers, a self-conjugate entry the
// real part alone; elsewhere zeta = (re + i im) / sqrt(2).
template <typename Real>
__global__ void __launch_bounds__(256) pse_noise(typename FftTypes<Real>::complex_t *__restrict__ spec, int64_t nh,
                                                 int nzh, PseConst<Real> c, Real inv_ng,
                                                 const Real *__restrict__ noise) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nh) return;
    int ix, iy, iz;
    Real kx, ky, kz;
    auto *v0 = spec + e;
    auto *v1 = spec + nh + e;
    auto *v2 = spec + 2 * nh + e;
    if (!wave_vector(e, c, nzh, ix, iy, iz, kx, ky, kz)) {
        v0->x = v0->y = v1->x = v1->y = v2->x = v2->y = Real(0);
        return;
    }
    const bool paired = iz == 0 || (c.grid[2] % 2 == 0 && iz == c.grid[2] / 2);
    int64_t src = e;
    Real sim = Real(1), sre = Real(0.70710678118654752440);
    if (paired) {
        const int px = ix == 0 ? 0 : c.grid[0] - ix;
        const int py = iy == 0 ? 0 : c.grid[1] - iy;
        const int64_t own = (int64_t)ix * c.grid[1] + iy, mate = (int64_t)px * c.grid[1] + py;
        if (own == mate) {
            sre = Real(1);
            sim = Real(0);
        } else if (own > mate) {
            src = ((int64_t)px * c.grid[1] + py) * nzh + iz;
            sim = Real(-1);
        }
    }
    Real zr[3], zi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const Real *nu = noise + 2 * ((size_t)d * nh + src);
        zr[d] = sre * nu[0];
        zi[d] = sim * sre * nu[1];
    }
    const Real k2 = fma(kx, kx, fma(ky, ky, kz * kz));
    const Real amp = sqrt(wave_scale(k2, c) * inv_ng);
    const Real ik = rsq(k2);
    const Real hx = kx * ik, hy = ky * ik, hz = kz * ik;
    const Real re = hx * zr[0] + hy * zr[1] + hz * zr[2];
    const Real im = hx * zi[0] + hy * zi[1] + hz * zi[2];
    v0->x = amp * (zr[0] - hx * re);
    v0->y = amp * (zi[0] - hx * im);
    v1->x = amp * (zr[1] - hy * re);
    v1->y = amp * (zi[1] - hy * im);
    v2->x = amp * (zr[2] - hz * re);
    v2->y = amp * (zi[2] - hz * im);
}

template <typename T>
__global__ void __launch_bounds__(256) pse_fill_zero(T *__restrict__ p, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = T(0);
}

template <typename T>
hipError_t fill_zero(T *p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL((pse_fill_zero<T>), dim3((unsigned)blocks), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
// Host: configuration, plans, products
// ---------------------------------------------------------------------------

namespace {

const char *fft_error(hipfftResult r) {
    switch (r) {
        case HIPFFT_SUCCESS: return "success";
        case HIPFFT_ALLOC_FAILED: return "allocation failed";
        case HIPFFT_INVALID_VALUE: return "invalid value";
        case HIPFFT_EXEC_FAILED: return "execution failed";
        case HIPFFT_SETUP_FAILED: return "setup failed";
        case HIPFFT_INVALID_SIZE: return "invalid size";
        default: return "error";
    }
}

#define FFT_TRY(s, expr)                                                                              \
    do {                                                                                              \
        hipfftResult r_ = (expr);                                                                     \
        if (r_ != HIPFFT_SUCCESS)                                                                     \
            return fail((s), r_ == HIPFFT_ALLOC_FAILED ? RPY_ERR_OUT_OF_MEMORY : RPY_ERR_HIP,        \
                        std::string("hipFFT ") + fft_error(r_) + " in " #expr);                       \
    } while (0)

void destroy_plans(PseState *p) {
    for (int d = 0; d < 2; ++d) {
        if (p->plan_r2c[d]) (void)hipfftDestroy(p->plan_r2c[d]);
        if (p->plan_c2r[d]) (void)hipfftDestroy(p->plan_c2r[d]);
        p->plan_r2c[d] = p->plan_c2r[d] = 0;
    }
}

template <typename Real>
PseConst<Real> make_const(const rpy_solver *s) {
    const PseState &p = *s->pse;
    PseConst<Real> c;
    for (int d = 0; d < 3; ++d) {
        c.L[d] = Real(p.box[d]);
        c.invL[d] = Real(1.0 / p.box[d]);
        c.ncell[d] = p.ncell[d];
        c.cell_scale[d] = Real(1.0 / (kTile * p.h[d]));
        const int wr = 2 * p.reach_real[d] + 1, ws = 2 * p.reach_spread + 1;
        c.nbr_cnt[d] = std::min(wr, p.ncell[d]);
        c.nbr_lo[d] = p.ncell[d] >= wr ? -p.reach_real[d] : 0;
        c.sp_cnt[d] = std::min(ws, p.ncell[d]);
        c.sp_lo[d] = p.ncell[d] >= ws ? -p.reach_spread : 0;
        c.grid[d] = p.grid[d];
        c.h[d] = Real(p.h[d]);
        c.invh[d] = Real(1.0 / p.h[d]);
        c.two_pi_invL[d] = Real(2.0 * M_PI / p.box[d]);
    }
    c.rc2 = Real(p.rc * p.rc);
    c.inv_dr = Real(1.0 / p.dr);
    c.P = p.P;
    c.inv_2s2 = Real(1.0 / (2.0 * p.sigma * p.sigma));
    c.gnorm3 = Real(std::pow(2.0 * M_PI * p.sigma * p.sigma, -1.5));
    c.xi = Real(p.xi);
    c.a = Real(s->radius);
    c.eta = Real(s->eta);
    c.sig2 = Real(p.sigma * p.sigma);
    return c;
}

// Derived configuration for the current parameters (host work only; the
// tables are uploaded here).
rpy_status configure(rpy_solver *s) {
    PseState &p = *s->pse;
    const double key[8] = {p.box[0], p.box[1], p.box[2], p.psi, p.tol, s->radius, s->eta, (double)s->n};
    if (p.ready && std::memcmp(key, p.key, sizeof(key)) == 0) return RPY_OK;
    p.ready = false;
    for (int d = 0; d < 3; ++d)
        if (!(p.box[d] > 0.0)) return fail(s, RPY_ERR_INVALID_ARG, "the periodic box needs Lx, Ly and Lz > 0");
    const double a = s->radius, tol = p.tol;
    const double lmin = std::min(p.box[0], std::min(p.box[1], p.box[2]));
    double xi = p.psi;
    if (!(xi > 0.0)) {
        // automatic: xi = rho^{1/3} balances near pairs against grid points
        // per particle at the library's grid rules, with rc < L/2
        xi = std::cbrt(std::max<double>(s->n, 1) / (p.box[0] * p.box[1] * p.box[2]));
        xi = std::max(xi, 0.05 / a);
    }
    const double rho = std::max<double>(s->n, 1) / (p.box[0] * p.box[1] * p.box[2]);
    double rc = real_cutoff(xi, a, tol, rho);
    if (!(p.psi > 0.0))
        for (int it = 0; it < 40 && rc >= 0.5 * lmin; ++it) {
            xi *= 1.25;
            rc = real_cutoff(xi, a, tol, rho);
        }
    if (rc >= 0.5 * lmin)
        return fail(s, RPY_ERR_INVALID_ARG,
                    "the real-space cutoff " + std::to_string(rc) + " reaches half the box; raise psi");
    // wave cutoff, grid, Gaussian
    const double ell = std::log(1.0 / tol);
    double q = ell;
    for (int it = 0; it < 60; ++it) q = ell + std::log1p(q);
    const double kc = 2.0 * xi * std::sqrt(q);
    const double hmax = M_PI / (2.0 * kc);
    int grid[3];
    double h[3];
    for (int d = 0; d < 3; ++d) {
        const double want = std::ceil(p.box[d] / hmax);
        if (want > kMaxGridAxis)
            return fail(s, RPY_ERR_INVALID_ARG, "the wave-space grid would exceed 4096 points per axis; lower psi");
        grid[d] = nice_fft_size((int)want);
        if (grid[d] > kMaxGridAxis)
            return fail(s, RPY_ERR_INVALID_ARG, "the wave-space grid would exceed 4096 points per axis; lower psi");
        h[d] = p.box[d] / grid[d];
    }
    if ((double)grid[0] * grid[1] * grid[2] > 1.5e9)
        return fail(s, RPY_ERR_INVALID_ARG, "the wave-space grid would exceed 1.5e9 points; lower psi");
    const double hx = std::max(h[0], std::max(h[1], h[2])), hn = std::min(h[0], std::min(h[1], h[2]));
    const double kn = M_PI / hx;
    const double sig2 = ell / (2.0 * kn * kn * (1.0 - kc / kn));
    const double sigma = std::sqrt(sig2);
    const int P = (int)std::ceil(2.0 * sigma * std::sqrt(2.0 * ell) / hn);
    if (P > kMaxSupport)
        return fail(s, RPY_ERR_INVALID_ARG, "tolerance too small: the Gaussian support exceeds 32 points");
    for (int d = 0; d < 3; ++d)
        if (P > grid[d]) return fail(s, RPY_ERR_INVALID_ARG, "the Gaussian support exceeds the grid");
    // particles are binned by tiles of kTile^3 grid points; a tile's real-space
    // neighbours lie within ceil(rc / (kTile h)) tiles, the supports that can
    // reach it within ceil((P/2 + 1) / kTile)
    int nc[3], reach[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = (grid[d] + kTile - 1) / kTile;
        reach[d] = (int)std::ceil(rc / (kTile * h[d]));
    }
    const int reach_sp = (int)std::ceil((0.5 * P + 1.0) / kTile);

    if (std::pow(std::min(2 * reach_sp + 1, std::max(nc[0], std::max(nc[1], nc[2]))), 3) > kMaxTileNbr)
        return fail(s, RPY_ERR_INVALID_ARG, "tolerance too small: the Gaussian support reaches too many tiles");
    // table of Wr on [-dr, rc + 2 dr]
    const double dr = rc / kTable;
    const WaveQuad wq = make_quad(xi, a, rc + 3.0 * dr);
    p.table.assign(2 * (kTable + 4), 0.0);
    for (int m = 0; m < kTable + 4; ++m) {
        double f, g;
        wave_kernel(wq, std::fabs((m - 1) * dr), f, g);
        p.table[2 * m] = f;
        p.table[2 * m + 1] = g;
    }
    std::vector<float> t32(p.table.begin(), p.table.end());
    HIP_TRY(s, p.tab64.ensure(sizeof(double) * p.table.size()));
    HIP_TRY(s, p.tab32.ensure(sizeof(float) * t32.size()));
    HIP_TRY(s, hipMemcpy(p.tab64.p, p.table.data(), sizeof(double) * p.table.size(), hipMemcpyHostToDevice));
    HIP_TRY(s, hipMemcpy(p.tab32.p, t32.data(), sizeof(float) * t32.size(), hipMemcpyHostToDevice));
    p.xi = xi;
    p.rc = rc;
    p.dr = dr;
    p.qc = kc;
    p.sigma = sigma;
    p.P = P;
    for (int d = 0; d < 3; ++d) {
        p.grid[d] = grid[d];
        p.h[d] = h[d];
        p.ncell[d] = nc[d];
        p.reach_real[d] = reach[d];
    }
    p.reach_spread = reach_sp;
    std::memcpy(p.key, key, sizeof(key));
    p.ready = true;
    return RPY_OK;
}

template <typename Real>
rpy_status ensure_plans(rpy_solver *s) {
    PseState &p = *s->pse;
    const int d = std::is_same<Real, double>::value ? 1 : 0;
    if (p.plan_r2c[d] && std::memcmp(p.plan_grid[d], p.grid, sizeof(p.grid)) == 0) return RPY_OK;
    if (p.plan_r2c[d]) (void)hipfftDestroy(p.plan_r2c[d]);
    if (p.plan_c2r[d]) (void)hipfftDestroy(p.plan_c2r[d]);
    p.plan_r2c[d] = p.plan_c2r[d] = 0;
    int dims[3] = {p.grid[0], p.grid[1], p.grid[2]};
    const int nr = dims[0] * dims[1] * dims[2];
    const int nc = dims[0] * dims[1] * (dims[2] / 2 + 1);
    FFT_TRY(s, hipfftPlanMany(&p.plan_r2c[d], 3, dims, nullptr, 1, nr, nullptr, 1, nc, d ? HIPFFT_D2Z : HIPFFT_R2C, 3));
    FFT_TRY(s, hipfftPlanMany(&p.plan_c2r[d], 3, dims, nullptr, 1, nc, nullptr, 1, nr, d ? HIPFFT_Z2D : HIPFFT_C2R, 3));
    std::memcpy(p.plan_grid[d], p.grid, sizeof(p.grid));
    return RPY_OK;
}

template <typename Real>
rpy_status fft_forward(rpy_solver *s, hipStream_t st) {
    PseState &p = *s->pse;
    const int d = std::is_same<Real, double>::value ? 1 : 0;
    FFT_TRY(s, hipfftSetStream(p.plan_r2c[d], st));
    if constexpr (std::is_same<Real, double>::value)
        FFT_TRY(s, hipfftExecD2Z(p.plan_r2c[d], p.rgrid.as<double>(), p.cgrid.as<hipfftDoubleComplex>()));
    else
        FFT_TRY(s, hipfftExecR2C(p.plan_r2c[d], p.rgrid.as<float>(), p.cgrid.as<hipfftComplex>()));
    return RPY_OK;
}

template <typename Real>
rpy_status fft_inverse(rpy_solver *s, hipStream_t st) {
    PseState &p = *s->pse;
    const int d = std::is_same<Real, double>::value ? 1 : 0;
    FFT_TRY(s, hipfftSetStream(p.plan_c2r[d], st));
    if constexpr (std::is_same<Real, double>::value)
        FFT_TRY(s, hipfftExecZ2D(p.plan_c2r[d], p.cgrid.as<hipfftDoubleComplex>(), p.rgrid.as<double>()));
    else
        FFT_TRY(s, hipfftExecC2R(p.plan_c2r[d], p.cgrid.as<hipfftComplex>(), p.rgrid.as<float>()));
    return RPY_OK;
}

// Cell list of the positions `pos` (vec4, n) with the staged vectors f
// gathered into slot order (f may be NULL: positions only).
template <typename Real>
rpy_status build_cells(rpy_solver *s, const vec4_t<Real> *pos, const vec4_t<Real> *f, const PseConst<Real> &c,
                       hipStream_t st) {
    PseState &p = *s->pse;
    const int64_t n = s->n;
    const int64_t ncells = (int64_t)p.ncell[0] * p.ncell[1] * p.ncell[2];
    const int64_t sblocks = (ncells + 4 * kScanBlock - 1) / (4 * kScanBlock);
    HIP_TRY(s, p.count.ensure(sizeof(int) * ncells));
    HIP_TRY(s, p.start.ensure(sizeof(int) * (ncells + 1)));
    HIP_TRY(s, p.scan_tmp.ensure(sizeof(int) * sblocks));
    HIP_TRY(s, p.cell_of.ensure(sizeof(int) * n));
    HIP_TRY(s, p.order.ensure(sizeof(int) * n));
    HIP_TRY(s, p.wrapped.ensure(sizeof(vec4_t<Real>) * n));
    HIP_TRY(s, p.spos.ensure(sizeof(vec4_t<Real>) * n));
    HIP_TRY(s, p.sfrc.ensure(sizeof(vec4_t<Real>) * n));
    HIP_TRY(s, fill_zero<int>(p.count.as<int>(), ncells, st));
    hipLaunchKernelGGL((pse_bin<Real>), dim3(blocks_for(n, 256)), dim3(256), 0, st, pos, (int)n, c,
                       p.count.as<int>(), p.cell_of.as<int>(), p.wrapped.as<vec4_t<Real>>());
    HIP_TRY(s, hipGetLastError());
    hipLaunchKernelGGL(scan_blocks, dim3((unsigned)sblocks), dim3(kScanBlock), 0, st, p.count.as<int>(), (int)ncells,
                       p.start.as<int>(), p.scan_tmp.as<int>());
    HIP_TRY(s, hipGetLastError());
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(kScanBlock), 0, st, p.scan_tmp.as<int>(), (int)sblocks,
                       p.start.as<int>(), (int)ncells);
    HIP_TRY(s, hipGetLastError());
    hipLaunchKernelGGL(scan_add, dim3(blocks_for(ncells, 256)), dim3(256), 0, st, p.start.as<int>(), (int)ncells,
                       p.scan_tmp.as<int>());
    HIP_TRY(s, hipGetLastError());
    hipLaunchKernelGGL(pse_place, dim3(blocks_for(n, 256)), dim3(256), 0, st, (int)n, p.cell_of.as<int>(),
                       p.start.as<int>(), p.count.as<int>(), p.order.as<int>());
    HIP_TRY(s, hipGetLastError());
    hipLaunchKernelGGL(pse_sort_cells, dim3(blocks_for(ncells, 256)), dim3(256), 0, st, (int)ncells,
                       p.start.as<int>(), p.order.as<int>());
    HIP_TRY(s, hipGetLastError());
    hipLaunchKernelGGL((pse_gather<Real>), dim3(blocks_for(n, 256)), dim3(256), 0, st, (int)n, p.order.as<int>(),
                       p.wrapped.as<vec4_t<Real>>(), f, p.spos.as<vec4_t<Real>>(), p.sfrc.as<vec4_t<Real>>());
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

template <typename Real>
rpy_status ensure_grids(rpy_solver *s) {
    PseState &p = *s->pse;
    const size_t nr = (size_t)p.grid[0] * p.grid[1] * p.grid[2];
    const size_t nc = (size_t)p.grid[0] * p.grid[1] * (p.grid[2] / 2 + 1);
    HIP_TRY(s, p.rgrid.ensure(3 * nr * sizeof(Real)));
    HIP_TRY(s, p.cgrid.ensure(3 * nc * 2 * sizeof(Real)));
    return ensure_plans<Real>(s);
}

template <typename Real>
const vec2_t<Real> *table_of(const PseState &p) {
    if constexpr (std::is_same<Real, double>::value)
        return p.tab64.as<double2>();
    else
        return p.tab32.as<float2>();
}

}  // namespace

// The real-space part: the wavefront-per-tile kernel where at most kRealNbr
// tiles lie within rc, else the thread-per-target kernel.
template <typename Real, typename Tout, bool ADD>
hipError_t launch_real(const PseState &p, const PseConst<Real> &c, const PairConst<Real> &pc, int64_t n, Real kf,
                       Tout *out, hipStream_t st) {
    const int nnb = c.nbr_cnt[0] * c.nbr_cnt[1] * c.nbr_cnt[2];
    const int64_t ntiles = (int64_t)p.ncell[0] * p.ncell[1] * p.ncell[2];
    if (nnb <= kRealNbr)
        hipLaunchKernelGGL((pse_real_tiles<Real, Tout, ADD>), dim3(blocks_for(ntiles, 4)), dim3(256), 0, st,
                           (int)ntiles, p.spos.as<vec4_t<Real>>(), p.sfrc.as<vec4_t<Real>>(), p.order.as<int>(),
                           p.start.as<int>(), c, pc, table_of<Real>(p), kf, out);
    else
        hipLaunchKernelGGL((pse_real_threads<Real, Tout, ADD>), dim3(blocks_for(n, 256)), dim3(256), 0, st, (int)n,
                           p.spos.as<vec4_t<Real>>(), p.sfrc.as<vec4_t<Real>>(), p.order.as<int>(), p.start.as<int>(),
                           c, pc, table_of<Real>(p), kf, out);
    return hipGetLastError();
}

// M F for the periodic suspension with F staged in s->f (vec4), positions
// `pos_in` (vec4) or the stored ones; lin (n x 3, Tout) is overwritten.
// With real_only set, the real-space part alone.
template <typename Real, typename Tout>
rpy_status apply_pse(rpy_solver *s, const vec4_t<Real> *f, Tout *lin, hipStream_t st, const void *pos_in) {
    PseState &p = *s->pse;
    rpy_status r = configure(s);
    if (r != RPY_OK) return r;
    const int64_t n = s->n;
    const PseConst<Real> c = make_const<Real>(s);
    const auto *pos = pos_in ? static_cast<const vec4_t<Real> *>(pos_in) : s->pos.as<vec4_t<Real>>();
    r = build_cells<Real>(s, pos, f, c, st);
    if (r != RPY_OK) return r;
    const PairConst<Real> pc = make_pair_const<Real>(s->radius);
    const Real kf = Real(k_factor(s));
    if (p.real_only) {
        HIP_TRY(s, (launch_real<Real, Tout, false>(p, c, pc, n, kf, lin, st)));
        return RPY_OK;
    }
    r = ensure_grids<Real>(s);
    if (r != RPY_OK) return r;
    const int64_t nr = (int64_t)p.grid[0] * p.grid[1] * p.grid[2];
    const int nzh = p.grid[2] / 2 + 1;
    const int64_t nh = (int64_t)p.grid[0] * p.grid[1] * nzh;
    const int64_t ntiles = (int64_t)p.ncell[0] * p.ncell[1] * p.ncell[2];
    hipLaunchKernelGGL((pse_spread_tiles<Real>), dim3((unsigned)ntiles), dim3(256), 0, st, p.spos.as<vec4_t<Real>>(),
                       p.sfrc.as<vec4_t<Real>>(), p.start.as<int>(), c, p.rgrid.as<Real>());
    HIP_TRY(s, hipGetLastError());
    r = fft_forward<Real>(s, st);
    if (r != RPY_OK) return r;
    hipLaunchKernelGGL((pse_scale<Real>), dim3(blocks_for(nh, 256)), dim3(256), 0, st,
                       p.cgrid.as<typename FftTypes<Real>::complex_t>(), nh, nzh, c, Real(1.0 / (double)nr));
    HIP_TRY(s, hipGetLastError());
    r = fft_inverse<Real>(s, st);
    if (r != RPY_OK) return r;
    const Real vol = Real(p.h[0] * p.h[1] * p.h[2]);
    hipLaunchKernelGGL((pse_interp<Real, Tout, false>), dim3(blocks_for(n, 4)), dim3(256), 0, st, (int)n,
                       p.spos.as<vec4_t<Real>>(), p.order.as<int>(), c, p.rgrid.as<Real>(), vol, lin);
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, (launch_real<Real, Tout, true>(p, c, pc, n, kf, lin, st)));
    return RPY_OK;
}

template rpy_status apply_pse<float, float>(rpy_solver *, const float4 *, float *, hipStream_t, const void *);
template rpy_status apply_pse<float, double>(rpy_solver *, const float4 *, double *, hipStream_t, const void *);
template rpy_status apply_pse<double, double>(rpy_solver *, const double4 *, double *, hipStream_t, const void *);

// Wave-space fluctuations added to lin: prefactor sqrt(vol) J^T A^{1/2} z
// (see pse_noise) for the stored positions.
template <typename Real>
rpy_status pse_wave_noise(rpy_solver *s, const Real *noise, double prefactor, Real *lin, hipStream_t st) {
    PseState &p = *s->pse;
    rpy_status r = configure(s);
    if (r != RPY_OK) return r;
    r = ensure_grids<Real>(s);
    if (r != RPY_OK) return r;
    const int64_t n = s->n;
    const PseConst<Real> c = make_const<Real>(s);
    r = build_cells<Real>(s, s->pos.as<vec4_t<Real>>(), nullptr, c, st);
    if (r != RPY_OK) return r;
    const int64_t nr = (int64_t)p.grid[0] * p.grid[1] * p.grid[2];
    const int nzh = p.grid[2] / 2 + 1;
    const int64_t nh = (int64_t)p.grid[0] * p.grid[1] * nzh;
    hipLaunchKernelGGL((pse_noise<Real>), dim3(blocks_for(nh, 256)), dim3(256), 0, st,
                       p.cgrid.as<typename FftTypes<Real>::complex_t>(), nh, nzh, c, Real(1.0 / (double)nr), noise);
    HIP_TRY(s, hipGetLastError());
    r = fft_inverse<Real>(s, st);
    if (r != RPY_OK) return r;
    const Real scale = Real(prefactor * std::sqrt(p.h[0] * p.h[1] * p.h[2]));
    hipLaunchKernelGGL((pse_interp<Real, Real, true>), dim3(blocks_for(n, 4)), dim3(256), 0, st, (int)n,
                       p.spos.as<vec4_t<Real>>(), p.order.as<int>(), c, p.rgrid.as<Real>(), scale, lin);
    HIP_TRY(s, hipGetLastError());
    return RPY_OK;
}

rpy_status pse_create(rpy_solver *s) {
    s->pse = new (std::nothrow) PseState();
    return s->pse ? RPY_OK : RPY_ERR_OUT_OF_MEMORY;
}

void pse_release(rpy_solver *s) {
    if (!s->pse) return;
    PseState *p = s->pse;
    destroy_plans(p);
    for (DevBuf *b : {&p->tab32, &p->tab64, &p->count, &p->start, &p->scan_tmp, &p->cell_of, &p->order, &p->wrapped,
                      &p->spos, &p->sfrc, &p->rgrid, &p->cgrid})
        b->release();
    delete p;
    s->pse = nullptr;
}

rpy_status pse_set_parameter(rpy_solver *s, const char *key, double value) {
    PseState &p = *s->pse;
    if (!std::isfinite(value)) return fail(s, RPY_ERR_INVALID_ARG, std::string("'") + key + "' must be finite");
    if (!std::strcmp(key, "Lx") || !std::strcmp(key, "Ly") || !std::strcmp(key, "Lz") || !std::strcmp(key, "boxSize")) {
        if (!(value > 0.0)) return fail(s, RPY_ERR_INVALID_ARG, "box lengths must be positive");
        if (!std::strcmp(key, "boxSize"))
            p.box[0] = p.box[1] = p.box[2] = value;
        else
            p.box[key[1] - 'x'] = value;
    } else if (!std::strcmp(key, "psi")) {
        if (value < 0.0) return fail(s, RPY_ERR_INVALID_ARG, "psi must be >= 0 (0 = automatic)");
        p.psi = value;
    } else if (!std::strcmp(key, "tolerance")) {
        if (!(value >= 1e-14 && value <= 1e-2)) return fail(s, RPY_ERR_INVALID_ARG, "tolerance must be in [1e-14, 1e-2]");
        p.tol = value;
    } else {
        return fail(s, RPY_ERR_INVALID_ARG,
                    std::string("the periodic geometry takes Lx, Ly, Lz (or boxSize), psi and tolerance (got '") +
                        key + "')");
    }
    s->err.clear();
    return RPY_OK;
}

}  // namespace rpy

using namespace rpy;

extern "C" rpy_status rpy_pse_info(rpy_solver *s, int64_t grid_out[3], double info_out[5]) {
    if (!s) return RPY_ERR_INVALID_ARG;
    if (!s->pse) return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY, "rpy_pse_info needs the periodic geometry");
    if (!s->initialized) return fail(s, RPY_ERR_NOT_INITIALIZED, "rpy_initialize has not been called");
    rpy_status r = configure(s);
    if (r != RPY_OK) return r;
    const PseState &p = *s->pse;
    if (grid_out)
        for (int d = 0; d < 3; ++d) grid_out[d] = p.grid[d];
    if (info_out) {
        info_out[0] = p.xi;
        info_out[1] = p.rc;
        info_out[2] = p.sigma;
        info_out[3] = p.P;
        info_out[4] = p.qc;
    }
    return RPY_OK;
}

extern "C" rpy_status rpy_pse_sqrt_mdot_w(rpy_solver *s, const void *w, const void *wave_noise, double prefactor,
                                          double tol, int max_iter, void *lin_out, int *iters_out, double *incr_out,
                                          void *hip_stream) {
    rpy_status r = check_ready(s);
    if (r != RPY_OK) return r;
    if (!s->pse) return fail(s, RPY_ERR_UNSUPPORTED_GEOMETRY, "rpy_pse_sqrt_mdot_w needs the periodic geometry");
    if (!w || !wave_noise || !lin_out)
        return fail(s, RPY_ERR_INVALID_ARG, "W, the wave noise and the output must not be NULL");
    if (!(tol > 0.0 && tol < 1.0)) return fail(s, RPY_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(s, RPY_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!std::isfinite(prefactor)) return fail(s, RPY_ERR_INVALID_ARG, "prefactor must be finite");
    r = configure(s);
    if (r != RPY_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // real part by Lanczos on M_real; the flag is cleared on every path
    s->pse->real_only = true;
    if (s->dtype == RPY_F64)
        r = lanczos_run<double>(s, static_cast<const double *>(w), prefactor, tol, max_iter,
                                static_cast<double *>(lin_out), nullptr, iters_out, incr_out, st, false);
    else
        r = lanczos_run<float>(s, static_cast<const float *>(w), prefactor, tol, max_iter,
                               static_cast<float *>(lin_out), nullptr, iters_out, incr_out, st, false);
    s->pse->real_only = false;
    if (r != RPY_OK && r != RPY_ERR_NOT_CONVERGED) return r;
    const rpy_status lz = r;
    if (s->dtype == RPY_F64)
        r = pse_wave_noise<double>(s, static_cast<const double *>(wave_noise), prefactor,
                                   static_cast<double *>(lin_out), st);
    else
        r = pse_wave_noise<float>(s, static_cast<const float *>(wave_noise), prefactor, static_cast<float *>(lin_out),
                                  st);
    if (r != RPY_OK) return r;
    return lz;
}

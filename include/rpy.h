/*
 * rpy.h - C interface of the MI355X (gfx950) open-boundary RPY mobility library.
 *
 * The library applies the grand mobility matrix M(X) of a suspension of N
 * equal spheres in an unbounded Stokes fluid (the "NBody" open-boundary
 * solver of the libMobility paper, Sec. 3.5; blocks of eq. (block_mobility),
 * Rotne-Prager-Yamakawa pair tensors including the overlap branch), and
 * builds the terms of the overdamped Langevin equation (eq. (bdhi)) on it:
 * deterministic displacements M [F; T] (Mdot), fluctuations M^{1/2} W by
 * Lanczos (sqrtMdotW, Sec. 3.3) and the thermal drift (divM, Sec. 3.4).  The
 * call sequence follows the paper's solver interface (Sec. 3.2):
 * constructor with per-axis periodicity, setParameters, initialize,
 * setPositions, then Mdot / sqrtMdotW / divM.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Arrays are DEVICE pointers owned by the caller and only borrowed for the
 *   duration of the call (stream-ordered).  Per-particle arrays (positions,
 *   forces, torques, linear and angular outputs) are N x 3 row-major:
 *   element (i, k) at offset 3*i + k.  Noise and Lanczos vectors have 3N
 *   entries (translational only) or 6N entries (first the 3N linear, then
 *   the 3N angular, each particle-major).
 * - Every array of a call has the element type given to the most recent
 *   rpy_set_positions (RPY_F32 = float, RPY_F64 = double).  float inputs
 *   select the float32 pair evaluation (compensated cross-tile sums);
 *   double inputs select the float64 one.
 * - `hip_stream` is a hipStream_t (NULL = the null stream).  Work is
 *   enqueued on it and the call returns without waiting, except where a
 *   call says it synchronises.
 * - Every call returns an rpy_status; no exception crosses the interface.
 *   rpy_last_error() describes the most recent failure of that solver.
 *   HIP failures (including asynchronous faults surfacing at a
 *   synchronising call) return RPY_ERR_HIP.
 * - A solver handle must not be used from two host threads at once.
 */
#ifndef RPY_H
#define RPY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpy_solver rpy_solver;

typedef enum {
    RPY_OK = 0,
    RPY_ERR_INVALID_ARG = 1,          /* null pointer, N <= 0, eta <= 0, a <= 0, bad tol ... */
    RPY_ERR_UNSUPPORTED_GEOMETRY = 2, /* geometry not built, or call not built for it    */
    RPY_ERR_NOT_INITIALIZED = 3,      /* rpy_initialize not called yet                     */
    RPY_ERR_NO_POSITIONS = 4,         /* rpy_set_positions not called yet                  */
    RPY_ERR_SIZE_MISMATCH = 5,        /* batch sizes inconsistent                          */
    RPY_ERR_DTYPE_MISMATCH = 6,       /* dtype other than RPY_F32 / RPY_F64                */
    RPY_ERR_ANGULAR_DISABLED = 7,     /* torques / angular output without include_angular  */
    RPY_ERR_NONFINITE = 8,            /* NaN or Inf in positions or noise                  */
    RPY_ERR_NOT_CONVERGED = 9,        /* Lanczos reached max_iter (last iterate written)    */
    RPY_ERR_NOT_SPD = 10,             /* Lanczos met a clearly negative Ritz value          */
    RPY_ERR_OUT_OF_MEMORY = 11,
    RPY_ERR_HIP = 12
} rpy_status;

/* Per-axis boundary condition (constructor of Sec. 3.2). */
typedef enum { RPY_PERIODIC = 0, RPY_OPEN = 1, RPY_SINGLE_WALL = 2, RPY_TWO_WALLS = 3 } rpy_periodicity;

typedef enum { RPY_F32 = 0, RPY_F64 = 1 } rpy_dtype;

/*
 * Create a solver for the given periodicity of the x, y and z axes
 * (Sec. 3.2, constructor; Sec. 3.5: the N-body solver is open in x and y,
 * and open or single_wall in z).  (open, open, open) gives the free-space
 * RPY blocks; (open, open, single_wall) the Swan-Brady kernel: RPY blocks
 * for a no-slip plane at z = wallHeight (rpy_set_parameter), built from the
 * Stokeslet and Blake's image system with Faxen corrections, with the
 * damping that keeps M positive definite for particles overlapping the
 * wall (Sec. 3.5): heights h = z - wallHeight are raised to max(h, a) and
 * particle i's rows and columns are scaled by min(max(h_i / a, 0), 1).
 * (periodic, periodic, periodic) gives the triply periodic RPY mobility
 * (Sec. 3.5, "Positively Split Ewald (PSE)"; forces only): the lattice sum
 * over wave vectors k != 0 of sinc^2(k a) (I - khat khat^T) / (eta k^2)
 * e^{i k . r} / V, evaluated as a real-space sum of RPY - Wr over pairs
 * closer than a cutoff (minimum image) plus a wave-space part on an FFT
 * grid, split by Hasimoto's function with parameter psi (both parts
 * positive definite); see rpy_set_parameter for the box and accuracy.
 * Anything else returns RPY_ERR_UNSUPPORTED_GEOMETRY and writes NULL.  The
 * caller owns *out and frees it with rpy_destroy.  Does not touch the GPU.
 * Above a wall, rpy_mdot, rpy_mdot_multi, rpy_sqrt_mdot_w(_multi),
 * rpy_div_m_rfd, rpy_mobility_solve and the deterministic (kbt = 0) time
 * steps work; rpy_div_m, rpy_mdot_backward, rpy_mdot_noalloc and the
 * stochastic (kbt > 0) time steps return RPY_ERR_UNSUPPORTED_GEOMETRY.
 * In the periodic box, rpy_mdot, rpy_mdot_multi, rpy_sqrt_mdot_w(_multi)
 * (Lanczos on the whole periodic M), rpy_pse_sqrt_mdot_w (the split
 * fluctuations), rpy_div_m (zero: M depends on differences of positions
 * and its kernel is divergence-free), rpy_div_m_rfd, rpy_mobility_solve and
 * the time steps work; include_angular, rpy_mdot_backward, rpy_mdot_noalloc
 * and rpy_sqrt_mdot_w_precond return RPY_ERR_UNSUPPORTED_GEOMETRY.
 */
rpy_status rpy_create(rpy_periodicity x, rpy_periodicity y, rpy_periodicity z, rpy_solver **out);

/*
 * Domain-specific parameter by name (Sec. 3.2, setParameters).  The
 * single_wall geometry takes "wallHeight" (finite; default 0), the z of the
 * wall (particles live above it).  The periodic geometry takes the box
 * lengths "Lx", "Ly", "Lz" (> 0; "boxSize" sets all three; no default), the
 * splitting parameter "psi" (xi > 0 in 1/length; 0, the default, chooses
 * xi = (N/V)^{1/3}, raised until the cutoff fits the box) and "tolerance"
 * (in [1e-14, 1e-2], default 1e-4): the relative accuracy each part aims
 * at, which fixes the real-space cutoff rc (|RPY - Wr| < tolerance / (6 pi
 * eta a) beyond it, and the root-mean-square sum of the pairs it drops, at
 * the suspension's number density and unit random forces, below half of
 * that), the wave cutoff kc ((1 + q) e^{-q} = tolerance, q =
 * kc^2 / (4 xi^2)), the grid (Nyquist frequency 2 kc, sizes multiples of 8
 * with factors 2, 3, 5, 7), the Gaussian width (aliasing of kc below tolerance) and its
 * support (truncation below tolerance).  The first call that needs the
 * configuration returns RPY_ERR_INVALID_ARG if rc reaches half the box
 * (raise psi), the grid exceeds 4096 points per axis or the support 32.
 * Open boundaries have none.  Any other key or a non-finite value returns
 * RPY_ERR_INVALID_ARG.
 */
rpy_status rpy_set_parameter(rpy_solver *s, const char *key, double value);

/*
 * Configuration of a periodic solver (Sec. 3.5, PSE) for the current
 * parameters, computing it if needed (host quadrature of the real-space
 * table, uploaded to the device; synchronous): grid_out = (Nx, Ny, Nz) of
 * the Fourier grid, info_out = (xi, rc, sigma, support P, kc).  Needs
 * rpy_initialize (and, with automatic psi, the particle count of
 * rpy_set_positions).  RPY_ERR_UNSUPPORTED_GEOMETRY for other geometries.
 * Either output may be NULL.
 */
rpy_status rpy_pse_info(rpy_solver *s, int64_t grid_out[3], double info_out[5]);

/*
 * Fluctuations of the periodic solver by the positive split (Sec. 3.5, PSE:
 * the fluctuations are drawn in Fourier space):
 *   lin_out = prefactor (M_real^{1/2} w + y_wave),
 * M_real^{1/2} w by Lanczos on the real-space part alone (tol, max_iter and
 * the stopping test of rpy_sqrt_mdot_w; w has 3N entries), y_wave a sample
 * with covariance M_wave drawn from `wave_noise`: 3 x Nx x Ny x (Nz/2 + 1)
 * x 2 independent N(0, 1) numbers of the solver's dtype (component, the
 * half spectrum in FFT order, real and imaginary part), turned into unit
 * complex normals zeta_k = (re + i im) / sqrt(2) with zeta_{-k} =
 * conj(zeta_k): on the planes kz = 0 and kz = Nz/2, which hold both k and
 * -k, the entry whose (kx, ky) index pair is lexicographically after its
 * partner's (-kx mod Nx, -ky mod Ny) uses the conjugate of the partner's
 * numbers (a self-conjugate entry its real number alone); k = 0 and the
 * Nyquist entries are dropped.  Then y_wave,i = V^{-1/2} sum_k
 * sqrt(Khat_w(k)) (I - khat khat^T) zeta_k e^{i k . x_i} up to the grid
 * tolerance, Khat_w = sinc^2(k a) H(k, xi) / (eta k^2).  The covariance of
 * lin_out is prefactor^2 (M_real + M_wave) = prefactor^2 M.  Synchronises
 * hip_stream; iters_out / incr_out as for rpy_sqrt_mdot_w (may be NULL);
 * RPY_ERR_NOT_CONVERGED leaves the last iterate plus the wave part.
 */
rpy_status rpy_pse_sqrt_mdot_w(rpy_solver *s, const void *w, const void *wave_noise, double prefactor, double tol,
                               int max_iter, void *lin_out, int *iters_out, double *incr_out, void *hip_stream);

/*
 * Shared physical parameters (Sec. 3.2, initialize): fluid viscosity eta > 0
 * and hydrodynamic radius a > 0 (self mobility 1/(6 pi eta a)), and whether
 * torques / angular velocities are accepted (includeAngular, default off in
 * the paper because it is cheaper without).  May be called again to change
 * them; stored positions are kept.  Does not touch the GPU.
 */
rpy_status rpy_initialize(rpy_solver *s, double viscosity, double hydrodynamic_radius,
                          int include_angular);

/*
 * Store the current positions (Sec. 3.2, setPositions): `pos` is a device
 * array of n x 3 elements of `dtype`.  The values are copied into
 * solver-owned storage, so `pos` may be reused after the call.  Checks the
 * positions for NaN/Inf (RPY_ERR_NONFINITE; nothing is stored) and
 * therefore synchronises `hip_stream`.  Grows solver buffers as needed
 * (RPY_ERR_OUT_OF_MEMORY on failure).
 */
rpy_status rpy_set_positions(rpy_solver *s, const void *pos, int64_t n, rpy_dtype dtype,
                             void *hip_stream);

/*
 * Deterministic displacements (Sec. 3.2, Mdot; first term of eq. (bdhi)):
 * lin_out = M_uF F + M_uT T and, when ang_out != NULL, ang_out =
 * M_wF F + M_wT T, with M the grand mobility of eq. (block_mobility) at the
 * stored positions.  forces and torques are n x 3 (either may be NULL, not
 * both; a missing one counts as zero).  Torques or ang_out require
 * include_angular (RPY_ERR_ANGULAR_DISABLED).  Outputs are overwritten.
 * Asynchronous.
 */
rpy_status rpy_mdot(rpy_solver *s, const void *forces, const void *torques,
                    void *lin_out, void *ang_out, void *hip_stream);

/*
 * rpy_mdot without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks and result as rpy_mdot (to rounding:
 * it always runs the ordinary one-sided pair kernel, never the symmetric
 * mode, with the source splits of the solver's tiles lowered until its
 * partial sums fit).  The staged forces / torques and the partial sums live
 * in one fixed 64 MiB device array per GPU (taken on the first call made
 * with that device current and held until the process ends), so N is
 * limited: with S = 16 (float) or 32 (double) bytes per staged vector and P
 * = 3 or 6 components x 4 or 8 bytes (float32 pairs keep sums and
 * compensations: 2 x 4), N x (S x (1 or 2 vectors) + P) must not exceed
 * 64 MiB, else RPY_ERR_INVALID_ARG (nothing enqueued).  The solver's
 * positions are those stored by rpy_set_positions (which does allocate).
 * Every call on one GPU shares that array: calls that overlap in time on
 * one GPU (several streams or host threads) race on it.  Asynchronous.
 */
rpy_status rpy_mdot_noalloc(rpy_solver *s, const void *forces, const void *torques,
                            void *lin_out, void *ang_out, void *hip_stream);

/*
 * Several deterministic products with one geometry (an addition beside the
 * paper's method, which applies M to one vector per call; Sec. 3.3 notes
 * that a Krylov method may need several products at the same positions):
 * for r = 0 .. nrhs-1,
 *   lin_out[r] = M_uF F[r] + M_uT T[r],  ang_out[r] = M_wF F[r] + M_wT T[r].
 * forces, torques, lin_out and ang_out hold nrhs consecutive n x 3 arrays
 * (element (r, i, k) at offset 3*n*r + 3*i + k); either of forces / torques
 * may be NULL (zero), not both; torques or ang_out need include_angular.
 * 1 <= nrhs <= 1024 and nrhs * n < 2^31.  The pair geometry (separation,
 * 1/r, the tensor coefficients) is evaluated once per pair for up to four
 * vectors.  With the same tile configuration, translational results are
 * bit-identical to rpy_mdot of each vector; with the angular blocks the
 * pair is evaluated in a form that is cheaper per vector, and results agree
 * with rpy_mdot's to rounding.  Asynchronous.
 */
rpy_status rpy_mdot_multi(rpy_solver *s, const void *forces, const void *torques, int nrhs,
                          void *lin_out, void *ang_out, void *hip_stream);

/* Targets per lane of the multi-vector pair kernel: 1, 2, or 0 (default)
 * for the measured choice (1 for the float32 product with angular blocks,
 * 2 otherwise); results do not depend on it.  RPY_ERR_INVALID_ARG
 * otherwise. */
rpy_status rpy_set_multi_config(rpy_solver *s, int targets_per_lane);

/*
 * Fluctuating displacements (Sec. 3.2, sqrtMdotW; second term of eq.
 * (bdhi)) by the Lanczos iteration of Sec. 3.3:
 * y = prefactor * M^{1/2} w, converging to the symmetric square root.
 * `w` has 3N entries (6N with include_angular); the caller draws it (the
 * caller also supplies prefactor = sqrt(2 kT dt)).  Writes the linear part
 * of y to lin_out (n x 3) and, with include_angular, the angular part to
 * ang_out (n x 3, required then).  Iterates until the relative change of
 * successive iterates is below `tol` (0 < tol < 1) or `max_iter` (>= 1)
 * iterations.  The Krylov basis and tridiagonal matrix are kept in float64
 * on the device; the products with M use the solver's dtype.  Synchronises
 * `hip_stream`; *iters_out and *incr_out (may be NULL) receive the number
 * of iterations and the last relative increment.  Returns
 * RPY_ERR_NOT_CONVERGED (result still written) at max_iter,
 * RPY_ERR_NOT_SPD when M is found indefinite, RPY_ERR_NONFINITE for a
 * non-finite w.  A zero w gives zero output.
 */
rpy_status rpy_sqrt_mdot_w(rpy_solver *s, const void *w, double prefactor, double tol,
                           int max_iter, void *lin_out, void *ang_out, int *iters_out,
                           double *incr_out, void *hip_stream);

/*
 * Fluctuating displacements for several noise vectors with one geometry (an
 * addition beside the paper's method): y_r = prefactor * M^{1/2} w_r for
 * r = 0 .. nrhs-1 by nrhs Lanczos recurrences advanced together, each
 * iteration applying M to all unconverged recurrences in one multi-vector
 * product (rpy_mdot_multi).  w holds nrhs consecutive vectors of 3N (6N with
 * include_angular) entries; lin_out / ang_out hold nrhs consecutive n x 3
 * arrays.  Each recurrence runs rpy_sqrt_mdot_w's iteration and stopping
 * rule: without include_angular it reproduces rpy_sqrt_mdot_w of its vector
 * bit for bit (same tile configuration); with it the products agree to
 * rounding, and so do the results (the stopping iteration can differ only
 * where an increment lies within rounding of tol).  iters_out and incr_out (host, nrhs entries,
 * may be NULL) receive each recurrence's iteration count and last relative
 * increment.  1 <= nrhs <= 1024 and nrhs * n < 2^31; the float64 workspace
 * holds nrhs bases of min(max_iter, 1024) + 1 vectors.  Synchronises
 * hip_stream.  Returns RPY_ERR_NOT_SPD if any recurrence found M
 * indefinite, else RPY_ERR_NOT_CONVERGED if any reached max_iter (all
 * results written), RPY_ERR_NONFINITE for a non-finite w_r.
 */
rpy_status rpy_sqrt_mdot_w_multi(rpy_solver *s, const void *w, int nrhs, double prefactor, double tol,
                                 int max_iter, void *lin_out, void *ang_out, int *iters_out,
                                 double *incr_out, void *hip_stream);

/*
 * Preconditioned fluctuations (Sec. 3.3 notes that a preconditioner can
 * speed up the Lanczos iteration; an addition beside the paper's release):
 *   y = prefactor * L (L^{-1} M L^{-T})^{1/2} w,
 * with L block diagonal: particles form groups of group_size consecutive
 * particles (1 <= group_size <= 512; the last group may be shorter; e.g. one
 * polymer chain or rigid body per group), and for each group L holds the
 * Cholesky factor of M restricted to the group's linear rows and,
 * separately, to its angular rows.  y y^T has expectation M for w ~ N(0, I)
 * (eq. (fdt) holds, as for the symmetric root), but y is not M^{1/2} w.  The
 * Lanczos iteration, its stopping rule (on the iterate z of the
 * preconditioned operator), tol, max_iter, the outputs and the status codes
 * are those of rpy_sqrt_mdot_w.  The blocks are assembled in float64 from
 * the stored positions (open or single-wall geometry) and factored once per
 * positions and group size, then kept: about (6 G)^2 x N / G x 8 bytes
 * (half without angular blocks) of device memory.  RPY_ERR_NOT_SPD when a
 * block is not positive definite.  Synchronises hip_stream.
 */
rpy_status rpy_sqrt_mdot_w_precond(rpy_solver *s, const void *w, int64_t group_size, double prefactor,
                                   double tol, int max_iter, void *lin_out, void *ang_out, int *iters_out,
                                   double *incr_out, void *hip_stream);

/*
 * Mobility solve by conjugate gradients (an addition beside the paper's
 * method: a Krylov consumer of the product): for r = 0 .. nrhs-1 finds
 * [F_r; T_r] with M [F_r; T_r] = [U_r; Omega_r], the forces (and torques)
 * that give prescribed linear (and angular) velocities at the stored
 * positions.  u_lin / f_out (and, with include_angular, u_ang / t_out, both
 * required then) hold nrhs consecutive n x 3 arrays in the solver's dtype.
 * The iteration runs in float64 on the device, one multi-vector product per
 * iteration for the right-hand sides not yet converged; each stops at the
 * first iteration whose recursive residual |b - M x| / |b| is below tol
 * (0 < tol < 1; float32 products limit the attainable residual to about
 * 1e-6 times the condition number).  A zero right-hand side gives zero.
 * iters_out and resid_out (host, nrhs entries, may be NULL) receive the
 * iteration count and the final relative residual.  1 <= nrhs <= 1024,
 * nrhs * n < 2^31, max_iter >= 1.  Synchronises hip_stream.  Returns
 * RPY_ERR_NOT_CONVERGED (last iterates written) if any right-hand side
 * reached max_iter, RPY_ERR_NOT_SPD if a search direction with
 * p^T M p <= 0 appeared, RPY_ERR_NONFINITE for a non-finite right-hand side.
 */
rpy_status rpy_mobility_solve(rpy_solver *s, const void *u_lin, const void *u_ang, int nrhs, double tol,
                              int max_iter, void *f_out, void *t_out, int *iters_out, double *resid_out,
                              void *hip_stream);

/*
 * Thermal drift d_X . M (Sec. 3.2, divM; third term of eq. (bdhi)).  In an
 * unbounded fluid M is translation invariant and isotropic, so the
 * divergence vanishes (Sec. 2, Sec. 3.4): writes zeros to lin_out (n x 3)
 * and to ang_out when given (requires include_angular).  Above a wall the
 * drift does not vanish and needs a random vector: this call returns
 * RPY_ERR_UNSUPPORTED_GEOMETRY there, and rpy_div_m_rfd (eq. (rfd), the
 * paper's default for such solvers, Sec. 3.4) computes it.  Asynchronous.
 */
rpy_status rpy_div_m(rpy_solver *s, void *lin_out, void *ang_out, void *hip_stream);

/*
 * One random finite difference of the thermal drift (eq. (rfd), Sec. 3.4):
 *   [lin; ang] = (1/delta) [ M(X + delta/2 W_X) W - M(X - delta/2 W_X) W ]
 * w: device, 3N entries (6N with include_angular: linear first, as for
 * rpy_sqrt_mdot_w), in the dtype of the stored positions; W_X is its first
 * 3N entries, the only part that displaces the particles (orientation does
 * not enter M).  delta > 0 is an absolute length (the paper leaves its size
 * open; 1e-3 a in float32 and 1e-4 a in float64 balance the O(delta^2)
 * bias against rounding amplified by 1/delta).  The displaced positions are
 * formed in float64 without fused multiply-add and rounded once to the
 * stored precision; the stored positions are not changed.  The two products
 * are reduced in float64, differenced and rounded once.  lin_out (n x 3)
 * and, with include_angular, ang_out (n x 3) are required.  Averaged over
 * W ~ N(0, I) the sample tends to d_X . M + O(delta^2), zero in open space.
 * Asynchronous.  RPY_ERR_INVALID_ARG for delta <= 0 or not finite.
 */
rpy_status rpy_div_m_rfd(rpy_solver *s, const void *w, double delta, void *lin_out, void *ang_out,
                         void *hip_stream);

/*
 * Euler-Maruyama velocities of eq. (bdhi) (Sec. 3.2, LangevinVelocities):
 *   [lin; ang] = M [F; T] + sqrt(2 kbt / dt) M^{1/2} W + kbt d_X . M,
 * so that X + dt * lin is one Euler-Maruyama step.  In open space the drift
 * term is zero.  forces / torques as for rpy_mdot (either may be NULL,
 * meaning zero; torques need include_angular); w as for rpy_sqrt_mdot_w
 * (required when kbt > 0, ignored when kbt == 0); the noise term uses the
 * Lanczos solver with tol and max_iter and is added to the deterministic
 * part in float64 before one rounding to the solver's dtype.  dt > 0,
 * kbt >= 0.  lin_out (n x 3) and, with include_angular, ang_out (n x 3) are
 * required.  iters_out (host, may be NULL) receives the Lanczos iteration
 * count (0 when kbt == 0).  Synchronises hip_stream when kbt > 0.  Returns
 * RPY_ERR_NOT_CONVERGED (outputs written with the last Lanczos iterate) or
 * RPY_ERR_NOT_SPD as rpy_sqrt_mdot_w does.
 */
rpy_status rpy_langevin_velocities(rpy_solver *s, const void *forces, const void *torques, const void *w,
                                   double dt, double kbt, double tol, int max_iter, void *lin_out,
                                   void *ang_out, int *iters_out, void *hip_stream);

/*
 * One step of the stochastic Adams-Bashforth scheme used for eq. (bdhi) in
 * Sec. 5.1, from the stored positions X^n:
 *   pos_out = X^n + dt (3/2 u^n - 1/2 u^{n-1}) + sqrt(2 kbt dt) (M^n)^{1/2} W^n
 *   ang_out = dt (3/2 w^n - 1/2 w^{n-1}) + (angular rows of the noise)
 * with [u; w]^n = M^n [F^n; T^n] + kbt (d_X . M)^n (the drift is zero in
 * open space).  history (device, 3N entries, 6N with include_angular, linear
 * first, solver dtype) holds [u; w]^{n-1} on entry when have_history != 0
 * and receives [u; w]^n on exit; with have_history == 0 the step is the
 * Euler-Maruyama step (coefficients 1 and 0), which is how a run starts.
 * The stored positions are not changed: the caller computes the next forces
 * at pos_out and calls rpy_set_positions(pos_out) before the next step.
 * pos_out (n x 3) and, with include_angular, ang_out (n x 3; the rotation
 * increment of the step) are required; w, tol, max_iter, iters_out and the
 * return codes are as for rpy_langevin_velocities (on NOT_CONVERGED the step
 * is completed with the last Lanczos iterate).  Synchronises hip_stream when
 * kbt > 0.
 */
rpy_status rpy_ab2_step(rpy_solver *s, const void *forces, const void *torques, const void *w, double dt,
                        double kbt, double tol, int max_iter, void *history, int have_history, void *pos_out,
                        void *ang_out, int *iters_out, void *hip_stream);

/*
 * Adjoint of rpy_mdot at the stored positions (an addition beside the
 * paper's method): for cotangents g_U = grad_lin and g_W = grad_ang of a
 * scalar loss with respect to the Mdot outputs, writes
 *   grad_pos    = dL/dX (n x 3),
 *   grad_forces = M_uF^T g_U + M_wF^T g_W (= the linear rows of M [g_U; g_W]),
 *   grad_torques= M_uT^T g_U + M_wT^T g_W (angular rows),
 * each output optional (NULL skips it; at least one required).  forces /
 * torques are the inputs of the forward call (either may be NULL, not both);
 * grad_ang / torques / grad_torques require include_angular.  A pair of
 * coincident particles contributes nothing to grad_pos.  Asynchronous.
 */
rpy_status rpy_mdot_backward(rpy_solver *s, const void *forces, const void *torques,
                             const void *grad_lin, const void *grad_ang, void *grad_pos,
                             void *grad_forces, void *grad_torques, void *hip_stream);

/*
 * Pair evaluation of rpy_mdot_backward: 0 = automatic (the symmetric mode
 * from N = 4096 on, the one-sided kernel below), 1 = one-sided (every
 * ordered pair evaluated for its target), 2 = symmetric (each unordered
 * pair once, its position-gradient term added to one particle and
 * subtracted from the other).  The symmetric mode's partials ((N/256) x 9
 * x N source-side values of the solver's dtype, plus the target-side ones)
 * are produced and reduced in slabs of target blocks of at most about
 * 8 GiB of workspace each.  Results agree to rounding.
 * RPY_ERR_INVALID_ARG for other values.
 */
rpy_status rpy_set_adjoint_mode(rpy_solver *s, int mode);

/*
 * Batched solver: many independent open-boundary systems of uneven size
 * (an addition beside the paper's method).  System s owns particles
 * offsets[s] .. offsets[s+1]-1 of every concatenated per-particle array
 * (positions, forces, torques, linear and angular outputs: total x 3
 * row-major).  Noise / Lanczos vectors give system s the entries
 * m*offsets[s] .. m*offsets[s+1]-1, m = 3 (translational) or 6 (with
 * include_angular: the system's 3 n_s linear entries, then its 3 n_s
 * angular ones).  Systems never interact.  All systems share one dtype;
 * viscosity and radius are per system.
 */
typedef struct rpy_batch rpy_batch;

/*
 * offsets (host, n_systems + 1 entries, offsets[0] = 0, strictly
 * increasing), viscosity and radius (host, n_systems entries each, > 0),
 * include_angular (Sec. 3.2, includeAngular: torques in, angular
 * velocities out).  The arrays are copied.  Allocates the device task lists
 * and the block-mode partial sums (about (n_s / 512 + 1) x 3 x n_s values
 * per system, 6 with angular blocks, plus 6 (12) x 512 per block task in
 * float32); the caller owns *out and frees it with rpy_batch_destroy.
 */
rpy_status rpy_batch_create(int32_t n_systems, const int64_t *offsets, const double *viscosity,
                            const double *radius, int include_angular, rpy_dtype dtype, rpy_batch **out);

/* Store the positions of every system (device, total x 3); checks for
 * NaN/Inf and therefore synchronises hip_stream. */
rpy_status rpy_batch_set_positions(rpy_batch *b, const void *pos, void *hip_stream);

/*
 * lin_out = M_uF F + M_uT T and, with include_angular, ang_out = M_wF F +
 * M_wT T for every system (device, total x 3 each; ang_out required with
 * include_angular, forbidden without, like torques).  forces / torques:
 * either may be NULL (zero), not both.  In the block mode (default) one
 * launch evaluates every system's unordered particle pairs once (tasks of
 * one 512-particle target block against one source block of the same
 * system, the symmetric pair machinery of the single-system solver) and a
 * second one sums each particle's partials in a fixed order; the one-sided
 * mode (translational only) is one persistent launch over (system, target
 * tile) tasks.  Asynchronous.
 */
rpy_status rpy_batch_mdot(rpy_batch *b, const void *forces, const void *torques, void *lin_out, void *ang_out,
                          void *hip_stream);

/*
 * lin_out (and, with include_angular, ang_out) = prefactor * M_s^{1/2} w_s
 * for every system (device w of m x total entries in the layout above;
 * outputs total x 3) by Lanczos (Sec. 3.3) with the stopping rule of
 * rpy_sqrt_mdot_w applied to each system separately: each system stops at
 * the first k >= 2 meeting it, as if it were solved alone.  All systems
 * advance together; one iteration (the batched product for all active
 * systems, segmented float64 vector operations, the per-system stopping
 * test decided on the device) is one replay of a captured HIP graph.  The
 * host polls the number of systems still active every `check_every`
 * iterations (>= 1); a larger value saves host round trips at the price of
 * up to check_every - 1 idle replays at the end, and does not change any
 * result.  iters_out (host, n_systems entries, may be NULL) receives each
 * system's iteration count.  Synchronises hip_stream.  Returns
 * RPY_ERR_NOT_CONVERGED if any system reached max_iter (all results
 * written), RPY_ERR_NOT_SPD if any system's matrix was found indefinite.
 */
rpy_status rpy_batch_sqrt_mdot_w(rpy_batch *b, const void *w, double prefactor, double tol, int max_iter,
                                 int check_every, void *lin_out, void *ang_out, int *iters_out, void *hip_stream);

/*
 * Configuration of the batched product: targets_per_lane = 0 selects the
 * block mode (the default; the only one with include_angular); 1 or 2 the
 * one-sided persistent kernel, each task covering 64 x targets_per_lane
 * targets of one system, with workgroups_per_cu in [1, 32] workgroups per
 * CU in its persistent grid (default 8).  Setting it rebuilds the one-sided
 * task list (synchronous host-to-device copy).  RPY_ERR_INVALID_ARG
 * outside those ranges.
 */
rpy_status rpy_batch_set_tile_config(rpy_batch *b, int targets_per_lane, int workgroups_per_cu);
rpy_status rpy_batch_get_tile_config(const rpy_batch *b, int *targets_per_lane, int *workgroups_per_cu);

/*
 * Autotuner of the batched product for the current systems and positions:
 * times the block mode and every (targets per lane, workgroups per CU) in
 * {1, 2} x {4, 8, 16} of the one-sided kernel on a fixed pseudo-random
 * force vector, screens them with single products, re-times the best of
 * each mode and tile width in interleaved rounds of ~100 ms bursts, and
 * keeps the fastest.  With include_angular only the block mode exists and
 * nothing is timed.  Synchronises hip_stream.  RPY_ERR_NO_POSITIONS before
 * rpy_batch_set_positions.
 */
rpy_status rpy_batch_autotune(rpy_batch *b, void *hip_stream);

/* Message describing the last failure of `b`; owned by `b`. */
const char *rpy_batch_last_error(const rpy_batch *b);

/* Release the batch, its graphs and device buffers.  NULL is ignored. */
void rpy_batch_destroy(rpy_batch *b);

/*
 * Tile configuration of the pair kernel, separately for products without
 * (angular = 0) and with (angular = 1) the angular blocks:
 * targets_per_lane in {1, 2, 4}; source_splits = number of source ranges
 * the grid is split into (0 = chosen from N; clamped to ceil(N/256)).
 * targets_per_lane = 0 selects the symmetric pair mode instead: every
 * unordered pair is evaluated once and applied in both directions (blocks
 * of 512 particles, two targets per lane), source_splits then being the
 * number of 512-particle source blocks per task (0 = automatic: 1 up to
 * N = 65536, 2 above); its
 * partials ((N/512) x 6 x N source-side values plus the target-side ones)
 * are produced and reduced in slabs of target blocks of at most about
 * 8 GiB of workspace each (the environment variable RPY_SYM_SLAB_BLOCKS=m
 * also caps a slab at m blocks, for testing).  targets_per_lane = 3 selects
 * the fused small-N kernel: one launch per product that reads the caller's
 * N x 3 forces and torques directly and writes the outputs (workgroups of
 * 16 wavefronts per 4, 8 or 16 targets, each wavefront a sixteenth of the
 * sources; source_splits ignored); the autotuner tries it up to N = 8192.
 * Until a configuration is set or tuned, an open-boundary solver uses two
 * targets per lane below N = 32768 and the symmetric mode (automatic span)
 * from N = 32768 on; rpy_get_tile_config reports the configuration the
 * products use.  Results do not depend on the configuration beyond float
 * rounding order.
 */
rpy_status rpy_set_tile_config(rpy_solver *s, int angular, int targets_per_lane, int source_splits);
rpy_status rpy_get_tile_config(const rpy_solver *s, int angular, int *targets_per_lane, int *source_splits);

/*
 * Autotuner (an addition beside the paper's method): for the stored
 * positions' N and dtype, times every candidate (targets per lane x source
 * splits, and for 4096 <= N <= 2^18 the symmetric mode with 1 or 2 source
 * blocks per task, and up to N = 8192 the fused kernel) of the pair kernel
 * with HIP events on hip_stream, for the
 * translational product and, with include_angular, the angular one: a
 * screen of single products, then the fastest split of each targets-per-lane
 * value (each span of the symmetric mode separately) re-timed in
 * interleaved rounds of back-to-back bursts (about 100 ms each), whose
 * median rate under sustained load decides; the winner becomes the solver's tile
 * configuration (<ms> below is its time per product).  With cache_path
 * != NULL the choice is looked up in / added to a text file of lines
 *   <arch>|<f32|f64>|<lin|ang>|<round(log2 N)> <targets_per_lane> <splits> <ms>
 * (a cached entry is used without timing).  Above N = 2^18, where every
 * candidate costs a product of order N^2, nothing is timed: the symmetric
 * mode with its automatic span is chosen (the faster one in the measured
 * sweeps of N = 2^17 to 2^20).  Synchronises hip_stream.  A
 * single_wall solver is not timed: its tile configuration is reset to the
 * defaults of the wall kernel (two targets per lane, one with the angular
 * blocks; splits from N).
 */
rpy_status rpy_autotune(rpy_solver *s, const char *cache_path, void *hip_stream);

/* Kernel classes reported by rpy_kernel_time. */
typedef enum {
    RPY_KERNEL_PAIR = 0,
    RPY_KERNEL_ADJOINT = 1,
    RPY_KERNEL_LANCZOS_CGS = 2,
    RPY_KERNEL_PAIR_MULTI = 3
} rpy_kernel;

/*
 * Instrumentation, not part of the method: with `enable` != 0 the solver
 * records a HIP event pair, on the stream of the call, around every launch
 * of its pair kernel (forward products, including those inside sqrtMdotW),
 * of its adjoint kernel, of the multi-vector pair kernels (one record per
 * rpy_mdot_multi call), and around the two classical Gram-Schmidt passes of
 * every Lanczos iteration (four launches: two projections V^T w and two
 * updates w -= V h).  Enabling (or re-enabling) clears the records.
 */
rpy_status rpy_enable_timing(rpy_solver *s, int enable);

/*
 * Sum of the recorded durations of one kernel class in milliseconds, the
 * number of records and the work they did: ordered particle pairs for
 * RPY_KERNEL_PAIR and RPY_KERNEL_ADJOINT, pairs times vectors for
 * RPY_KERNEL_PAIR_MULTI; algorithmic HBM bytes for
 * RPY_KERNEL_LANCZOS_CGS (per pass at iteration k with basis vectors of n
 * doubles: (k + 1) n reads for V^T w, (k + 1) n reads and n writes for the
 * update, times 8 bytes; the second pass counts only where it ran: it is
 * skipped when the first removed at most half of |w|^2).  Waits for the
 * recorded events (host blocking).
 * Any output pointer may be NULL.
 */
rpy_status rpy_kernel_time(rpy_solver *s, rpy_kernel kernel, double *ms_total, int64_t *launches,
                           double *work);

/* Message describing the last failure of `s` ("" if none); owned by `s`. */
const char *rpy_last_error(const rpy_solver *s);

/* Release the solver and every device buffer it owns.  NULL is ignored. */
void rpy_destroy(rpy_solver *s);

#ifdef __cplusplus
}
#endif

#endif /* RPY_H */

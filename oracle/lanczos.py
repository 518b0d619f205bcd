"""Oracle: M^{1/2} W by Lanczos, and the exact symmetric root, in float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper computes the fluctuating term M^{1/2} W of eq. (bdhi) with the
Krylov (Lanczos) method of Ando, Chow, Saad & Skolnick (2012) whenever a
solver only applies M [Sec. 3.3]; it requires M symmetric positive definite
and gives no tolerance, stopping rule or reorthogonalisation.  The readings
taken here (listed with the design notes):

* start from v_1 = W / beta_0, beta_0 = |W|; W = 0 gives 0;
* three-term recurrence w = M v_k - beta_{k-1} v_{k-1}, alpha_k = v_k . w,
  w -= alpha_k v_k, then full re-orthogonalisation against every basis
  vector, done twice (classical Gram-Schmidt applied two times);
* T_k = tridiag(beta, alpha, beta) = Q diag(lambda) Q^T;  eigenvalues below
  -1e-10 lambda_max mean M is not positive definite; smaller negative ones
  are round-off and are clamped to 0;
* y_k = beta_0 V_k Q diag(lambda)^{1/2} Q^T e_1;
* stop at the first k >= 2 with |y_k - y_{k-1}| / |y_k| < tol;
* stop early (exact result) when beta_k <= 1e-14 max_i(|alpha_i|, beta_i);
* after ``maxit`` iterations return y_maxit flagged as not converged;
* the caller's prefactor (sqrt(2 kT dt) in eq. (bdhi)) multiplies y.

``exact_sqrt_mdot_w`` is the symmetric root Q Lambda^{1/2} Q^T W from a full
eigendecomposition of the assembled matrix (LAPACK through numpy).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class LanczosInfo:
    iters: int
    increment: float        # |y_k - y_{k-1}| / |y_k| at the last iteration
    converged: bool
    not_spd: bool = False
    breakdown: bool = False
    alphas: np.ndarray | None = None
    betas: np.ndarray | None = None


def tridiagonal_sqrt_e1(alphas, betas):
    """(s, lambda) with s = T^{1/2} e_1 for T = tridiag(betas, alphas, betas)."""
    k = len(alphas)
    t = np.diag(np.asarray(alphas, dtype=np.float64))
    if k > 1:
        off = np.asarray(betas[: k - 1], dtype=np.float64)
        t += np.diag(off, 1) + np.diag(off, -1)
    lam, q = np.linalg.eigh(t)
    return q @ (np.sqrt(np.clip(lam, 0.0, None)) * q[0, :]), lam


def lanczos_sqrt(matvec, w, tol: float = 1e-6, maxit: int = 500,
                 prefactor: float = 1.0, iters: int | None = None):
    """Lanczos approximation of prefactor * M^{1/2} w.

    ``matvec(v)`` applies M to a float64 vector.  With ``iters`` set, exactly
    that many iterations are run (no convergence test), which is how results
    are compared at a matched iteration count.
    """
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    beta0 = float(np.linalg.norm(w))
    if beta0 == 0.0:
        return np.zeros(n), LanczosInfo(0, 0.0, True)
    cap = iters if iters is not None else maxit
    basis = np.zeros((min(cap, n) + 1, n))
    basis[0] = w / beta0
    alphas, betas = [], []
    y_prev = None
    info = LanczosInfo(0, np.inf, False)
    y = np.zeros(n)
    for k in range(1, cap + 1):
        v = basis[k - 1]
        z = np.asarray(matvec(v), dtype=np.float64).copy()
        if k > 1:
            z -= betas[-1] * basis[k - 2]
        alpha = float(v @ z)
        z -= alpha * v
        vk = basis[:k]
        for _ in range(2):
            z -= vk.T @ (vk @ z)
        alphas.append(alpha)
        s, lam = tridiagonal_sqrt_e1(alphas, betas)
        info.iters = k
        if lam.min() < -1e-10 * max(lam.max(), 0.0):
            info.not_spd = True
            y = beta0 * (vk.T @ s)
            break
        y = beta0 * (vk.T @ s)
        if y_prev is not None:
            info.increment = float(np.linalg.norm(y - y_prev) / np.linalg.norm(y))
            if iters is None and info.increment < tol:
                info.converged = True
                break
        beta = float(np.linalg.norm(z))
        scale = max(max(abs(a) for a in alphas), max(betas) if betas else 0.0)
        if beta <= 1e-14 * scale or k == n:
            info.breakdown = True
            info.converged = True
            break
        if k == cap:
            break
        betas.append(beta)
        basis[k] = z / beta
        y_prev = y
    if iters is not None:
        info.converged = True
    info.alphas = np.array(alphas)
    info.betas = np.array(betas)
    return prefactor * y, info


def exact_sqrt_mdot_w(m, w, prefactor: float = 1.0):
    """prefactor * Q Lambda^{1/2} Q^T w for the symmetric matrix ``m``."""
    lam, q = np.linalg.eigh(m)
    return prefactor * (q @ (np.sqrt(np.clip(lam, 0.0, None)) * (q.T @ w)))


def exact_inv_sqrt(m):
    """M^{-1/2} through the eigendecomposition (the FDT test of Sec. 4)."""
    lam, q = np.linalg.eigh(m)
    return (q / np.sqrt(lam)) @ q.T


def group_cholesky(m, n_particles: int, group: int, angular: bool = False):
    """Block-diagonal lower-triangular L for the preconditioned Lanczos.

    Particles are split into groups of ``group`` consecutive particles (the
    last one may be shorter).  For each group, L holds the lower Cholesky
    factor of M restricted to the group's linear rows and columns (3 per
    particle, in the vector's order) and, with ``angular``, separately of its
    angular rows and columns; every other entry of L is zero.  Returns L as
    a dense (3N or 6N) square matrix.
    """
    dim = (6 if angular else 3) * n_particles
    L = np.zeros((dim, dim))
    for g0 in range(0, n_particles, group):
        p = np.arange(g0, min(n_particles, g0 + group))
        lin = (3 * p[:, None] + np.arange(3)).reshape(-1)
        for idx in ([lin, lin + 3 * n_particles] if angular else [lin]):
            L[np.ix_(idx, idx)] = np.linalg.cholesky(m[np.ix_(idx, idx)])
    return L


def preconditioned_lanczos_sqrt(matvec, L, w, tol: float = 1e-6, maxit: int = 500, prefactor: float = 1.0,
                                iters: int | None = None):
    """prefactor * L (L^{-1} M L^{-T})^{1/2} w, the square root of the
    preconditioned operator taken by ``lanczos_sqrt`` (same recurrence,
    re-orthogonalisation and stopping rule, applied to the iterate z of the
    preconditioned operator), then multiplied by L.

    With y = L z and z = (L^{-1} M L^{-T})^{1/2} w, y y^T has expectation
    L L^{-1} M L^{-T} L^T = M for w ~ N(0, I): a valid fluctuating term of
    eq. (bdhi) (Sec. 3.3 notes that a preconditioner can speed up Lanczos),
    though not the symmetric root M^{1/2} w.
    """
    from scipy.linalg import solve_triangular

    def op(v):
        t = solve_triangular(L, v, lower=True, trans="T")
        return solve_triangular(L, np.asarray(matvec(t), dtype=np.float64), lower=True)

    z, info = lanczos_sqrt(op, w, tol=tol, maxit=maxit, prefactor=1.0, iters=iters)
    return prefactor * (L @ z), info


def exact_preconditioned_sqrt(m, L, w, prefactor: float = 1.0):
    """prefactor * L (L^{-1} M L^{-T})^{1/2} w from an eigendecomposition."""
    from scipy.linalg import solve_triangular
    li = solve_triangular(L, np.eye(L.shape[0]), lower=True)
    return prefactor * (L @ exact_sqrt_mdot_w(li @ m @ li.T, w))

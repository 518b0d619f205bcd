"""Oracle: conjugate gradients on the mobility matrix, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A Krylov consumer of the product of Sec. 3.2 (Mdot): the forces (and
torques) x with M x = b for prescribed velocities b.  M is symmetric
positive definite, so the textbook conjugate-gradient recurrence applies:

    x_0 = 0, r_0 = p_0 = b
    alpha_k = (r_k . r_k) / (p_k . M p_k)
    x_{k+1} = x_k + alpha_k p_k,   r_{k+1} = r_k - alpha_k M p_k
    beta_k  = (r_{k+1} . r_{k+1}) / (r_k . r_k),   p_{k+1} = r_{k+1} + beta_k p_k

stopping at the first k with |r_k| / |b| < tol (the recursive residual).
``iters`` runs exactly that many iterations instead (matched comparisons).
Returns (x, iterations, relative recursive residual); a non-positive
p . M p raises ValueError (M not positive definite).
"""
from __future__ import annotations

import numpy as np


def conjugate_gradients(matvec, b, tol: float = 1e-8, maxit: int = 1000, iters: int | None = None):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bb = float(b @ b)
    if bb == 0.0:
        return x, 0, 0.0
    r = b.copy()
    p = r.copy()
    rr = bb
    cap = iters if iters is not None else maxit
    k = 0
    res = 1.0
    while k < cap:
        q = np.asarray(matvec(p), dtype=np.float64)
        pq = float(p @ q)
        if not pq > 0.0:
            raise ValueError("p . M p <= 0: the matrix is not positive definite")
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        k += 1
        res = (rr_new / bb) ** 0.5
        if iters is None and res < tol:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, k, res

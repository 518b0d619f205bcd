"""Oracle: adjoint of (U, Omega) = M(X) [F; T] in float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The adjoint is an addition beside the paper's method (the paper only applies
M).  For cotangents g_U = dL/dU and g_W = dL/dOmega:

* dL/dF, dL/dT: the grand mobility is symmetric, so [dF; dT] = M [g_U; g_W].
* dL/dX_k: U_i depends on X through the pair blocks M(X_i - X_j).  Writing
  each block as a function of r = X_i - X_j, with s_j = (F_j, T_j) and
  g_i = (g_U,i, g_W,i) and Phi(g, s; r) = g^T M(r) s,

      dL/dX_k = sum_{j != k} [ grad_r Phi(g_k, s_j; X_k - X_j)
                               - grad_r Phi(g_j, s_k; X_j - X_k) ].

  With the blocks written as  M_tt = A I + B r r^T,  M_rr = D I + E r r^T
  and coupling  F -> G F x r  (same block for T -> U), where A = c1,
  B = c2/r^2, D = d1, E = d2/r^2, G = f/r of ``oracle.mobility``:

      grad_r Phi = A' rhat (gU.F) + B' rhat (r.gU)(r.F) + B[(r.F) gU + (r.gU) F]
                 + G' rhat (gU.(T x r)) + G (gU x T)
                 + G' rhat (gW.(F x r)) + G (gW x F)
                 + D' rhat (gW.T) + E' rhat (r.gW)(r.T) + E[(r.T) gW + (r.gW) T].

  The blocks are C^1 but not C^2 at r = 2a and not differentiable at r = 0
  (coincident particles); a zero-distance pair contributes nothing.

This analytic form is pinned by complex-step differentiation of the dense
forward map in ``oracle.mobility`` (a different route to the same numbers).
"""
from __future__ import annotations

import math

import numpy as np

from .mobility import mdot_dense, mdot_rows, self_mobility


def _scalar_functions(r, a, eta):
    """(A, A', B, B', D, D', E, E', G, G') at distance r > 0 (real arrays)."""
    mu_t, mu_r = self_mobility(eta, a)
    near = r < 2.0 * a
    rf = np.where(near, 2.0 * a, r)
    rn = np.where(near, r, 2.0 * a)
    pe = math.pi * eta
    far = (
        mu_t * (3 * a / (4 * rf) + a ** 3 / (2 * rf ** 3)),
        mu_t * (-3 * a / (4 * rf ** 2) - 3 * a ** 3 / (2 * rf ** 4)),
        mu_t * (3 * a / (4 * rf ** 3) - 3 * a ** 3 / (2 * rf ** 5)),
        mu_t * (-9 * a / (4 * rf ** 4) + 15 * a ** 3 / (2 * rf ** 6)),
        -1.0 / (16 * pe * rf ** 3),
        3.0 / (16 * pe * rf ** 4),
        3.0 / (16 * pe * rf ** 5),
        -15.0 / (16 * pe * rf ** 6),
        1.0 / (8 * pe * rf ** 3),
        -3.0 / (8 * pe * rf ** 4),
    )
    near_v = (
        mu_t * (1 - 9 * rn / (32 * a)),
        np.full_like(rn, -9 * mu_t / (32 * a)),
        mu_t * 3 / (32 * a * rn),
        -3 * mu_t / (32 * a * rn ** 2),
        mu_r * (1 - 27 * rn / (32 * a) + 5 * rn ** 3 / (64 * a ** 3)),
        mu_r * (-27 / (32 * a) + 15 * rn ** 2 / (64 * a ** 3)),
        mu_r * (9 / (32 * a * rn) - 3 * rn / (64 * a ** 3)),
        mu_r * (-9 / (32 * a * rn ** 2) - 3 / (64 * a ** 3)),
        (1 / a - 3 * rn / (8 * a ** 2)) / (16 * pe * a ** 2),
        np.full_like(rn, -3.0 / (128 * pe * a ** 4)),
    )
    return tuple(np.where(near, n, f) for n, f in zip(near_v, far))


def _dot(u, v):
    return (u * v).sum(-1)


def _grad_phi(r, g_u, g_w, f, t, a, eta):
    """grad_r Phi(g, s; r) for stacked r[..., 3] (zero where r = 0)."""
    rn = np.sqrt(_dot(r, r))
    zero = rn == 0.0
    rs = np.where(zero, 1.0, rn)
    rhat = r / rs[..., None]
    A, Ap, B, Bp, D, Dp, E, Ep, G, Gp = _scalar_functions(np.where(zero, 1.0, rn), a, eta)
    ex = lambda s: s[..., None]
    rf_, rgu = _dot(r, f), _dot(r, g_u)
    out = (ex(Ap * _dot(g_u, f)) * rhat + ex(Bp * rgu * rf_) * rhat
           + ex(B) * (ex(rf_) * g_u + ex(rgu) * f))
    if t is not None:
        rt, rgw = _dot(r, t), _dot(r, g_w)
        out = out + ex(Gp * _dot(g_u, np.cross(t, r))) * rhat + ex(G) * np.cross(g_u, t)
        out = out + ex(Gp * _dot(g_w, np.cross(f, r))) * rhat + ex(G) * np.cross(g_w, f)
        out = out + ex(Dp * _dot(g_w, t)) * rhat + ex(Ep * rgw * rt) * rhat
        out = out + ex(E) * (ex(rt) * g_w + ex(rgw) * t)
    return np.where(zero[..., None], 0.0, out)


def grad_positions(x, forces, torques, g_u, g_w, a, eta, rows=None, chunk: int = 32):
    """dL/dX for the particles ``rows`` (default: all), shape (len(rows), 3)."""
    n = x.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    f = np.zeros((n, 3)) if forces is None else forces
    out = np.zeros((len(rows), 3))
    for s in range(0, len(rows), chunk):
        sel = rows[s:s + chunk]
        r = x[sel][:, None, :] - x[None, :, :]            # X_k - X_j
        gk_u = np.broadcast_to(g_u[sel][:, None, :], r.shape)
        fj = np.broadcast_to(f[None, :, :], r.shape)
        gj_u = np.broadcast_to(g_u[None, :, :], r.shape)
        fk = np.broadcast_to(f[sel][:, None, :], r.shape)
        if torques is None:
            t1 = _grad_phi(r, gk_u, None, fj, None, a, eta)
            t2 = _grad_phi(-r, gj_u, None, fk, None, a, eta)
        else:
            gk_w = np.broadcast_to(g_w[sel][:, None, :], r.shape)
            gj_w = np.broadcast_to(g_w[None, :, :], r.shape)
            tj = np.broadcast_to(torques[None, :, :], r.shape)
            tk = np.broadcast_to(torques[sel][:, None, :], r.shape)
            t1 = _grad_phi(r, gk_u, gk_w, fj, tj, a, eta)
            t2 = _grad_phi(-r, gj_u, gj_w, fk, tk, a, eta)
        out[s:s + chunk] = (t1 - t2).sum(axis=1)
    return out


def mdot_vjp(x, forces, torques, g_u, g_w, a, eta):
    """(dX, dF, dT) for cotangents (g_U, g_W); dT is None without torques."""
    dx = grad_positions(x, forces, torques, g_u, g_w, a, eta)
    if torques is None:
        df, _ = mdot_dense(x, g_u, None, a, eta)
        return dx, df, None
    df, dt = mdot_dense(x, g_u, g_w, a, eta)
    return dx, df, dt


def mdot_vjp_rows(x, forces, torques, g_u, g_w, a, eta, rows):
    """(dX, dF, dT) restricted to the particles ``rows``, for large N."""
    dx = grad_positions(x, forces, torques, g_u, g_w, a, eta, rows=rows)
    df, dt = mdot_rows(x, rows, g_u, g_w, a, eta)
    return dx, df, dt


def complex_step_grad(fun, x, coords, h: float = 1e-30):
    """d fun / d x.flat[c] for each c in ``coords`` by the complex step.

    ``fun`` must accept a complex array and be real-analytic in it; the
    derivative is Im fun(x + i h e_c) / h (Squire & Trapp 1998).
    """
    out = np.empty(len(coords))
    for k, c in enumerate(coords):
        xc = x.astype(np.complex128)
        xc.flat[c] += 1j * h
        out[k] = np.imag(fun(xc)) / h
    return out

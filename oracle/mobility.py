"""Oracle: the open-boundary Rotne-Prager-Yamakawa grand mobility, in float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``); shares no code with the
HIP path.

What the paper fixes
--------------------
* Eq. (block_mobility): the 6N x 6N grand mobility with blocks
  [[M_uF, M_uT], [M_wF, M_wT]] maps stacked forces and torques [F; T] to
  stacked linear and angular velocities [U; Omega].  Without torques only
  the 3N x 3N block M_uF is used.
* Eq. (stokestomob): each block pairs two particles through the Stokes
  Green's function averaged with the particles' regularising envelopes.
* Sec. 3.5 ("RPY kernels (NBody)"): for open boundaries these blocks are the
  free-space Rotne-Prager-Yamakawa tensors, summed brute-force over all
  pairs; the self block is the Stokes drag (6 pi eta a)^{-1} I of the
  SelfMobility paragraph.
* Eq. (kinetic_constraint): angular velocity is half the local vorticity,
  which fixes the sign of the translation-rotation coupling.

What the paper leaves to the literature (reading R1 of the design notes)
------------------------------------------------------------------------
The paper names the RPY tensors without printing them.  The coefficient
functions below are the standard equal-sphere generalised RPY tensors
(Rotne & Prager 1969, Yamakawa 1970 for r >= 2a; Wajnryb, Mizerski, Zuk &
Szymczak 2013 for overlapping spheres r < 2a and for the rotational
blocks).  With mu_t = 1/(6 pi eta a), mu_r = 1/(8 pi eta a^3) and
r_ij = X_i - X_j, r = |r_ij|, rhat = r_ij / r:

    U_i   = sum_j  M_tt(r_ij) F_j + f(r) T_j x rhat
    Omega_i = sum_j  f(r) F_j x rhat + M_rr(r_ij) T_j
    M_tt = c1 I + c2 rhat rhat^T ,   M_rr = d1 I + d2 rhat rhat^T

    r >= 2a:  c1 = mu_t (3a/(4r) + a^3/(2r^3))   c2 = mu_t (3a/(4r) - 3a^3/(2r^3))
              d1 = -1/(16 pi eta r^3)            d2 = 3/(16 pi eta r^3)
              f  = 1/(8 pi eta r^2)
    r <  2a:  c1 = mu_t (1 - 9r/(32a))           c2 = mu_t 3r/(32a)
              d1 = mu_r (1 - 27r/(32a) + 5r^3/(64a^3))
              d2 = mu_r (9r/(32a) - 3r^3/(64a^3))
              f  = (1/(16 pi eta a^2)) (r/a - 3r^2/(8a^2))

The self pair and coincident distinct particles take the r -> 0 limit of the
overlap branch: mu_t I, mu_r I and no coupling.  A tie at exactly r = 2a
goes to the far branch; the two branches agree there in value and slope.

Every function accepts complex positions so that complex-step
differentiation can be applied to it; branch decisions look at the real
part only.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "coefficients", "pair_blocks", "grand_mobility", "mdot_dense", "mdot_rows",
    "self_mobility",
]


def self_mobility(eta: float, a: float) -> tuple[float, float]:
    """(mu_t, mu_r): translational 1/(6 pi eta a) and rotational 1/(8 pi eta a^3)."""
    return 1.0 / (6.0 * math.pi * eta * a), 1.0 / (8.0 * math.pi * eta * a ** 3)


def coefficients(r, a: float, eta: float):
    """The five scalar functions (c1, c2, d1, d2, f) of the pair distance r.

    ``r`` may be any array (real or complex); the branch is chosen on
    ``r.real < 2a``.
    """
    r = np.asarray(r)
    mu_t, mu_r = self_mobility(eta, a)
    near = r.real < 2.0 * a
    # keep each branch finite where the other one is selected
    rf = np.where(near, 2.0 * a, r)
    rn = np.where(near, r, 0.0)
    c1_far = mu_t * (3.0 * a / (4.0 * rf) + a ** 3 / (2.0 * rf ** 3))
    c2_far = mu_t * (3.0 * a / (4.0 * rf) - 3.0 * a ** 3 / (2.0 * rf ** 3))
    d1_far = -1.0 / (16.0 * math.pi * eta * rf ** 3)
    d2_far = 3.0 / (16.0 * math.pi * eta * rf ** 3)
    f_far = 1.0 / (8.0 * math.pi * eta * rf ** 2)
    c1_near = mu_t * (1.0 - 9.0 * rn / (32.0 * a))
    c2_near = mu_t * 3.0 * rn / (32.0 * a)
    d1_near = mu_r * (1.0 - 27.0 * rn / (32.0 * a) + 5.0 * rn ** 3 / (64.0 * a ** 3))
    d2_near = mu_r * (9.0 * rn / (32.0 * a) - 3.0 * rn ** 3 / (64.0 * a ** 3))
    f_near = (rn / a - 3.0 * rn ** 2 / (8.0 * a ** 2)) / (16.0 * math.pi * eta * a ** 2)
    pick = lambda n, f: np.where(near, n, f)
    return (pick(c1_near, c1_far), pick(c2_near, c2_far), pick(d1_near, d1_far),
            pick(d2_near, d2_far), pick(f_near, f_far))


def _cross_matrix(v):
    """Matrix C(v) with C(v) @ u = u x v, for stacked vectors v[..., 3]."""
    z = np.zeros_like(v[..., 0])
    x, y, w = v[..., 0], v[..., 1], v[..., 2]
    # (u x v)_0 = u1 v2 - u2 v1, (u x v)_1 = u2 v0 - u0 v2, (u x v)_2 = u0 v1 - u1 v0
    return np.stack([np.stack([z, w, -y], -1),
                     np.stack([-w, z, x], -1),
                     np.stack([y, -x, z], -1)], -2)


def pair_blocks(xt, xs, a: float, eta: float, angular: bool = False):
    """3x3 blocks between targets ``xt`` (P,3) and sources ``xs`` (Q,3).

    Returns ``tt`` (P,Q,3,3) mapping F_j to U_i and, with ``angular``,
    ``rr`` (mapping T_j to Omega_i) and ``c`` (mapping F_j to Omega_i; the same
    block maps T_j to U_i).  A pair at zero distance gets the self limit.
    """
    d = xt[:, None, :] - xs[None, :, :]
    r = np.sqrt((d * d).sum(-1))
    zero = (r.real == 0.0) & (r.imag == 0.0)
    rhat = d / np.where(zero, 1.0, r)[..., None]
    rhat = np.where(zero[..., None], 0.0, rhat)
    c1, c2, d1, d2, f = coefficients(np.where(zero, 0.0, r), a, eta)
    eye = np.eye(3)
    outer = rhat[..., :, None] * rhat[..., None, :]
    tt = c1[..., None, None] * eye + c2[..., None, None] * outer
    if not angular:
        return tt
    rr = d1[..., None, None] * eye + d2[..., None, None] * outer
    c = f[..., None, None] * _cross_matrix(rhat)
    return tt, rr, c


def grand_mobility(x, a: float, eta: float, angular: bool = False):
    """Dense grand mobility: 3N x 3N, or 6N x 6N ordered [linear 3N; angular 3N].

    Row/column ``3*i + k`` is component k of particle i in each half.
    """
    n = x.shape[0]
    if not angular:
        tt = pair_blocks(x, x, a, eta)
        return tt.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
    tt, rr, c = pair_blocks(x, x, a, eta, angular=True)
    flat = lambda b: b.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
    cm = flat(c)
    return np.block([[flat(tt), cm], [cm, flat(rr)]])


def mdot_dense(x, forces=None, torques=None, a: float = 1.0, eta: float = 1.0 / (6 * math.pi)):
    """(U, Omega) = M(X) [F; T] through the assembled matrix.

    Forces default to zero when only torques are given; ``Omega`` is None
    when no torques are given.
    """
    n = x.shape[0]
    if forces is None and torques is None:
        raise ValueError("need forces or torques")
    f = np.zeros((n, 3), dtype=x.dtype) if forces is None else forces
    if torques is None:
        m = grand_mobility(x, a, eta)
        return (m @ f.reshape(-1)).reshape(n, 3), None
    m = grand_mobility(x, a, eta, angular=True)
    v = m @ np.concatenate([f.reshape(-1), torques.reshape(-1)])
    return v[: 3 * n].reshape(n, 3), v[3 * n:].reshape(n, 3)


def mdot_rows(x, rows, forces=None, torques=None, a: float = 1.0,
              eta: float = 1.0 / (6 * math.pi), chunk: int = 16):
    """Block rows of M [F; T] for the target particles ``rows`` only.

    Assembles the blocks of a few target rows at a time against every
    source, multiplies, and discards them.
    """
    rows = np.asarray(rows)
    n = x.shape[0]
    f = np.zeros((n, 3)) if forces is None else forces
    u = np.zeros((len(rows), 3), dtype=np.result_type(x, f))
    w = None if torques is None else np.zeros_like(u)
    for s in range(0, len(rows), chunk):
        sel = rows[s:s + chunk]
        if torques is None:
            tt = pair_blocks(x[sel], x, a, eta)
            u[s:s + chunk] = np.einsum("pqab,qb->pa", tt, f)
        else:
            tt, rr, c = pair_blocks(x[sel], x, a, eta, angular=True)
            u[s:s + chunk] = np.einsum("pqab,qb->pa", tt, f) + np.einsum("pqab,qb->pa", c, torques)
            w[s:s + chunk] = np.einsum("pqab,qb->pa", c, f) + np.einsum("pqab,qb->pa", rr, torques)
    return u, w

"""Oracle: the wall-corrected RPY mobility above one no-slip wall, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``); shares no code with the
HIP path.

What the paper fixes (Sec. 3.5, "RPY kernels (NBody)"; Sec. 3.2)
----------------------------------------------------------------
* The N-body solver accepts ``single_wall`` along z (x and y open) and then
  uses the Swan-Brady kernel: the RPY mobility corrected for a planar
  no-slip wall.  ``setParameters(wallHeight=...)`` places the wall.
* That kernel is not positive definite when particles overlap the wall; the
  solver applies the damping-matrix approach of the rollers paper it cites
  (its Appendix A), under which a particle's mobility goes smoothly to zero
  as it approaches the wall while M stays symmetric positive definite.

Readings (the paper names the kernels without printing them)
------------------------------------------------------------
* The kernel of Swan & Brady (Phys. Fluids 19, 113306, 2007) is the RPY
  construction applied to Blake's Green's function for a Stokeslet above a
  no-slip plane (Blake, Proc. Camb. Phil. Soc. 70, 303, 1971): with G the
  Stokeslet plus Blake's image system, x the receiving and y the source
  particle centre, and 1/(8 pi eta) in front of every block,
      M_tt = (1 + a^2/6 Lap_x)(1 + a^2/6 Lap_y) G(x, y)
      M_rt = 1/2 curl_x (1 + a^2/6 Lap_y) G(x, y)        (force -> rotation)
      M_tr = 1/2 (1 + a^2/6 Lap_x) curl_y G(x, y)        (torque -> velocity)
      M_rr = 1/4 curl_x curl_y G(x, y)
  i.e. Faxen's laws on each side (translation: the sphere-surface average,
  exact here because every term of G is biharmonic; rotation: half the
  vorticity).  The free-space Stokeslet part gives the open-boundary RPY
  blocks of ``oracle.mobility`` (including its overlap branch r < 2a and the
  self block); only the image part is added here, for every pair and for
  the self pair (x = y).
* Damping (the cited Appendix A, as read here): with h_i = z_i - wallHeight,
  every height is replaced by max(h_i, a) and the whole 6N x 6N matrix is
  multiplied on both sides by D = diag(d_i), d_i = min(max(h_i / a, 0), 1),
  applied to a particle's linear and angular rows alike.  D M D is
  congruent to an SPD matrix, so it stays SPD while every d_i > 0, and a
  particle's row and column vanish as it reaches the wall.

The image blocks are obtained here by symbolic differentiation (sympy) of
Blake's image system as written below, lambdified to numpy; the pins in the
tests compare them with surface quadratures of ``blake_image`` and with the
classical near-wall series of a single sphere.
"""
from __future__ import annotations

import math

import numpy as np

from .mobility import grand_mobility, mdot_rows

__all__ = ["blake_image", "image_blocks", "effective_heights", "grand_mobility_wall", "mdot_wall",
           "mdot_wall_rows"]


def blake_image(x, y):
    """Image part of Blake's tensor: G(x, y) = S(x - y) + blake_image(x, y),
    S the Stokeslet (I/r + r r^T / r^3), wall at z = 0, source y above it.

    With the image point y* = (y1, y2, -y3), R = x - y*, h = y3 and
    P = diag(1, 1, -1):
        G^im_ij = -S_ij(R) + 2 h P_jj d/dR_j [ h R_i / |R|^3 - (delta_i3 / |R| + R_i R_3 / |R|^3) ].
    ``x`` (..., 3) and ``y`` (..., 3) broadcast; returns (..., 3, 3),
    index [i, j] = velocity component i for force component j (without
    the 1/(8 pi eta)).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x, y = np.broadcast_arrays(x, y)
    h = y[..., 2]
    R = x - y * np.array([1.0, 1.0, -1.0])
    rn = np.sqrt((R * R).sum(-1))
    r1, r3, r5 = 1.0 / rn, 1.0 / rn ** 3, 1.0 / rn ** 5
    eye = np.eye(3)
    RR = R[..., :, None] * R[..., None, :]
    S = eye * r1[..., None, None] + RR * r3[..., None, None]
    # dphi[..., i, k] = d/dR_k of phi_i = h R_i/R^3 - delta_i3/R - R_i R_3/R^3
    R3 = R[..., 2]
    e3 = np.array([0.0, 0.0, 1.0])
    dphi = (h[..., None, None] * (eye * r3[..., None, None] - 3.0 * RR * r5[..., None, None])
            + e3[:, None] * (R * r3[..., None])[..., None, :]
            - (eye * R3[..., None, None] + R[..., :, None] * e3[None, :]) * r3[..., None, None]
            + 3.0 * RR * (R3 * r5)[..., None, None])
    P = np.array([1.0, 1.0, -1.0])
    return -S + 2.0 * h[..., None, None] * dphi * P


_FUNCS = None


def _image_functions():
    """Lambdified (tt, rt, tr, rr) image blocks as functions of
    (R1, R2, R3, h_source, a), R = x - y* (built once per process)."""
    global _FUNCS
    if _FUNCS is not None:
        return _FUNCS
    import sympy as sp
    R1, R2, R3, hh, a = sp.symbols("R1 R2 R3 hh a", real=True)
    Rv = [R1, R2, R3]
    rn = sp.sqrt(R1 ** 2 + R2 ** 2 + R3 ** 2)
    P = [1, 1, -1]
    G = sp.zeros(3, 3)
    for i in range(3):
        phi = hh * Rv[i] / rn ** 3 - ((1 if i == 2 else 0) / rn + Rv[i] * Rv[2] / rn ** 3)
        for j in range(3):
            G[i, j] = -((1 if i == j else 0) / rn + Rv[i] * Rv[j] / rn ** 3) + 2 * hh * P[j] * sp.diff(phi, Rv[j])
    # x enters only through R; y through R (R_1,2 = x_1,2 - y_1,2, R_3 = x_3 + y_3) and hh = y_3
    dx = lambda f, m: sp.diff(f, Rv[m])
    dy = lambda f, m: -sp.diff(f, Rv[m]) if m < 2 else sp.diff(f, R3) + sp.diff(f, hh)
    lap_x = lambda f: sum(dx(dx(f, m), m) for m in range(3))
    lap_y = lambda f: sum(dy(dy(f, m), m) for m in range(3))
    eps = sp.LeviCivita
    gy = G.applyfunc(lambda g: g + a ** 2 / 6 * lap_y(g))   # Faxen on the source (force) side
    gx = G.applyfunc(lambda g: g + a ** 2 / 6 * lap_x(g))   # Faxen on the receiving side
    tt = gy.applyfunc(lambda g: g + a ** 2 / 6 * lap_x(g))
    rt = sp.Matrix(3, 3, lambda k, l: sp.Rational(1, 2) * sum(
        eps(k, m, n) * dx(gy[n, l], m) for m in range(3) for n in range(3) if eps(k, m, n) != 0))
    tr = sp.Matrix(3, 3, lambda k, l: sp.Rational(1, 2) * sum(
        eps(l, m, n) * dy(gx[k, n], m) for m in range(3) for n in range(3) if eps(l, m, n) != 0))
    rr = sp.Matrix(3, 3, lambda k, p: sp.Rational(1, 4) * sum(
        eps(k, m, n) * eps(p, q, s) * dx(dy(G[n, s], q), m)
        for m in range(3) for n in range(3) for q in range(3) for s in range(3)
        if eps(k, m, n) != 0 and eps(p, q, s) != 0))
    args = (R1, R2, R3, hh, a)
    _FUNCS = tuple(sp.lambdify(args, [[blk[i, j] for j in range(3)] for i in range(3)], "numpy", cse=True)
                   for blk in (tt, rt, tr, rr))
    return _FUNCS


def _stack(mat, shape):
    """Nested 3x3 lists of arrays/scalars from a lambdified matrix -> (..., 3, 3)."""
    return np.stack([np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), shape)
                               for v in row], -1) for row in mat], -2)


def image_blocks(xt, xs, a: float, eta: float, angular: bool = False):
    """Image-part blocks between targets ``xt`` (P, 3) and sources ``xs``
    (Q, 3), positions with z = height above the wall (z > 0).

    Returns tt (P, Q, 3, 3) (force_j -> velocity_i) and, with ``angular``,
    also rt (force_j -> rotation_i), tr (torque_j -> velocity_i) and rr
    (torque_j -> rotation_i), each including 1/(8 pi eta).
    """
    xt = np.asarray(xt, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    R1 = xt[:, None, 0] - xs[None, :, 0]
    R2 = xt[:, None, 1] - xs[None, :, 1]
    R3 = xt[:, None, 2] + xs[None, :, 2]
    hh = np.broadcast_to(xs[None, :, 2], R1.shape)
    f_tt, f_rt, f_tr, f_rr = _image_functions()
    k = 1.0 / (8.0 * math.pi * eta)
    shape = R1.shape
    tt = k * _stack(f_tt(R1, R2, R3, hh, a), shape)
    if not angular:
        return tt
    return (tt, k * _stack(f_rt(R1, R2, R3, hh, a), shape), k * _stack(f_tr(R1, R2, R3, hh, a), shape),
            k * _stack(f_rr(R1, R2, R3, hh, a), shape))


def effective_heights(x, a: float, wall_height: float = 0.0):
    """(positions with z replaced by the height max(z - wall, a) above the
    wall, damping factors d = min(max((z - wall)/a, 0), 1))."""
    x = np.asarray(x, dtype=np.float64)
    h = x[:, 2] - wall_height
    xe = x.copy()
    xe[:, 2] = np.maximum(h, a)
    d = np.clip(h / a, 0.0, 1.0)
    return xe, d


def grand_mobility_wall(x, a: float, eta: float, angular: bool = False, wall_height: float = 0.0,
                        damping: bool = True):
    """Dense 3N x 3N (or 6N x 6N, [linear; angular]) mobility above the wall.

    ``damping=False`` evaluates the undamped kernel at the actual heights
    (used to show that it is not positive definite for wall overlaps)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if damping:
        xe, d = effective_heights(x, a, wall_height)
    else:
        xe = x.copy()
        xe[:, 2] -= wall_height
        d = np.ones(n)
    m = grand_mobility(xe, a, eta, angular)
    flat = lambda b: b.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
    if angular:
        tt, rt, tr, rr = image_blocks(xe, xe, a, eta, True)
        m = m + np.block([[flat(tt), flat(tr)], [flat(rt), flat(rr)]])
        dd = np.concatenate([np.repeat(d, 3), np.repeat(d, 3)])
    else:
        m = m + flat(image_blocks(xe, xe, a, eta))
        dd = np.repeat(d, 3)
    return dd[:, None] * m * dd[None, :]


def mdot_wall(x, forces=None, torques=None, a: float = 1.0, eta: float = 1.0 / (6 * math.pi),
              wall_height: float = 0.0):
    """(U, Omega or None) = M_wall [F; T] through the assembled matrix."""
    n = x.shape[0]
    f = np.zeros((n, 3)) if forces is None else np.asarray(forces, dtype=np.float64)
    if torques is None:
        m = grand_mobility_wall(x, a, eta, False, wall_height)
        return (m @ f.reshape(-1)).reshape(n, 3), None
    m = grand_mobility_wall(x, a, eta, True, wall_height)
    v = m @ np.concatenate([f.reshape(-1), np.asarray(torques, dtype=np.float64).reshape(-1)])
    return v[:3 * n].reshape(n, 3), v[3 * n:].reshape(n, 3)


def mdot_wall_rows(x, rows, forces=None, torques=None, a: float = 1.0, eta: float = 1.0 / (6 * math.pi),
                   wall_height: float = 0.0, chunk: int = 8):
    """Block rows of M_wall [F; T] for the particles ``rows`` (large N)."""
    x = np.asarray(x, dtype=np.float64)
    rows = np.asarray(rows)
    n = x.shape[0]
    xe, d = effective_heights(x, a, wall_height)
    f = np.zeros((n, 3)) if forces is None else np.asarray(forces, dtype=np.float64)
    fd = f * d[:, None]
    td = None if torques is None else np.asarray(torques, dtype=np.float64) * d[:, None]
    u, w = mdot_rows(xe, rows, fd, td, a, eta)
    for s in range(0, len(rows), chunk):
        sel = rows[s:s + chunk]
        if td is None:
            tt = image_blocks(xe[sel], xe, a, eta)
            u[s:s + chunk] += np.einsum("pqab,qb->pa", tt, fd)
        else:
            tt, rt, tr, rr = image_blocks(xe[sel], xe, a, eta, True)
            u[s:s + chunk] += np.einsum("pqab,qb->pa", tt, fd) + np.einsum("pqab,qb->pa", tr, td)
            w[s:s + chunk] += np.einsum("pqab,qb->pa", rt, fd) + np.einsum("pqab,qb->pa", rr, td)
    u *= d[rows][:, None]
    if w is not None:
        w *= d[rows][:, None]
    return u, w

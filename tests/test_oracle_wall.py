"""Pins of the wall-corrected oracle (oracle/wall.py) against what the
mathematics and the classical single-sphere results fix (CPU only).

* Blake's image system: zero velocity on the wall, incompressible, and
  reciprocal (G(x, y) = G(y, x)^T) - together with the free Stokeslet's
  singularity and decay these determine it.
* The image blocks against direct surface quadratures of Blake's tensor over
  both spheres (translation: surface average; rotation: 3/(2a) times the
  surface average of n x u; a torque as the surface force density
  3/(8 pi a^3) L x m), which is what the operator definitions equal for
  Stokes flows.
* One sphere near the wall: Faxen's series for translation parallel to the
  wall, Lorentz's and Brenner's for translation normal to it, and Goldman,
  Cox & Brenner's leading terms for rotation and for the
  translation-rotation coupling (sign: a sphere pushed along the wall turns
  as if rolling on it).
* Far from the wall the open-boundary mobility is recovered; the matrix is
  symmetric and, with damping, positive definite (also for particles
  overlapping the wall, where the undamped kernel is not); the damping is
  continuous at h = a and takes a particle's rows to zero at the wall.
* Thermal drift of one sphere: the finite-difference divergence equals the
  derivative of the normal self mobility.
"""
import math

import numpy as np
import pytest

from oracle import drift, mobility, wall

ETA = 1.0 / (6.0 * math.pi)
A = 1.0


def _stokeslet(d):
    r = np.sqrt((d * d).sum(-1))
    return np.eye(3) / r[..., None, None] + d[..., :, None] * d[..., None, :] / r[..., None, None] ** 3


def test_blake_no_slip_on_the_wall():
    rng = np.random.default_rng(11)
    y = np.column_stack([rng.normal(size=(20, 2)), 0.2 + 3 * rng.random(20)])
    x = np.column_stack([y[:, :2] + rng.normal(size=(20, 2)) * 2, np.zeros(20)])
    g = _stokeslet(x - y) + wall.blake_image(x, y)
    assert np.abs(g).max() <= 1e-14 * np.abs(_stokeslet(x - y)).max()


def test_blake_incompressible_and_reciprocal():
    rng = np.random.default_rng(12)
    y = np.array([0.4, -0.3, 1.3])
    full = lambda x, yy: _stokeslet(x - yy) + wall.blake_image(x, yy)
    for _ in range(5):
        x = np.array([*rng.normal(size=2), 0.5 + 2 * rng.random()])
        h = 1e-5
        div = sum((full(x + h * e, y)[k] - full(x - h * e, y)[k]) / (2 * h) for k, e in enumerate(np.eye(3)))
        assert np.abs(div).max() <= 1e-8 * np.abs(full(x, y)).max()
        assert np.abs(full(x, y) - full(y, x).T).max() <= 1e-14 * np.abs(full(x, y)).max()


def _sphere_nodes(nt, nph):
    mu, w = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    st = np.sqrt(1 - mu ** 2)
    n = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)), np.outer(mu, np.ones(nph))], -1).reshape(-1, 3)
    wt = np.outer(w, np.ones(nph)).reshape(-1) / (2 * nph)      # weights of the surface average (sum 1)
    return n, wt


def _quadrature_blocks(xi, xj, a, nt=24, nph=48):
    """Surface-quadrature image blocks (without 1/(8 pi eta))."""
    n, wt = _sphere_nodes(nt, nph)
    eps = np.zeros((3, 3, 3))
    for i, j, k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        eps[i, j, k], eps[i, k, j] = 1.0, -1.0
    tt = np.zeros((3, 3))
    rt = np.zeros((3, 3))
    tr = np.zeros((3, 3))
    rr = np.zeros((3, 3))
    c = 3.0 / (2.0 * a)
    for p in range(len(n)):     # receiving node
        g = wall.blake_image((xi + a * n[p])[None, :], xj + a * n)     # (Q, 3, 3), source nodes
        gm = np.einsum("q,qab->ab", wt, g)                             # source-averaged
        gl = c * np.einsum("q,qau,urs,qs->ar", wt, g, eps, n)          # torque source: G (L x m)
        tt += wt[p] * gm
        rt += wt[p] * c * np.einsum("kpq,p,ql->kl", eps, n[p], gm)
        tr += wt[p] * gl
        rr += wt[p] * c * np.einsum("kpq,p,qr->kr", eps, n[p], gl)
    return tt, rt, tr, rr


@pytest.mark.parametrize("xi,xj", [
    ((0.0, 0.0, 2.5), (0.0, 0.0, 2.5)),          # self pair
    ((0.3, -0.4, 2.2), (3.1, 1.0, 4.0)),
    ((1.0, 0.5, 6.0), (-1.5, 0.2, 2.4)),
    ((0.0, 0.0, 2.1), (0.2, 0.1, 4.4)),          # nearly above each other
])
def test_image_blocks_match_surface_quadrature(xi, xj):
    xi, xj = np.array(xi), np.array(xj)
    k = 8 * math.pi * ETA
    tt, rt, tr, rr = (b[0, 0] * k for b in wall.image_blocks(xi[None], xj[None], A, ETA, angular=True))
    qt, qrt, qtr, qrr = _quadrature_blocks(xi, xj, A)
    scale = np.abs(qt).max()
    for got, ref in ((tt, qt), (rt, qrt), (tr, qtr), (rr, qrr)):
        assert np.abs(got - ref).max() <= 1e-10 * scale


@pytest.mark.parametrize("xi_", [0.1, 0.05, 0.02])
def test_one_sphere_near_the_wall_classical_series(xi_):
    h = A / xi_
    m = wall.grand_mobility_wall(np.array([[0.3, -0.7, h]]), A, ETA, angular=True)
    mu_t, mu_r = mobility.self_mobility(ETA, A)
    # translation parallel (Faxen) and normal (Lorentz; Brenner) to the wall, through xi^3
    assert abs(m[0, 0] / mu_t - (1 - 9 / 16 * xi_ + xi_ ** 3 / 8)) <= 0.2 * xi_ ** 4
    assert abs(m[1, 1] - m[0, 0]) <= 1e-15
    assert abs(m[2, 2] / mu_t - (1 - 9 / 8 * xi_ + xi_ ** 3 / 2)) <= 0.6 * xi_ ** 4
    # rotation about an axis parallel / normal to the wall (Goldman, Cox & Brenner), leading term
    assert abs(m[3, 3] / mu_r - (1 - 5 / 16 * xi_ ** 3)) <= 0.1 * xi_ ** 4
    assert abs(m[5, 5] / mu_r - (1 - xi_ ** 3 / 8)) <= 0.1 * xi_ ** 4
    # coupling: force along +x turns the sphere about +y (rolling sense), (3/32) xi^4 mu_t / a
    assert abs(m[4, 0] / (mu_t / A) - 3 / 32 * xi_ ** 4) <= xi_ ** 5
    assert m[4, 0] > 0 and abs(m[3, 1] + m[4, 0]) <= 1e-15 and abs(m[5, 2]) <= 1e-15
    # no translation-rotation coupling normal to the wall, no cross terms
    for i, j in ((0, 1), (0, 2), (1, 2), (3, 5), (3, 4)):
        assert abs(m[i, j]) <= 1e-15


def test_open_mobility_recovered_far_from_the_wall():
    rng = np.random.default_rng(13)
    x = rng.random((6, 3)) * 8
    x[:, 2] += 1e4
    for ang in (False, True):
        mw = wall.grand_mobility_wall(x, A, ETA, ang)
        mo = mobility.grand_mobility(x, A, ETA, ang)
        assert np.abs(mw - mo).max() <= 2.0 / 1e4 * np.abs(mo).max()


def _config(n, seed, low=0.2):
    rng = np.random.default_rng(seed)
    side = (n * 4 / 3 * math.pi / 0.2) ** (1 / 3)
    return np.column_stack([rng.random((n, 2)) * side, low + rng.random(n) * side * 0.3])


@pytest.mark.parametrize("angular", [False, True])
def test_symmetric_and_positive_definite_with_damping(angular):
    x = _config(40, 14)
    assert (x[:, 2] < A).sum() >= 3          # some particles overlap the wall
    m = wall.grand_mobility_wall(x, A, ETA, angular)
    assert np.abs(m - m.T).max() <= 1e-14 * np.abs(m).max()
    assert np.linalg.eigvalsh(m).min() > 0
    m0 = wall.grand_mobility_wall(x, A, ETA, angular, damping=False)
    assert np.abs(m0 - m0.T).max() <= 1e-14 * np.abs(m0).max()
    assert np.linalg.eigvalsh(m0).min() < 0       # the undamped kernel is not SPD here


def test_damping_continuous_at_contact_and_zero_at_the_wall():
    x = _config(12, 15, low=2.0)
    for eps in (1e-7, -1e-7):
        xp = x.copy()
        xp[0, 2] = A * (1 + eps)
        x0 = x.copy()
        x0[0, 2] = A
        d = wall.grand_mobility_wall(xp, A, ETA, True) - wall.grand_mobility_wall(x0, A, ETA, True)
        assert np.abs(d).max() <= 1e-5
    xw = x.copy()
    xw[0, 2] = 0.0
    m = wall.grand_mobility_wall(xw, A, ETA, True)
    rows = [0, 1, 2, 36, 37, 38]
    assert np.abs(m[rows]).max() == 0.0 and np.abs(m[:, rows]).max() == 0.0
    # a wall placed elsewhere shifts every height
    xs = x.copy()
    xs[:, 2] += 3.5
    assert np.abs(wall.grand_mobility_wall(xs, A, ETA, True, wall_height=3.5)
                  - wall.grand_mobility_wall(x, A, ETA, True)).max() <= 1e-13


def test_drift_of_one_sphere_is_the_slope_of_its_normal_mobility():
    mu_t, _ = mobility.self_mobility(ETA, A)
    for h in (1.5, 3.0, 8.0):
        x = np.array([[0.2, 0.1, h]])
        fd = drift.divergence_fd(x, 1e-4, A, ETA, angular=True,
                                 mobility=lambda xx, a, eta, ang: wall.grand_mobility_wall(xx, a, eta, ang))
        slope = mu_t * (9 * A / (8 * h ** 2) - 3 * A ** 3 / (2 * h ** 4) + 5 * A ** 5 / (8 * h ** 6))
        assert np.abs(fd[[0, 1, 3, 4, 5]]).max() <= 1e-9
        assert abs(fd[2] - slope) <= 1e-7 * slope

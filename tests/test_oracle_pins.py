"""Pins of the oracle's mobility against facts the paper and classical
hydrodynamics fix independently of its formulas (CPU only).

* Eq. (stokestomob) with the sphere-surface envelope: every pair block is the
  surface average, over sphere i, of the flow that a force (or torque)
  spread over sphere j's surface creates.  That flow is the classical Stokes
  solution for a translating (rotating) rigid sphere outside sphere j and a
  rigid motion inside it, and the angular velocity is half the vorticity
  (eq. (kinetic_constraint)), i.e. (3/(2a)) <n x v> over the surface.  The
  quadrature below builds all four blocks from those textbook fields alone.
* The self block is the Stokes drag 1/(6 pi eta a) (Sec. 3.5, SelfMobility).
* Far field: the Oseen tensor plus the a^2/3 Laplacian correction; its
  half-curl gives the coupling block.
* Symmetry, positive definiteness, equivariance and zero divergence of the
  assembled matrix (Sec. 2, Sec. 4).
"""
import math

import numpy as np
import pytest

from oracle import mobility as mob
from oracle import drift

A_RADIUS = 1.3
ETA = 0.7


# ---------------------------------------------------------------------------
# independent construction from single-sphere Stokes solutions
# ---------------------------------------------------------------------------

def _sphere_flow_force(p, F, a, eta):
    """Velocity at points p (...,3) due to force F spread on a sphere at 0.

    Outside: Stokes' translating-sphere solution with U = F/(6 pi eta a);
    inside: the rigid translation U.
    """
    U = F / (6 * math.pi * eta * a)
    rho = np.linalg.norm(p, axis=-1)[..., None]
    up = (p @ U)[..., None]
    out = (0.75 * a * (U / rho + up * p / rho ** 3)
           + 0.25 * a ** 3 * (U / rho ** 3 - 3 * up * p / rho ** 5))
    return np.where(rho < a, U, out)


def _sphere_flow_torque(p, T, a, eta):
    """Velocity at p due to torque T spread on a sphere at 0 (rotating sphere)."""
    om = T / (8 * math.pi * eta * a ** 3)
    rho = np.linalg.norm(p, axis=-1)[..., None]
    rot = np.cross(om, p)
    return np.where(rho < a, rot, rot * (a / rho) ** 3)


def _surface_nodes(r, a, nq=64, nphi=16):
    """Quadrature nodes n and weights on the unit sphere, split where the
    surface of sphere i (centre r z) crosses the surface of sphere j (centre 0)."""
    mus = []
    ws = []
    cuts = [-1.0, 1.0]
    if 0 < r < 2 * a:
        cuts = [-1.0, -r / (2 * a), 1.0]
    x, w = np.polynomial.legendre.leggauss(nq)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        mus.append(0.5 * (hi - lo) * x + 0.5 * (hi + lo))
        ws.append(0.5 * (hi - lo) * w)
    mu = np.concatenate(mus)
    wmu = np.concatenate(ws)
    phi = 2 * math.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - mu ** 2)
    n = np.stack([st[:, None] * np.cos(phi)[None, :], st[:, None] * np.sin(phi)[None, :],
                  np.broadcast_to(mu[:, None], (len(mu), nphi))], -1).reshape(-1, 3)
    wt = (wmu[:, None] * np.full(nphi, 1.0 / nphi)[None, :]).reshape(-1) / 2.0
    return n, wt


def _blocks_by_quadrature(r, a, eta):
    """(M_tt, M_wF, M_uT, M_rr) for r_ij = r z by surface averaging."""
    n, wt = _surface_nodes(r, a)
    p = np.array([0.0, 0.0, r]) + a * n
    tt = np.zeros((3, 3)); wf = np.zeros((3, 3)); ut = np.zeros((3, 3)); rr = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3); e[k] = 1.0
        vf = _sphere_flow_force(p, e, a, eta)
        vt = _sphere_flow_torque(p, e, a, eta)
        tt[:, k] = wt @ vf
        ut[:, k] = wt @ vt
        wf[:, k] = 1.5 / a * (wt @ np.cross(n, vf))
        rr[:, k] = 1.5 / a * (wt @ np.cross(n, vt))
    return tt, wf, ut, rr


@pytest.mark.parametrize("r_over_a", [0.0, 0.05, 0.3, 0.77, 1.0, 1.5, 1.99, 2.0, 2.01, 2.6, 4.0, 9.0])
def test_blocks_equal_surface_average_of_stokes_flows(r_over_a):
    a, eta = A_RADIUS, ETA
    r = r_over_a * a
    tt_q, wf_q, ut_q, rr_q = _blocks_by_quadrature(r, a, eta)
    xt = np.array([[0.0, 0.0, r]])
    xs = np.array([[0.0, 0.0, 0.0]])
    tt, rr, c = mob.pair_blocks(xt, xs, a, eta, angular=True)
    scale_t = 1 / (6 * math.pi * eta * a)
    scale_r = 1 / (8 * math.pi * eta * a ** 3)
    scale_c = 1 / (8 * math.pi * eta * a ** 2)
    np.testing.assert_allclose(tt[0, 0], tt_q, atol=1e-12 * scale_t, rtol=0)
    np.testing.assert_allclose(rr[0, 0], rr_q, atol=1e-12 * scale_r, rtol=0)
    np.testing.assert_allclose(c[0, 0], wf_q, atol=1e-12 * scale_c, rtol=0)
    np.testing.assert_allclose(c[0, 0], ut_q, atol=1e-12 * scale_c, rtol=0)


def test_self_block_is_stokes_drag():
    a, eta = A_RADIUS, ETA
    x = np.array([[0.3, -1.0, 2.0]])
    F = np.array([[1.0, -2.0, 0.5]])
    T = np.array([[0.2, 0.4, -1.1]])
    U, W = mob.mdot_dense(x, F, T, a, eta)
    np.testing.assert_allclose(U, F / (6 * math.pi * eta * a), rtol=1e-15)
    np.testing.assert_allclose(W, T / (8 * math.pi * eta * a ** 3), rtol=1e-15)
    mu_t, mu_r = mob.self_mobility(1.0 / (6 * math.pi), 1.0)
    assert mu_t == pytest.approx(1.0, rel=1e-15) and mu_r == pytest.approx(0.75, rel=1e-15)


def _oseen(p, eta):
    rho = np.linalg.norm(p)
    return (np.eye(3) / rho + np.outer(p, p) / rho ** 3) / (8 * math.pi * eta)


def _fd_laplacian(fun, p, h):
    out = 0.0
    for k in range(3):
        e = np.zeros(3); e[k] = h
        out = out + (-fun(p + 2 * e) + 16 * fun(p + e) - 30 * fun(p) + 16 * fun(p - e) - fun(p - 2 * e)) / (12 * h * h)
    return out


@pytest.mark.parametrize("r_over_a", [2.0, 2.5, 5.0, 40.0])
def test_far_field_is_oseen_plus_laplacian_correction(r_over_a):
    a, eta = A_RADIUS, ETA
    rng = np.random.default_rng(5)
    d = rng.standard_normal(3); d /= np.linalg.norm(d)
    p = r_over_a * a * d
    fun = lambda q: _oseen(q, eta)
    ref = fun(p) + a * a / 3 * _fd_laplacian(fun, p, 1e-2 * np.linalg.norm(p))
    tt = mob.pair_blocks(p[None], np.zeros((1, 3)), a, eta)[0, 0]
    np.testing.assert_allclose(tt, ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_oseen_limit_and_self_mobility_limit():
    a, eta = 1.0, 1 / (6 * math.pi)
    for r in [1e3, 1e4, 1e6]:
        d = np.array([r, 0.0, 0.0])
        tt = mob.pair_blocks(d[None], np.zeros((1, 3)), a, eta)[0, 0]
        os_ = _oseen(d, eta)
        assert np.abs(tt - os_).max() <= 1.01 * (2 * a * a / r ** 2) * np.abs(os_).max()
    x = np.array([[0.0, 0, 0], [1e6, 0, 0], [0, 1e6, 0]])
    m = mob.grand_mobility(x, a, eta)
    np.testing.assert_allclose(m, np.eye(9), atol=1.6e-6)   # off-diagonal 2/(8 pi eta r) = 1.5e-6


@pytest.mark.parametrize("r_over_a", [2.5, 7.0, 30.0])
def test_coupling_is_half_curl_of_stokeslet(r_over_a):
    a, eta = A_RADIUS, ETA
    rng = np.random.default_rng(9)
    d = rng.standard_normal(3); d /= np.linalg.norm(d)
    p = r_over_a * a * d
    F = rng.standard_normal(3)
    field = lambda q: _oseen(q, eta) @ F + a * a / 6 * _fd_laplacian(lambda s: _oseen(s, eta), q, 1e-2 * np.linalg.norm(q)) @ F
    h = 1e-4 * np.linalg.norm(p)
    jac = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3); e[k] = h
        jac[:, k] = (field(p + e) - field(p - e)) / (2 * h)
    curl = np.array([jac[2, 1] - jac[1, 2], jac[0, 2] - jac[2, 0], jac[1, 0] - jac[0, 1]])
    _, _, c = mob.pair_blocks(p[None], np.zeros((1, 3)), a, eta, angular=True)
    np.testing.assert_allclose(c[0, 0] @ F, 0.5 * curl, rtol=0, atol=1e-6 * np.abs(curl).max())
    # sign fixed by physics: F along x at the origin, target on +y -> spin about +z
    _, _, c2 = mob.pair_blocks(np.array([[0.0, 5.0, 0.0]]), np.zeros((1, 3)), a, eta, angular=True)
    assert (c2[0, 0] @ np.array([1.0, 0, 0]))[2] > 0


def test_coefficients_continuous_and_c1_at_contact():
    a, eta = A_RADIUS, ETA
    eps = 1e-7 * a
    lo = np.array(mob.coefficients(np.array([2 * a - eps, 2 * a - 2 * eps]), a, eta))
    hi = np.array(mob.coefficients(np.array([2 * a + eps, 2 * a + 2 * eps]), a, eta))
    at = np.array(mob.coefficients(np.array([2 * a]), a, eta))[:, 0]
    scale = np.abs(at) + 1e-300
    assert np.all(np.abs(lo[:, 0] - hi[:, 0]) <= 1e-6 * scale.max())
    slope_lo = (lo[:, 0] - lo[:, 1]) / eps
    slope_hi = (hi[:, 1] - hi[:, 0]) / eps
    np.testing.assert_allclose(slope_lo, slope_hi, rtol=1e-4, atol=1e-6 * np.abs(slope_hi).max())
    # exactly one ulp either side of contact
    r_lo = np.nextafter(2 * a, 0.0)
    r_hi = np.nextafter(2 * a, 10.0)
    np.testing.assert_allclose(np.array(mob.coefficients(np.array([r_lo]), a, eta)),
                               np.array(mob.coefficients(np.array([r_hi]), a, eta)), rtol=1e-12)


def _configs():
    rng = np.random.default_rng(11)
    yield "dilute", (rng.random((12, 3)) - 0.5) * 20.0
    yield "overlapping", (rng.random((40, 3)) - 0.5) * 4.0
    yield "chain", np.cumsum(np.r_[[[0.0, 0, 0]], 2.1 * rng.standard_normal((15, 3)) / np.sqrt(3)], axis=0)


@pytest.mark.parametrize("angular", [False, True])
def test_grand_mobility_symmetric_positive_definite(angular):
    a, eta = 1.0, 1 / (6 * math.pi)
    for name, x in _configs():
        m = mob.grand_mobility(x, a, eta, angular)
        np.testing.assert_allclose(m, m.T, rtol=0, atol=1e-15 * np.abs(m).max(), err_msg=name)
        lam = np.linalg.eigvalsh(m)
        assert lam.min() > 0, (name, lam.min())


def test_coincident_particles_make_matrix_semidefinite():
    a, eta = 1.0, 1 / (6 * math.pi)
    x = np.array([[0.0, 0, 0], [0.0, 0, 0]])
    lam = np.linalg.eigvalsh(mob.grand_mobility(x, a, eta, True))
    assert abs(lam.min()) < 1e-14 and lam.max() > 0


def test_equivariance_rotation_translation_permutation_scaling():
    a, eta = 1.0, 1 / (6 * math.pi)
    rng = np.random.default_rng(3)
    x = (rng.random((25, 3)) - 0.5) * 6
    F = rng.standard_normal((25, 3)); T = rng.standard_normal((25, 3))
    U, W = mob.mdot_dense(x, F, T, a, eta)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    t = rng.standard_normal(3) * 10
    U2, W2 = mob.mdot_dense(x @ q.T + t, F @ q.T, T @ q.T, a, eta)
    np.testing.assert_allclose(U2, U @ q.T, atol=1e-13)
    np.testing.assert_allclose(W2, W @ q.T, atol=1e-13)
    perm = rng.permutation(25)
    U3, W3 = mob.mdot_dense(x[perm], F[perm], T[perm], a, eta)
    np.testing.assert_allclose(U3, U[perm], atol=1e-14)
    np.testing.assert_allclose(W3, W[perm], atol=1e-14)
    s = 2.5
    U4, W4 = mob.mdot_dense(s * x, F, T, s * a, eta)
    np.testing.assert_allclose(U4, mob.mdot_dense(x, F, None, a, eta)[0] / s
                               + (mob.mdot_dense(x, np.zeros_like(F), T, a, eta)[0]) / s ** 2, atol=1e-13)


def test_linearity_and_torque_only_input():
    a, eta = 1.0, 1 / (6 * math.pi)
    rng = np.random.default_rng(4)
    x = (rng.random((10, 3)) - 0.5) * 5
    F1, F2 = rng.standard_normal((2, 10, 3))
    T = rng.standard_normal((10, 3))
    u1, _ = mob.mdot_dense(x, F1, None, a, eta)
    u2, _ = mob.mdot_dense(x, F2, None, a, eta)
    u12, _ = mob.mdot_dense(x, 2 * F1 - 3 * F2, None, a, eta)
    np.testing.assert_allclose(u12, 2 * u1 - 3 * u2, atol=1e-13)
    ut, wt = mob.mdot_dense(x, None, T, a, eta)
    uz, wz = mob.mdot_dense(x, np.zeros_like(T), T, a, eta)
    np.testing.assert_array_equal(ut, uz)
    np.testing.assert_array_equal(wt, wz)
    with pytest.raises(ValueError):
        mob.mdot_dense(x, None, None, a, eta)


@pytest.mark.parametrize("angular", [False, True])
def test_divergence_vanishes_in_open_space(angular):
    a, eta = 1.0, 1 / (6 * math.pi)
    rng = np.random.default_rng(8)
    x = (rng.random((6, 3)) - 0.5) * 3.0       # several overlapping pairs
    div = drift.divergence_fd(x, 1e-4, a, eta, angular)
    assert np.abs(div).max() < 1e-8
    lin, ang = drift.div_m_open(6, angular)
    assert not lin.any() and (ang is None or not ang.any())


def test_dense_rows_and_c_pairloop_agree(pairloop):
    a, eta = 1.0, 1 / (6 * math.pi)
    rng = np.random.default_rng(12)
    n = 300
    x = (rng.random((n, 3)) - 0.5) * 12
    F = rng.standard_normal((n, 3)); T = rng.standard_normal((n, 3))
    for torques in (None, T):
        U, W = mob.mdot_dense(x, F, torques, a, eta)
        Uc, Wc = pairloop.mdot(x, F, torques, a, eta)
        scale = np.abs(U).max()
        np.testing.assert_allclose(Uc, U, rtol=0, atol=1e-14 * scale * 4)
        rows = rng.choice(n, 37, replace=False)
        Ur, Wr = mob.mdot_rows(x, rows, F, torques, a, eta)
        Ucr, Wcr = pairloop.mdot_rows(x, rows, F, torques, a, eta)
        np.testing.assert_allclose(Ur, U[rows], rtol=0, atol=1e-14 * scale * 4)
        np.testing.assert_allclose(Ucr, U[rows], rtol=0, atol=1e-14 * scale * 4)
        if torques is not None:
            ws = np.abs(W).max()
            np.testing.assert_allclose(Wc, W, rtol=0, atol=1e-14 * ws * 4)
            np.testing.assert_allclose(Wr, W[rows], rtol=0, atol=1e-14 * ws * 4)
            np.testing.assert_allclose(Wcr, W[rows], rtol=0, atol=1e-14 * ws * 4)
    # torque only through the C loop
    Ut, Wt = pairloop.mdot(x, None, T, a, eta)
    U0, W0 = mob.mdot_dense(x, None, T, a, eta)
    np.testing.assert_allclose(Ut, U0, atol=1e-13)
    np.testing.assert_allclose(Wt, W0, atol=1e-13)


def test_pairloop_binding_rejects_malformed_inputs(pairloop):
    """The C loop reads 3N values of every array and any row index it is
    given: the binding refuses shapes and rows that would take it outside."""
    rng = np.random.default_rng(11)
    x = rng.random((6, 3))
    f = rng.standard_normal((6, 3))
    for call in (lambda: pairloop.mdot(x, f[:5]),
                 lambda: pairloop.mdot(x.reshape(-1), f),
                 lambda: pairloop.mdot(x, f, f[:, :2]),
                 lambda: pairloop.mdot_rows(x, [6], f),
                 lambda: pairloop.mdot_rows(x, [-1], f),
                 lambda: pairloop.mdot_rows(x, [0.0], f),
                 lambda: pairloop.mdot_rows(x, [[0, 1]], f)):
        with pytest.raises(ValueError):
            call()
    u, _ = pairloop.mdot_rows(x, np.array([], dtype=np.int64), f)
    assert u.shape == (0, 3)
    u_all, _ = pairloop.mdot(x, f)
    u5, _ = pairloop.mdot_rows(x, [5, 0], f)
    assert np.array_equal(u5, u_all[[5, 0]])

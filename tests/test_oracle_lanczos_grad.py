"""Pins of the oracle's Lanczos square root, adjoint and drift (CPU only).

* Lanczos [Sec. 3.3]: with as many iterations as unknowns the Krylov space is
  the whole space, so the result must equal the exact symmetric root from a
  full eigendecomposition; the root squared must give back M; the small
  tridiagonal root is checked against scipy's Schur-based ``sqrtm`` (a
  different algorithm); the norm identity |y_k|^2 = W^T M W holds at every k.
* Fluctuation-dissipation [eq. (fdt), Sec. 4]: Z = M^{-1/2} M^{1/2} W is
  standard normal (Kolmogorov-Smirnov test).
* Adjoint: the analytic gradient equals the complex-step derivative of the
  dense forward map, and dL/dF is M g.
* Drift [eq. (rfd), Sec. 4]: random finite differences average to the
  (zero) divergence within their standard error.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import drift, gradient, lanczos, mobility as mob

A, ETA = 1.0, 1 / (6 * math.pi)


def _system(n, side, seed):
    rng = np.random.default_rng(seed)
    x = (rng.random((n, 3)) - 0.5) * side
    return x, rng


@pytest.mark.parametrize("angular", [False, True])
def test_full_krylov_space_gives_exact_root(angular):
    x, rng = _system(5, 3.0, 21)
    m = mob.grand_mobility(x, A, ETA, angular)
    w = rng.standard_normal(m.shape[0])
    y, info = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=0.0, maxit=m.shape[0])
    exact = lanczos.exact_sqrt_mdot_w(m, w)
    np.testing.assert_allclose(y, exact, rtol=0, atol=1e-12 * np.abs(exact).max())
    # the exact root really is a square root of M
    q = np.stack([lanczos.exact_sqrt_mdot_w(m, e) for e in np.eye(m.shape[0])], 1)
    np.testing.assert_allclose(q @ q, m, atol=1e-13)
    np.testing.assert_allclose(q, q.T, atol=1e-14)


def test_tridiagonal_root_matches_schur_sqrtm():
    rng = np.random.default_rng(2)
    k = 9
    al = 2 + rng.random(k)
    be = 0.5 * rng.random(k - 1)
    s, lam = lanczos.tridiagonal_sqrt_e1(al, be)
    t = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    ref = scipy.linalg.sqrtm(t).real[:, 0]
    np.testing.assert_allclose(s, ref, atol=1e-13)


def test_converged_lanczos_close_to_exact_root_and_norm_identity():
    x, rng = _system(150, 11.0, 22)
    m = mob.grand_mobility(x, A, ETA)
    w = rng.standard_normal(m.shape[0])
    y, info = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=1e-6)
    assert info.converged and not info.not_spd and 2 <= info.iters < 150
    exact = lanczos.exact_sqrt_mdot_w(m, w)
    err = np.linalg.norm(y - exact) / np.linalg.norm(exact)
    assert err < 1e-5, err
    # |y_k|^2 = beta0^2 e1^T T_k e1 = W^T M W while the basis stays orthonormal
    assert abs(y @ y - w @ m @ w) <= 1e-12 * (w @ m @ w)
    # matched-iteration rerun reproduces the same iterate bit for bit
    y2, info2 = lanczos.lanczos_sqrt(lambda v: m @ v, w, iters=info.iters)
    np.testing.assert_array_equal(y, y2)


def test_lanczos_prefactor_zero_vector_and_not_converged_flag():
    x, rng = _system(20, 6.0, 23)
    m = mob.grand_mobility(x, A, ETA)
    w = rng.standard_normal(60)
    y1, _ = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=1e-8)
    y2, _ = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=1e-8, prefactor=0.25)
    np.testing.assert_allclose(y2, 0.25 * y1, rtol=1e-15)
    z, info = lanczos.lanczos_sqrt(lambda v: m @ v, np.zeros(60))
    assert not z.any() and info.iters == 0
    _, info = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=0.0, maxit=3)
    assert not info.converged and info.iters == 3


def test_lanczos_flags_indefinite_operator():
    rng = np.random.default_rng(4)
    q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    m = q @ np.diag(np.r_[-1.0, np.ones(11)]) @ q.T
    _, info = lanczos.lanczos_sqrt(lambda v: m @ v, rng.standard_normal(12), tol=1e-10)
    assert info.not_spd


def test_fluctuation_dissipation_ks():
    x, rng = _system(8, 4.0, 24)
    m = mob.grand_mobility(x, A, ETA, True)
    inv_sqrt = lanczos.exact_inv_sqrt(m)
    zs = []
    for _ in range(400):
        w = rng.standard_normal(m.shape[0])
        y, _ = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=1e-10)
        zs.append(inv_sqrt @ y)
    z = np.concatenate(zs)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    cov = np.cov(np.stack(zs).T)
    assert np.abs(cov - np.eye(m.shape[0])).max() < 0.35


@pytest.mark.parametrize("angular", [False, True])
def test_adjoint_matches_complex_step(angular):
    x, rng = _system(9, 3.2, 25)               # several overlapping pairs
    F = rng.standard_normal((9, 3))
    T = rng.standard_normal((9, 3)) if angular else None
    gu = rng.standard_normal((9, 3))
    gw = rng.standard_normal((9, 3)) if angular else None

    def loss(xc):
        u, w = mob.mdot_dense(xc, F.astype(xc.dtype), None if T is None else T.astype(xc.dtype), A, ETA)
        val = (u * gu).sum()
        if angular:
            val = val + (w * gw).sum()
        return val

    dx, df, dt = gradient.mdot_vjp(x, F, T, gu, gw, A, ETA)
    cs = gradient.complex_step_grad(loss, x, range(27)).reshape(9, 3)
    np.testing.assert_allclose(dx, cs, rtol=0, atol=1e-12 * np.abs(cs).max())
    # dL/dF: the loss is linear in F, so the complex step is exact as well
    def loss_f(fc):
        u, w = mob.mdot_dense(x.astype(fc.dtype), fc, None if T is None else T.astype(fc.dtype), A, ETA)
        return (u * gu).sum() + ((w * gw).sum() if angular else 0.0)
    csf = gradient.complex_step_grad(loss_f, F, range(27)).reshape(9, 3)
    np.testing.assert_allclose(df, csf, rtol=0, atol=1e-13 * np.abs(csf).max())
    rows = np.array([0, 4, 7])
    dxr, dfr, dtr = gradient.mdot_vjp_rows(x, F, T, gu, gw, A, ETA, rows)
    np.testing.assert_allclose(dxr, dx[rows], atol=1e-13)
    np.testing.assert_allclose(dfr, df[rows], atol=1e-13)


def test_adjoint_central_difference_of_quadratic_loss():
    x, rng = _system(30, 6.0, 26)
    F = rng.standard_normal((30, 3))
    ustar = mob.mdot_dense(x + 0.1 * rng.standard_normal(x.shape), F, None, A, ETA)[0]
    def L(xx):
        u = mob.mdot_dense(xx, F, None, A, ETA)[0]
        return 0.5 * ((u - ustar) ** 2).sum()
    g = mob.mdot_dense(x, F, None, A, ETA)[0] - ustar
    dx, df, _ = gradient.mdot_vjp(x, F, None, g, None, A, ETA)
    h = 1e-4
    for c in rng.choice(90, 12, replace=False):
        xp = x.copy(); xp.flat[c] += h
        xm = x.copy(); xm.flat[c] -= h
        fd = (L(xp) - L(xm)) / (2 * h)
        assert abs(fd - dx.flat[c]) <= 1e-6 * max(1.0, abs(fd))


def test_random_finite_differences_average_to_zero():
    x, rng = _system(6, 3.0, 27)
    samples = []
    for _ in range(600):
        w = rng.standard_normal(18)
        lin, _ = drift.rfd_sample(x, w, 1e-4, A, ETA)
        samples.append(lin.reshape(-1))
    s = np.array(samples)
    mean = s.mean(0)
    se = s.std(0, ddof=1) / math.sqrt(len(s))
    assert np.all(np.abs(mean) <= 5 * se)
    det = drift.divergence_fd(x, 1e-4, A, ETA)
    assert np.abs(det - 0).max() < 1e-8


@pytest.mark.parametrize("angular", [False, True])
def test_rfd_sample_is_the_directional_derivative(angular):
    """One random finite difference [eq. (rfd)] equals (M'(X)[W_X]) W, the
    derivative of M along the positional part of W applied to W, up to
    O(delta^2): checked against the complex-step derivative of the oracle's
    mobility along W_X (independent of the difference formula; a sign or
    factor slip in either the displacement or the 1/delta fails)."""
    x, rng = _system(30, 9.0, 28)          # overlapping and far pairs
    w = rng.standard_normal(6 * 30 if angular else 3 * 30)
    delta = 1e-5
    lin, ang = drift.rfd_sample(x, w, delta, A, ETA, angular)
    wp = w[:90].reshape(30, 3)
    wt = w[90:].reshape(30, 3) if angular else None
    h = 1e-30
    u, om = mob.mdot_dense(x.astype(np.complex128) + 1j * h * wp, wp, wt, A, ETA)
    du = np.imag(u) / h
    assert np.abs(lin - du).max() <= 1e-7 * np.abs(du).max()
    if angular:
        dom = np.imag(om) / h
        assert np.abs(ang - dom).max() <= 1e-7 * np.abs(dom).max()


def _chain_matrix(n_chains=6, beads=20, angular=False):
    import workloads
    s = workloads.c5_chains(n_chains=n_chains, beads=beads)
    return s.pos, mob.grand_mobility(s.pos, 1.0, 1.0 / (6.0 * math.pi), angular)


@pytest.mark.parametrize("angular", [False, True])
def test_preconditioned_root_covariance_is_the_mobility(angular):
    """B = L (L^{-1} M L^{-T})^{1/2} satisfies B B^T = M (the fluctuation-
    dissipation balance of eq. (fdt) holds for the preconditioned noise),
    and Lanczos at k = n reproduces it (finite termination)."""
    x, m = _chain_matrix(3, 8, angular)
    n = x.shape[0]
    L = lanczos.group_cholesky(m, n, 8, angular)
    dim = m.shape[0]
    li = scipy.linalg.solve_triangular(L, np.eye(dim), lower=True)
    lam, q = np.linalg.eigh(li @ m @ li.T)
    B = L @ (q * np.sqrt(lam)) @ q.T
    assert np.abs(B @ B.T - m).max() <= 1e-12 * np.abs(m).max()
    e = np.random.default_rng(2).standard_normal(dim)
    assert np.abs(lanczos.exact_preconditioned_sqrt(m, L, e) - B @ e).max() <= 1e-12 * np.abs(B @ e).max()
    assert np.abs(np.tril(L) - L).max() == 0.0
    w = np.random.default_rng(3).standard_normal(dim)
    y, info = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, w, iters=dim)
    ex = lanczos.exact_preconditioned_sqrt(m, L, w)
    assert np.linalg.norm(y - ex) <= 1e-9 * np.linalg.norm(ex)


def test_preconditioned_with_single_particle_groups_is_plain_lanczos():
    """In open space every 3x3 self block is mu_t I, so groups of one particle
    give L = sqrt(mu_t) I: the preconditioned iterate is the plain one at
    every k and stops at the same iteration."""
    x, m = _chain_matrix(4, 10)
    L = lanczos.group_cholesky(m, x.shape[0], 1)
    assert np.abs(L - np.sqrt(m[0, 0]) * np.eye(m.shape[0])).max() <= 1e-15
    w = np.random.default_rng(4).standard_normal(m.shape[0])
    y0, i0 = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=1e-6)
    y1, i1 = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, w, tol=1e-6)
    assert i0.iters == i1.iters
    assert np.abs(y1 - y0).max() <= 1e-12 * np.abs(y0).max()


def test_group_preconditioner_cuts_iterations_on_chains():
    x, m = _chain_matrix(8, 24)
    w = np.random.default_rng(5).standard_normal(m.shape[0])
    _, i0 = lanczos.lanczos_sqrt(lambda v: m @ v, w, tol=1e-6)
    L = lanczos.group_cholesky(m, x.shape[0], 24)
    _, i1 = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, w, tol=1e-6)
    assert i1.iters < 0.7 * i0.iters


def test_preconditioned_noise_passes_the_fdt_ks_test():
    """Sec. 4: M^{-1/2} y is standard normal for the preconditioned noise too
    (the KS test is agnostic to which square root is used)."""
    import scipy.stats
    x, m = _chain_matrix(2, 12)
    L = lanczos.group_cholesky(m, x.shape[0], 12)
    minv = lanczos.exact_inv_sqrt(m)
    rng = np.random.default_rng(6)
    samples = []
    for _ in range(300):
        y, _ = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, rng.standard_normal(m.shape[0]), tol=1e-8)
        samples.append(minv @ y)
    p = scipy.stats.kstest(np.concatenate(samples), "norm").pvalue
    assert p > 1e-3

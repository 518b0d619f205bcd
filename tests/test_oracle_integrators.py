"""Pins of the oracle's time stepping of eq. (bdhi) (Sec. 3.2
LangevinVelocities as an Euler-Maruyama step; the stochastic Adams-Bashforth
scheme of Sec. 5.1) by properties the mathematics fixes:

* one sphere under a constant force moves by dt mu_t F per step exactly
  (both Adams-Bashforth weights see the same velocity; 3/2 - 1/2 = 1);
* without noise the scheme is second-order accurate: against a tight
  reference solution of dX/dt = M(X) F(X), halving dt divides the error
  at a fixed time by about 4 (a wrong weight pair, e.g. 1/2 and 1/2 or
  3/2 and 1/2 with the wrong sign, drops to first order or diverges);
* the first step, with no history, is the Euler-Maruyama step;
* the noise of the Langevin velocities has covariance (2 kT / dt) M
  (eq. (fdt) with dW = sqrt(dt) W).
"""
import math

import numpy as np
import pytest
import scipy.integrate

from oracle import integrators, lanczos, mobility

A, ETA = 1.0, 1 / (6 * math.pi)   # mu_t = 1


def _exact_root(angular=False):
    def f(x, v):
        m = mobility.grand_mobility(x, A, ETA, angular)
        return lanczos.exact_sqrt_mdot_w(m, v)
    return f


def test_single_sphere_constant_force_moves_exactly():
    x = np.array([[0.3, -1.2, 2.0]])
    F = np.array([[0.7, -0.2, 1.1]])
    dt = 0.05
    u_prev = None
    for _ in range(10):
        x, _, u_prev = integrators.ab2_step(x, F, None, None, dt, 0.0, A, ETA, None, u_prev)
    ref = np.array([[0.3, -1.2, 2.0]]) + 10 * dt * F      # mu_t = 1
    assert np.abs(x - ref).max() <= 1e-14


def _spring_forces(x):
    # two spheres tied by a Hookean spring of stiffness 0.5 and rest length 4,
    # plus a weak tether of every sphere to the origin (stiffness 0.05)
    d = x[0] - x[1]
    r = np.linalg.norm(d)
    f = -0.5 * (r - 4.0) * d / r
    return np.stack([f, -f]) - 0.05 * x


def test_deterministic_scheme_is_second_order():
    x0 = np.array([[3.5, 0.4, -0.2], [-3.1, -0.3, 0.5]])   # far apart: smooth far-field RPY
    T = 4.0

    def rhs(t, y):
        x = y.reshape(2, 3)
        u, _ = mobility.mdot_dense(x, _spring_forces(x), None, A, ETA)
        return u.reshape(-1)

    ref = scipy.integrate.solve_ivp(rhs, (0, T), x0.reshape(-1), method="DOP853", rtol=1e-13,
                                    atol=1e-13).y[:, -1].reshape(2, 3)
    errs = []
    for steps in (40, 80, 160):
        dt = T / steps
        x, u_prev = x0.copy(), None
        for _ in range(steps):
            x, _, u_prev = integrators.ab2_step(x, _spring_forces(x), None, None, dt, 0.0, A, ETA, None, u_prev)
        errs.append(np.abs(x - ref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8, errs


@pytest.mark.parametrize("angular", [False, True])
def test_first_step_is_euler_maruyama(angular):
    rng = np.random.default_rng(3)
    n = 6
    x = (rng.random((n, 3)) - 0.5) * 6.0
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3)) if angular else None
    w = rng.standard_normal(6 * n if angular else 3 * n)
    dt, kt = 0.02, 0.7
    root = _exact_root(angular)
    xn, dth, _ = integrators.ab2_step(x, F, T, w, dt, kt, A, ETA, root, None, angular)
    v, om = integrators.langevin_velocities(x, F, T, w, dt, kt, A, ETA, root, angular)
    assert np.abs(xn - (x + dt * v)).max() <= 1e-13
    if angular:
        assert np.abs(dth - dt * om).max() <= 1e-13


def test_langevin_noise_covariance_is_2kt_over_dt_m():
    rng = np.random.default_rng(4)
    x = np.array([[0.0, 0.0, 0.0], [1.7, 0.9, 0.2]])        # overlapping pair
    F = np.zeros((2, 3))
    dt, kt = 0.1, 0.5
    m = mobility.grand_mobility(x, A, ETA)
    root = _exact_root()
    samples = np.array([integrators.langevin_velocities(x, F, None, rng.standard_normal(6), dt, kt, A, ETA,
                                                        root)[0].reshape(-1) for _ in range(20000)])
    cov = np.cov(samples.T)
    target = 2 * kt / dt * m
    # standard error of a sample covariance entry of a Gaussian vector
    se = np.sqrt((np.outer(np.diag(target), np.diag(target)) + target ** 2) / len(samples))
    assert np.all(np.abs(cov - target) <= 5 * se)

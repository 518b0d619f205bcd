"""Pins of the oracle's conjugate gradients (``oracle.krylov``) by what the
mathematics fixes, independent of its own recurrence:

* finite termination: on an SPD matrix with m distinct eigenvalues CG
  reaches the solution in m iterations (here m = 3 in dimension 12), and
  not earlier for a right-hand side touching every eigenspace;
* a multiple of the identity is solved in one iteration;
* on the grand mobility (overlapping pairs present, angular blocks) the
  result matches a direct LU solve (numpy) to the tolerance times the
  condition number;
* the M-norm of the error decreases at every iteration (CG minimises it
  over the growing Krylov space); a wrong alpha or beta breaks this.
"""
import math

import numpy as np
import pytest

from oracle import krylov, mobility


def test_finite_termination_three_eigenvalues():
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.repeat([1.0, 3.0, 7.5], 4)
    a = (q * lam) @ q.T
    b = rng.standard_normal(12)
    x2, k2, res2 = krylov.conjugate_gradients(lambda v: a @ v, b, iters=2)
    x3, k3, res3 = krylov.conjugate_gradients(lambda v: a @ v, b, iters=3)
    assert res2 > 1e-3
    assert res3 < 1e-12
    assert np.abs(x3 - np.linalg.solve(a, b)).max() < 1e-12


def test_identity_multiple_in_one_iteration():
    b = np.arange(1.0, 7.0)
    x, k, res = krylov.conjugate_gradients(lambda v: 2.5 * v, b, tol=1e-14)
    assert k == 1 and np.allclose(x, b / 2.5, rtol=0, atol=1e-15)


def test_zero_rhs():
    x, k, res = krylov.conjugate_gradients(lambda v: v, np.zeros(5))
    assert k == 0 and not x.any()


@pytest.mark.parametrize("angular", [False, True])
def test_mobility_solve_matches_direct_solve(angular):
    rng = np.random.default_rng(12)
    n = 40
    x = (rng.random((n, 3)) - 0.5) * 7.0       # dense enough for overlapping pairs
    m = mobility.grand_mobility(x, 1.0, 1 / (6 * math.pi), angular)
    b = rng.standard_normal(m.shape[0])
    tol = 1e-12
    sol, k, res = krylov.conjugate_gradients(lambda v: m @ v, b, tol=tol)
    ref = np.linalg.solve(m, b)
    kappa = np.linalg.cond(m)
    assert res < tol
    assert np.linalg.norm(sol - ref) / np.linalg.norm(ref) <= 10 * kappa * tol


def test_error_energy_norm_decreases():
    rng = np.random.default_rng(13)
    x = (rng.random((30, 3)) - 0.5) * 8.0
    m = mobility.grand_mobility(x, 1.0, 1 / (6 * math.pi), True)
    b = rng.standard_normal(m.shape[0])
    ref = np.linalg.solve(m, b)
    errs = []
    for k in range(1, 25):
        xk, _, _ = krylov.conjugate_gradients(lambda v: m @ v, b, iters=k)
        e = xk - ref
        errs.append(float(e @ m @ e))
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))


def test_indefinite_matrix_is_reported():
    a = np.diag([1.0, -2.0, 3.0])
    with pytest.raises(ValueError):
        krylov.conjugate_gradients(lambda v: a @ v, np.array([1.0, 1.0, 1.0]), tol=1e-14)

"""Pins of the triply periodic oracle (oracle/periodic.py) against what the
mathematics fixes, independent of its own formulas:

* the Ewald split is exact: the total does not depend on the splitting
  parameter xi (a wrong sign, factor or term in either part breaks this);
* Hasimoto's expansion of the self mobility of one sphere in a cubic box,
  mu/mu0 = 1 - C (a/L) + (4 pi/3)(a/L)^3, C = 2.8372974794806 (Hasimoto 1959);
  the RPY lattice sum has no term of order (a/L)^6 (measured below 1e-10);
* the large-box limit: M_per - M_open -> -(C/(6 pi eta L)) I for every 3x3
  block, with the remainder falling as L^-3;
* the small-radius limit of the wave kernel at r = 0 (a closed form of the
  Gaussian integrals): Wr(0)/mu0 = 3 xi a / sqrt(pi) - (10/(3 sqrt(pi))) (xi a)^3 + O((xi a)^5);
* symmetry, positive definiteness of M, M_real and M_wave separately (the
  "positive" split), and invariance under periodic shifts;
* the Fourier-space fluctuations have covariance exactly M_wave: the linear
  map T from noise to sample satisfies T T^T = M_wave (the Hermitian pairing
  of the noise and its normalisation).
"""
import math

import numpy as np
import pytest

from oracle import mobility, periodic

A, ETA = 1.0, 1.0 / (6.0 * math.pi)      # mu0 = 1
HASIMOTO_C = 2.8372974794806


def _cfg(n, box, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (n, 3)) * np.asarray(box)


def test_total_is_independent_of_the_splitting_parameter():
    box = np.array([7.0, 8.0, 6.5])
    x = _cfg(9, box, 1)
    x[1] = x[0] + [1.2, 0.3, -0.5]           # an overlapping pair
    m1 = periodic.grand_mobility_periodic(x, box, A, ETA, xi=0.45)
    m2 = periodic.grand_mobility_periodic(x, box, A, ETA, xi=0.9)
    assert np.abs(m1 - m2).max() <= 1e-11 * np.abs(m1).max()
    # the two parts do depend on xi
    r1 = periodic.real_matrix(x, box, A, ETA, 0.45)
    r2 = periodic.real_matrix(x, box, A, ETA, 0.9)
    assert np.abs(r1 - r2).max() > 1e-2


@pytest.mark.parametrize("L", [6.0, 10.0, 25.0])
def test_hasimoto_self_mobility(L):
    x = np.array([[0.3 * L, 0.6 * L, 0.1 * L]])
    m = periodic.grand_mobility_periodic(x, L, A, ETA)
    e = A / L
    ref = 1.0 - HASIMOTO_C * e + (4.0 * math.pi / 3.0) * e ** 3
    assert np.abs(m - ref * np.eye(3)).max() <= 1e-10


def test_large_box_limit_is_the_open_mobility_shifted_by_the_lattice_constant():
    x = np.array([[10.0, 10.0, 10.0], [12.5, 11.0, 10.4], [10.3, 9.1, 11.9]])
    mo = mobility.grand_mobility(x, A, ETA, False)
    shift = np.kron(np.ones((3, 3)), np.eye(3))
    res = []
    for L in (100.0, 200.0):
        mp = periodic.grand_mobility_periodic(x, L, A, ETA)
        res.append(np.abs(mp - mo + (HASIMOTO_C / L) * shift).max())
    assert res[0] < 1e-4
    assert abs(res[0] / res[1] - 8.0) < 0.1          # remainder ~ L^-3


@pytest.mark.parametrize("xi", [1.0, 3.0])
def test_wave_kernel_at_zero_small_radius_limit(xi):
    a = 0.01 / xi
    f, g = periodic.wave_radial(np.array([0.0]), a, ETA, xi)
    mu0 = 1.0 / (6.0 * math.pi * ETA * a)
    e = xi * a
    ref = 3.0 * e / math.sqrt(math.pi) - 10.0 / (3.0 * math.sqrt(math.pi)) * e ** 3
    assert abs(f[0] / mu0 - ref) <= 1e-9
    assert g[0] == 0.0


def test_real_space_kernel_vanishes_at_the_cutoff():
    xi = 0.7
    r = np.array([7.5 / xi])
    c1, c2, *_ = mobility.coefficients(r, A, ETA)
    f, g = periodic.wave_radial(r, A, ETA, xi)
    assert abs(c1[0] - f[0]) < 1e-12 and abs(c2[0] - g[0]) < 1e-12


def test_symmetric_positive_definite_and_each_part_too():
    box = np.array([6.0, 6.0, 7.0])
    x = _cfg(14, box, 2)
    x[3] = x[2]                                   # coincident pair
    xi = 0.8
    mr = periodic.real_matrix(x, box, A, ETA, xi)
    mw = periodic.wave_matrix(x, box, A, ETA, xi)
    for m in (mr, mw, mr + mw):
        assert np.abs(m - m.T).max() <= 1e-13 * np.abs(m).max()
    # the coincident pair makes M singular in exact arithmetic: positive semidefinite
    for m in (mr, mw):
        assert np.linalg.eigvalsh(0.5 * (m + m.T)).min() > -1e-12
    x[3] += [0.4, 0.0, 0.0]
    m = periodic.grand_mobility_periodic(x, box, A, ETA, xi)
    assert np.linalg.eigvalsh(0.5 * (m + m.T)).min() > 1e-6


def test_periodic_shift_and_translation_invariance():
    box = np.array([6.5, 7.0, 6.0])
    x = _cfg(7, box, 3)
    m = periodic.grand_mobility_periodic(x, box, A, ETA)
    n = np.random.default_rng(4).integers(-3, 4, (7, 3))
    m_img = periodic.grand_mobility_periodic(x + n * box, box, A, ETA)
    m_tr = periodic.grand_mobility_periodic(x + [0.37, -1.1, 2.9], box, A, ETA)
    assert np.abs(m_img - m).max() <= 1e-12
    assert np.abs(m_tr - m).max() <= 1e-12


def test_wave_fluctuations_have_covariance_m_wave():
    """T T^T = M_wave where T maps the half-spectrum noise to the sample
    (grid fine enough to hold every wave vector with |k| <= 14 xi)."""
    box = np.array([5.0, 5.5, 4.5])
    xi, grid = 0.3, (8, 10, 9)
    x = _cfg(4, box, 5)
    m = 3 * grid[0] * grid[1] * (grid[2] // 2 + 1) * 2
    T = np.zeros((12, m))
    e = np.zeros(m)
    for c in range(m):
        e[c] = 1.0
        T[:, c] = periodic.wave_fluctuation(x, box, A, ETA, xi, grid, e).reshape(-1)
        e[c] = 0.0
    mw = periodic.wave_matrix(x, box, A, ETA, xi)
    assert np.abs(T @ T.T - mw).max() <= 1e-14 * np.abs(mw).max() + 1e-15

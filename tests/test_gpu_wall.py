"""GPU parity of the single-wall geometry (Sec. 3.5, NBody with single_wall:
the Swan-Brady kernel with damping for wall overlaps) against the float64
oracle (oracle/wall.py), through the C interface.

* Mdot: every N from one particle to several tiles with a ragged tail,
  linear and angular, float32 and float64, particles overlapping the wall
  and each other, a wall away from z = 0, particles on and below the wall;
  sampled rows at N = 16,384.
* sqrtMdotW: matched-iteration parity against the oracle's Lanczos on the
  dense wall mobility, and against its exact symmetric root at tol 1e-6.
* Drift: one random finite difference (eq. (rfd)) against the oracle's
  sample for the same W, and the mean of many samples against the oracle's
  deterministic finite-difference divergence (nonzero above a wall).
* Multi-vector products and error paths of the wall solver.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import drift, lanczos, wall
from tests.gpu_util import emax, host, rounded, say, to_dev, tol_for

pytestmark = pytest.mark.gpu
DTYPES = [torch.float64, torch.float32]


def _solver(angular, wall_height=0.0, a=workloads.RADIUS, eta=workloads.VISCOSITY):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver("open", "open", "single_wall")
    s.setParameters(wallHeight=wall_height)
    s.initialize(viscosity=eta, hydrodynamicRadius=a, includeAngular=angular)
    return s


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("n", [1, 2, 7, 257, 700])
def test_wall_mdot_against_oracle(dtype, angular, n):
    say(f"case wall mdot n={n} angular={angular} {dtype}")
    s = workloads.wall_suspension(n, 300 + n, hg=1.5, phi2d=0.3, torques=angular, wall_height=-2.5)
    wh = s.extra["wall_height"]
    sol = _solver(angular, wh)
    sol.setPositions(to_dev(s.pos, dtype))
    lin, ang = sol.Mdot(to_dev(s.forces, dtype), to_dev(s.torques, dtype) if angular else None)
    x, f = rounded(s.pos, dtype), rounded(s.forces, dtype)
    t = rounded(s.torques, dtype) if angular else None
    u, w = wall.mdot_wall(x, f, t, s.radius, s.viscosity, wh)
    e = emax(host(lin), u)
    if angular:
        e = max(e, emax(host(ang), w))
    say(f"  e_max {e:.3e}")
    assert e <= tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_wall_torque_only_force_only_and_particles_on_or_below_the_wall(dtype):
    say(f"case wall special rows {dtype}")
    s = workloads.wall_suspension(300, 41, hg=2.0, phi2d=0.4, torques=True)
    x = s.pos.copy()
    x[0, 2] = 0.0          # on the wall: damping 0
    x[1, 2] = -0.7         # below it: damping 0
    x[2, 2] = 1.0          # at contact: damping 1
    x[3] = x[4]            # coincident pair
    sol = _solver(True)
    sol.setPositions(to_dev(x, dtype))
    xr = rounded(x, dtype)
    T = to_dev(s.torques, dtype)
    lin, ang = sol.Mdot(None, T)
    u, w = wall.mdot_wall(xr, None, rounded(s.torques, dtype), s.radius, s.viscosity)
    e = max(emax(host(lin), u), emax(host(ang), w))
    lin2, ang2 = sol.Mdot(to_dev(s.forces, dtype), None)
    u2, w2 = wall.mdot_wall(xr, rounded(s.forces, dtype), np.zeros((300, 3)), s.radius, s.viscosity)
    e = max(e, emax(host(lin2), u2), emax(host(ang2), w2))
    say(f"  e_max {e:.3e}")
    assert e <= tol_for(dtype)
    for rows in (host(lin), host(ang), host(lin2), host(ang2)):
        assert np.abs(rows[:2]).max() == 0.0


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
def test_wall_sqrt_mdot_w_matched_and_exact(dtype, angular):
    say(f"case wall lanczos angular={angular} {dtype}")
    n = 240
    s = workloads.wall_suspension(n, 77, hg=1.8, phi2d=0.35, w=True, angular_w=angular)
    sol = _solver(angular)
    sol.setPositions(to_dev(s.pos, dtype))
    lin, ang = sol.sqrtMdotW(to_dev(s.w, dtype), prefactor=0.7, tol=1e-6)
    k = sol.last_iterations
    y = np.concatenate([host(lin).reshape(-1)] + ([host(ang).reshape(-1)] if angular else []))
    xr, wr = rounded(s.pos, dtype), rounded(s.w, dtype)
    m = wall.grand_mobility_wall(xr, s.radius, s.viscosity, angular)
    y_ref, _ = lanczos.lanczos_sqrt(lambda v: m @ v, wr, iters=k, prefactor=0.7)
    e = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
    exact = lanczos.exact_sqrt_mdot_w(m, wr, 0.7)
    e2 = float(np.linalg.norm(y - exact) / np.linalg.norm(exact))
    say(f"  {k} iterations; matched max rel {e:.3e}; vs exact root {e2:.3e}")
    assert e <= (1e-12 if dtype == torch.float64 else 1e-5)
    assert e2 <= 1e-5


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
def test_wall_rfd_sample_against_oracle(dtype, angular):
    say(f"case wall rfd sample angular={angular} {dtype}")
    n = 150
    s = workloads.wall_suspension(n, 91, hg=1.6, phi2d=0.3, w=True, angular_w=angular)
    sol = _solver(angular)
    sol.setPositions(to_dev(s.pos, dtype))
    delta = 1e-3 if dtype == torch.float32 else 1e-4
    lin, ang = sol.divM_rfd(to_dev(s.w, dtype), delta=delta)
    xr, wr = rounded(s.pos, dtype), rounded(s.w, dtype)
    npd = np.float32 if dtype == torch.float32 else np.float64
    rnd = lambda v: np.asarray(v, npd).astype(np.float64)
    mdot = lambda x, f, t, a, eta: wall.mdot_wall(x, f, t, a, eta)
    ul, ua = drift.rfd_sample(xr, wr, delta, s.radius, s.viscosity, angular, round_positions=rnd, mdot=mdot)
    # each product at its Mdot bar: 2 bar max|M(X +- delta/2 W) W| / delta, absolute
    wp = wr[:3 * n].reshape(n, 3)
    wt = wr[3 * n:].reshape(n, 3) if angular else None
    up, op = mdot(rnd(xr + 0.5 * delta * wp), wp, wt, s.radius, s.viscosity)
    scale = max(np.abs(up).max(), np.abs(op).max() if angular else 0.0)
    bar = 2 * tol_for(dtype) * scale / delta
    err = np.abs(host(lin) - ul).max()
    if angular:
        err = max(err, np.abs(host(ang) - ua).max())
    say(f"  max abs diff {err:.3e} (bar {bar:.3e}); drift scale {np.abs(ul).max():.3e}")
    assert err <= bar


def test_wall_rfd_mean_against_oracle_divergence():
    """The average of float64 RFD samples converges to the oracle's
    deterministic divergence (5 standard errors), which is not zero."""
    say("case wall rfd mean")
    n = 12
    s = workloads.wall_suspension(n, 5, hg=1.4, phi2d=0.5, overlap=0.0)
    sol = _solver(False)
    sol.setPositions(to_dev(s.pos, torch.float64))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(123)
    samples = []
    for _ in range(4000):
        lin, _ = sol.divM_rfd(delta=1e-4, generator=gen)
        samples.append(host(lin).reshape(-1))
    smp = np.array(samples)
    mean = smp.mean(0)
    se = smp.std(0, ddof=1) / math.sqrt(len(smp))
    ref = drift.divergence_fd(s.pos, 1e-5, s.radius, s.viscosity, False,
                              mobility=lambda x, a, eta, ang: wall.grand_mobility_wall(x, a, eta, ang))
    z = np.abs(mean - ref) / np.maximum(se, 1e-300)
    say(f"  max |mean - div| / se = {z.max():.2f}; |div|_max = {np.abs(ref).max():.3e}")
    assert np.abs(ref).max() > 5 * se.max()
    assert z.max() <= 5.0


@pytest.mark.parametrize("dtype", DTYPES)
def test_wall_sampled_rows_n16384(dtype):
    say(f"case wall N=16384 sampled rows {dtype}")
    n = 16384
    s = workloads.wall_suspension(n, 2024, hg=1.5, torques=True)
    sol = _solver(True)
    sol.setPositions(to_dev(s.pos, dtype))
    lin, ang = sol.Mdot(to_dev(s.forces, dtype), to_dev(s.torques, dtype))
    rows = np.sort(np.random.default_rng(9).choice(n, 24, replace=False))
    rows[0] = int(np.argmin(s.pos[:, 2]))          # one that overlaps the wall
    x, f, t = rounded(s.pos, dtype), rounded(s.forces, dtype), rounded(s.torques, dtype)
    u, w = wall.mdot_wall_rows(x, rows, f, t, s.radius, s.viscosity)
    e = max(emax(host(lin)[rows], u), emax(host(ang)[rows], w))
    say(f"  e_max {e:.3e}")
    assert e <= tol_for(dtype)


def test_wall_multi_vector_products_equal_single_products():
    say("case wall multi")
    n = 500
    s = workloads.wall_suspension(n, 17, hg=2.0, torques=True)
    sol = _solver(True)
    sol.setPositions(to_dev(s.pos, torch.float32))
    rng = np.random.default_rng(4)
    F = to_dev(rng.standard_normal((3, n, 3)), torch.float32)
    T = to_dev(rng.standard_normal((3, n, 3)), torch.float32)
    lm, am = sol.MdotMulti(F, T)
    for r in range(3):
        l1, a1 = sol.Mdot(F[r], T[r])
        assert torch.equal(l1, lm[r]) and torch.equal(a1, am[r])


def test_wall_error_paths():
    import paper_2510_02135_amd as rpy
    from paper_2510_02135_amd import _lib
    say("case wall errors")
    sol = _solver(True)
    sol.setPositions(to_dev(np.array([[0.0, 0.0, 2.0], [3.0, 0.0, 1.5]]), torch.float64))
    F = to_dev(np.ones((2, 3)), torch.float64)
    with pytest.raises(_lib.RpyError) as ei:
        sol.Mdot_backward(F, None, F)
    assert ei.value.status == _lib.Status.UNSUPPORTED_GEOMETRY
    lin = torch.empty((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.RpyError) as ei:
        _lib.rpy_div_m(sol._h, lin, lin, torch.float64, 2)
    assert ei.value.status == _lib.Status.UNSUPPORTED_GEOMETRY
    with pytest.raises(_lib.RpyError):
        sol.setParameters(boxSize=3.0)
    op = rpy.Solver()
    with pytest.raises(_lib.RpyError):
        op.setParameters(wallHeight=0.0)
    with pytest.raises(_lib.RpyError) as ei:
        rpy.Solver("open", "open", "two_walls")
    assert ei.value.status == _lib.Status.UNSUPPORTED_GEOMETRY
    # the drift of divM above a wall is one random finite difference (nonzero)
    dl, da = sol.divM()
    assert torch.isfinite(dl).all() and float(dl.abs().max()) > 0

"""GPU parity of the preconditioned Lanczos fluctuations
(rpy_sqrt_mdot_w_precond: y = L (L^{-1} M L^{-T})^{1/2} W with L the block
Cholesky factor of M over groups of consecutive particles) against the
float64 oracle's algorithm (oracle.lanczos.preconditioned_lanczos_sqrt on the
dense mobility), through the C interface."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import lanczos, mobility, wall
from tests.gpu_util import host, rounded, say, to_dev

pytestmark = pytest.mark.gpu
DTYPES = [torch.float64, torch.float32]


def _solver(angular, geometry="open"):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver("open", "open", geometry)
    s.initialize(viscosity=workloads.VISCOSITY, hydrodynamicRadius=workloads.RADIUS, includeAngular=angular)
    return s


def _flat(lin, ang):
    return np.concatenate([host(lin).reshape(-1)] + ([host(ang).reshape(-1)] if ang is not None else []))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("chains,beads,group", [(6, 40, 40), (5, 48, 32), (3, 16, 1)])
def test_precond_lanczos_against_oracle(dtype, angular, chains, beads, group):
    say(f"case precond chains={chains}x{beads} group={group} angular={angular} {dtype}")
    s = workloads.c5_chains(n_chains=chains, beads=beads)
    n = s.n
    rng = np.random.default_rng(100 + chains)
    w = rng.standard_normal((6 if angular else 3) * n)
    sol = _solver(angular)
    sol.setPositions(to_dev(s.pos, dtype))
    lin, ang = sol.sqrtMdotWPrecond(to_dev(w, dtype), groupSize=group, prefactor=0.6, tol=1e-6)
    k = sol.last_iterations
    y = _flat(lin, ang)
    xr, wr = rounded(s.pos, dtype), rounded(w, dtype)
    m = mobility.grand_mobility(xr, s.radius, s.viscosity, angular)
    L = lanczos.group_cholesky(m, n, group, angular)
    y_ref, _ = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, wr, iters=k, prefactor=0.6)
    _, info = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, wr, tol=1e-6)
    _, plain = lanczos.lanczos_sqrt(lambda v: m @ v, wr, tol=1e-6)
    e = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
    say(f"  {k} iterations (oracle {info.iters}, unpreconditioned {plain.iters}); matched max rel {e:.3e}")
    assert e <= (1e-12 if dtype == torch.float64 else 1e-5)
    if dtype == torch.float64:
        assert k == info.iters
    else:
        assert abs(k - info.iters) <= 1


def test_precond_with_one_particle_groups_equals_plain_lanczos():
    """Open space, translational, groups of one particle: L = sqrt(mu_t) I, so
    the iterate and the stopping iteration are those of the unpreconditioned
    solver (with angular rows L would also scale them by sqrt(mu_r), a
    different operator)."""
    say("case precond group 1 vs plain")
    s = workloads.uniform_cube(300, 0.2, 55, w=True)
    sol = _solver(False)
    sol.setPositions(to_dev(s.pos, torch.float64))
    W = to_dev(s.w, torch.float64)
    y0 = _flat(*sol.sqrtMdotW(W, tol=1e-6))
    k0 = sol.last_iterations
    y1 = _flat(*sol.sqrtMdotWPrecond(W, groupSize=1, tol=1e-6))
    assert sol.last_iterations == k0
    assert np.abs(y1 - y0).max() <= 1e-12 * np.abs(y0).max()


@pytest.mark.parametrize("dtype", DTYPES)
def test_precond_above_a_wall(dtype):
    say(f"case precond wall {dtype}")
    s = workloads.wall_suspension(200, 61, hg=1.6, phi2d=0.4, w=True, angular_w=True)
    sol = _solver(True, "single_wall")
    sol.setPositions(to_dev(s.pos, dtype))
    lin, ang = sol.sqrtMdotWPrecond(to_dev(s.w, dtype), groupSize=25, tol=1e-6)
    k = sol.last_iterations
    xr, wr = rounded(s.pos, dtype), rounded(s.w, dtype)
    m = wall.grand_mobility_wall(xr, s.radius, s.viscosity, True)
    L = lanczos.group_cholesky(m, s.n, 25, True)
    y_ref, _ = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, wr, iters=k)
    e = float(np.abs(_flat(lin, ang) - y_ref).max() / np.abs(y_ref).max())
    say(f"  {k} iterations; matched max rel {e:.3e}")
    assert e <= (1e-12 if dtype == torch.float64 else 1e-5)


def test_precond_positions_change_rebuilds_and_errors():
    from paper_2510_02135_amd import _lib
    say("case precond rebuild / errors")
    s = workloads.c5_chains(n_chains=4, beads=30)
    sol = _solver(False)
    sol.setPositions(to_dev(s.pos, torch.float64))
    W = to_dev(np.random.default_rng(3).standard_normal(3 * s.n), torch.float64)
    y1 = _flat(*sol.sqrtMdotWPrecond(W, groupSize=30))
    x2 = s.pos + 0.3
    x2[:, 0] *= 1.05
    sol.setPositions(to_dev(x2, torch.float64))
    y2 = _flat(*sol.sqrtMdotWPrecond(W, groupSize=30))
    m = mobility.grand_mobility(x2, 1.0, workloads.VISCOSITY)
    L = lanczos.group_cholesky(m, s.n, 30)
    y_ref, _ = lanczos.preconditioned_lanczos_sqrt(lambda v: m @ v, L, host(W), iters=sol.last_iterations)
    assert np.abs(y2 - y_ref).max() <= 1e-12 * np.abs(y_ref).max()
    assert np.abs(y2 - y1).max() > 1e-3 * np.abs(y1).max()
    for bad in (0, 513):
        with pytest.raises(_lib.RpyError) as ei:
            sol.sqrtMdotWPrecond(W, groupSize=bad)
        assert ei.value.status == _lib.Status.INVALID_ARG

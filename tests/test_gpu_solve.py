"""GPU parity of the conjugate-gradient mobility solve rpy_mobility_solve
(forces and torques for prescribed velocities) through the C interface:

* against the oracle's CG run for the iteration count the library reports
  (matched iterations; float64 bar 1e-10: two CG implementations whose
  products differ in summation order drift apart by about k eps kappa), and
  against a direct solve of the oracle's dense M (10 kappa tol);
* the true residual |b - M x| / |b| with the oracle's M below 2 tol (float64)
  or 5e-5 (float32, tol 1e-5);
* a round trip F -> Mdot -> solve recovers F;
* several right-hand sides at once against one call each (translational:
  bit-identical, the products are; angular: products differ in rounding, so
  the two converged solutions differ by at most 2 kappa tol), a zero
  right-hand side, max_iter and non-finite input;
* the N = 65,536 suspension (float32, angular): the solve's residual on
  sampled rows evaluated by the oracle's pair loop.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import krylov, mobility, pairloop
from tests.gpu_util import emax, host, rounded, say, to_dev

pytestmark = pytest.mark.gpu
DTYPES = [torch.float64, torch.float32]
A, ETA = 1.0, 1 / (6 * math.pi)


def _solver(angular, a=A, eta=ETA):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver("open", "open", "open")
    s.initialize(viscosity=eta, hydrodynamicRadius=a, includeAngular=angular)
    return s


def _flat(lin, ang):
    v = host(lin).reshape(-1)
    return v if ang is None else np.concatenate([v, host(ang).reshape(-1)])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
def test_solve_against_oracle(dtype, angular):
    say(f"case CG solve angular={angular} {dtype}")
    rng = np.random.default_rng(51)
    n = 300
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.2)
    U = rng.standard_normal((n, 3))
    Om = rng.standard_normal((n, 3)) if angular else None
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    sol = _solver(angular)
    sol.setPositions(to_dev(x, dtype))
    F, T = sol.solve(to_dev(U, dtype), to_dev(Om, dtype), tol=tol)
    k, res = sol.last_iterations[0], sol.last_residual[0]
    xr = rounded(x, dtype)
    m = mobility.grand_mobility(xr, A, ETA, angular)
    b = np.concatenate([rounded(U, dtype).reshape(-1)] + ([rounded(Om, dtype).reshape(-1)] if angular else []))
    got = _flat(F, T)
    true_res = np.linalg.norm(b - m @ got) / np.linalg.norm(b)
    ref = np.linalg.solve(m, b)
    kappa = np.linalg.cond(m)
    e_direct = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  iterations {k}, reported residual {res:.2e}, true residual {true_res:.2e}, "
        f"vs direct solve {e_direct:.2e} (kappa {kappa:.1f})")
    assert res < tol
    if dtype == torch.float64:
        x_cg, _, _ = krylov.conjugate_gradients(lambda v: m @ v, b, iters=k)
        e_cg = np.linalg.norm(got - x_cg) / np.linalg.norm(x_cg)
        say(f"  matched-iteration oracle CG {e_cg:.2e}")
        assert e_cg <= 1e-10
        assert true_res <= 2 * tol
    else:
        assert true_res <= 5e-5
    assert e_direct <= 10 * kappa * max(tol, true_res)


@pytest.mark.parametrize("dtype", DTYPES)
def test_solve_round_trip(dtype):
    say(f"case CG round trip {dtype}")
    s = workloads.uniform_cube(500, 0.15, 52, torques=True)
    sol = _solver(True, s.radius, s.viscosity)
    sol.setPositions(to_dev(s.pos, dtype))
    Fd, Td = to_dev(s.forces, dtype), to_dev(s.torques, dtype)
    U, Om = sol.Mdot(Fd, Td)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    F, T = sol.solve(U, Om, tol=tol)
    e = max(emax(host(F), host(Fd)), emax(host(T), host(Td)))
    say(f"  iterations {sol.last_iterations[0]}, max rel error of F and T {e:.2e}")
    assert e <= (1e-9 if dtype == torch.float64 else 2e-4)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
def test_solve_multi_matches_single(dtype, angular):
    say(f"case CG several right-hand sides angular={angular} {dtype}")
    rng = np.random.default_rng(53)
    n = 400
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.05)
    U = rng.standard_normal((4, n, 3))
    U[2] = 0.0                                        # a zero right-hand side
    U[3] *= 1e4
    Om = rng.standard_normal((4, n, 3)) if angular else None
    if angular:
        Om[2] = 0.0
    tol = 1e-9 if dtype == torch.float64 else 1e-5
    sol = _solver(angular)
    sol.setPositions(to_dev(x, dtype))
    Ud, Omd = to_dev(U, dtype), to_dev(Om, dtype)
    F, T = sol.solve(Ud, Omd, tol=tol)
    its = list(sol.last_iterations)
    assert its[2] == 0 and not F[2].any()
    if angular:
        # two solutions with relative residuals below tol differ by at most
        # 2 kappa tol (relative): the bar for products that differ in rounding
        lam = np.linalg.eigvalsh(mobility.grand_mobility(rounded(x, dtype), A, ETA, True))
        bar = 2 * (lam[-1] / lam[0]) * tol
    for r in (0, 1, 3):
        f1, t1 = sol.solve(Ud[r], Omd[r] if angular else None, tol=tol)
        if angular:
            e = max(emax(host(F[r]), host(f1)), emax(host(T[r]), host(t1)))
            say(f"  rhs {r}: {its[r]} / {sol.last_iterations[0]} iterations, difference {e:.2e} (bar {bar:.1e})")
            assert abs(sol.last_iterations[0] - its[r]) <= 1, (r, its, sol.last_iterations)
            assert e <= bar, r
        else:
            assert sol.last_iterations[0] == its[r], (r, its, sol.last_iterations)
            assert torch.equal(F[r], f1), r
    say(f"  iterations {its}")


def test_solve_not_converged_and_errors():
    import paper_2510_02135_amd as rpy
    say("case CG edge cases")
    s = workloads.uniform_cube(200, 0.2, 54)
    sol = _solver(False)
    sol.setPositions(to_dev(s.pos, torch.float64))
    U = to_dev(s.forces, torch.float64)
    with pytest.raises(rpy.NotConvergedError) as ei:
        sol.solve(U, tol=1e-14, maxIter=2)
    assert ei.value.iters == [2]
    bad = U.clone()
    bad[3, 1] = float("inf")
    with pytest.raises(rpy.RpyError):
        sol.solve(bad)
    with pytest.raises(ValueError):
        sol.solve(U, Omega=U)                          # no angular blocks


def test_solve_full_size_sampled_residual():
    """N = 65,536 float32 with angular blocks, tol 1e-4: the residual
    b - M x on 64 sampled particles, with M x evaluated by the oracle's
    float64 pair loop from the library's x."""
    say("case CG full size N=65536 fp32 angular")
    s = workloads.c2_suspension()
    sol = _solver(True, s.radius, s.viscosity)
    sol.setPositions(to_dev(s.pos, torch.float32))
    rng = np.random.default_rng(55)
    U = rng.standard_normal((s.n, 3))
    Om = rng.standard_normal((s.n, 3))
    F, T = sol.solve(to_dev(U, torch.float32), to_dev(Om, torch.float32), tol=1e-4)
    rows = np.sort(rng.choice(s.n, 64, replace=False))
    xr = rounded(s.pos, torch.float32)
    u, w = pairloop.mdot_rows(xr, rows, host(F), host(T), s.radius, s.viscosity)
    ur, wr = rounded(U, torch.float32)[rows], rounded(Om, torch.float32)[rows]
    res = max(emax(u, ur), emax(w, wr))
    say(f"  iterations {sol.last_iterations[0]}, reported residual {sol.last_residual[0]:.2e}, "
        f"sampled-row residual {res:.2e}")
    assert res <= 5e-4

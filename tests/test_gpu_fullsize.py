"""Full-size GPU checks at the sizes the benchmark and the large workloads
use, against the float64 oracle: stored oracle results (tests/golden/,
written by make_goldens.py from ``oracle/`` only) where the oracle needs
minutes, the oracle's C pair loop on sampled rows otherwise.

* N = 65,536 suspension (phi = 0.1, torques), in the launch configuration
  the benchmark's autotuner picks there (the symmetric pair mode, one
  source block per task): the Lanczos iterate y_20 (Sec. 3.3) in float32
  and float64 pair modes against the oracle's Lanczos run for exactly 20
  iterations with pair-loop products, on 1024 sampled particles, and
  |y_20|^2 against the oracle's W^T M W; the converged float32 solve
  (tol 1e-6) against the same W^T M W (|y_k|^2 = beta_0^2 alpha_1 = W^T M W
  at every k while the basis stays orthonormal).
* 4096 chains x 256 beads (N = 1,048,576), float32 with torques: Mdot and
  the backward pass on sampled particles against the C oracle; M W on
  sampled particles and |y_12|^2 of the Lanczos iterate against the
  oracle's W^T M W from one full float64 pair-loop product.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import gradient, pairloop
from tests.golden import load as golden
from tests.gpu_util import emax, host, rounded, say

pytestmark = pytest.mark.gpu


def _solver(angular):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver()
    s.initialize(viscosity=workloads.VISCOSITY, hydrodynamicRadius=workloads.RADIUS, includeAngular=angular)
    return s


def _flat(lin, ang):
    return np.concatenate([host(lin).reshape(-1), host(ang).reshape(-1)])


def _run_k(sol, W, k):
    import paper_2510_02135_amd as rpy
    try:
        return sol.sqrtMdotW(W, tol=1e-15, maxIter=k)
    except rpy.NotConvergedError as e:
        return e.result


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_c2_lanczos_k20_against_oracle(dtype):
    s = workloads.c2_suspension()
    n = s.n
    tag = "f32" if dtype == torch.float32 else "f64"
    ref = golden.c2_lanczos(tag)
    say(f"case c2 lanczos k={ref['k']} N={n} {tag}")
    sol = _solver(True)
    sol.setPositions(torch.tensor(s.pos, dtype=dtype, device="cuda"))
    sol.setTileConfig(True, 0, 1)
    W = torch.tensor(s.w, dtype=dtype, device="cuda")
    lin, ang = _run_k(sol, W, ref["k"])
    p = ref["particles"]
    e = max(emax(host(lin)[p], ref["lin"]), emax(host(ang)[p], ref["ang"]))
    y = _flat(lin, ang)
    rn = abs(float(y @ y) / ref["wmw"] - 1.0)
    bar = 1e-5 if dtype == torch.float32 else 1e-12
    say(f"  y_20 on {len(p)} particles e_max {e:.3e}; |y_20|^2 / (W^T M W)_oracle - 1 = {rn:.2e}")
    assert e <= bar
    assert rn <= bar
    if dtype == torch.float32:
        # converged solve: the norm identity against the oracle's W^T M W
        lin, ang = sol.sqrtMdotW(W, tol=1e-6)
        y = _flat(lin, ang)
        rn = abs(float(y @ y) / ref["wmw"] - 1.0)
        say(f"  converged in {sol.last_iterations} iterations; |y|^2 / (W^T M W)_oracle - 1 = {rn:.2e}")
        assert rn <= 1e-5
    sol.close()


@pytest.mark.timeout(600)
def test_c5_chains_sampled_rows_and_lanczos_norm():
    s = workloads.c5_chains()
    n = s.n
    say(f"case c5 chains N={n}")
    f32 = torch.float32
    sol = _solver(True)
    sol.setPositions(torch.tensor(s.pos, dtype=f32, device="cuda"))
    F = torch.tensor(s.forces, dtype=f32, device="cuda")
    T = torch.tensor(s.torques, dtype=f32, device="cuda")
    lin, ang = sol.Mdot(F, T)
    rows = s.extra["subset"][:48]
    xr, fr, tr = rounded(s.pos, f32), rounded(s.forces, f32), rounded(s.torques, f32)
    u, w = pairloop.mdot_rows(xr, rows, fr, tr, s.radius, s.viscosity)
    e = max(emax(host(lin)[rows], u), emax(host(ang)[rows], w))
    say(f"  Mdot sampled e_max {e:.3e}")
    assert e <= 1e-5
    # backward with cotangents (g_U, g_W) ~ N(0, 1)
    rng = np.random.default_rng(55)
    gu, gw = rng.standard_normal((2, n, 3))
    gp, gf, gt = sol.Mdot_backward(F, T, torch.tensor(gu, dtype=f32, device="cuda"),
                                   torch.tensor(gw, dtype=f32, device="cuda"))
    gur, gwr = rounded(gu, f32), rounded(gw, f32)
    mf, mt = pairloop.mdot_rows(xr, rows[:16], gur, gwr, s.radius, s.viscosity)
    e2 = max(emax(host(gf)[rows[:16]], mf), emax(host(gt)[rows[:16]], mt))
    dx = gradient.grad_positions(xr, fr, tr, gur, gwr, s.radius, s.viscosity, rows=rows[:4], chunk=1)
    e3 = emax(host(gp)[rows[:4]], dx)
    say(f"  backward sampled dF/dT e_max {e2:.3e}, dX e_max {e3:.3e}")
    assert e2 <= 1e-5 and e3 <= 1e-5
    del gp, gf, gt
    ref = golden.c5_wmw()
    if ref is None:
        pytest.skip("tests/golden/c5_wmw.txt has not been written (make_goldens.py c5_wmw)")
    W = torch.tensor(s.w, dtype=f32, device="cuda")
    # M W on sampled particles against the oracle's full product
    ml, ma = sol.Mdot(W[:3 * n].reshape(n, 3), W[3 * n:].reshape(n, 3))
    p = ref["particles"]
    e4 = max(emax(host(ml)[p], ref["lin"]), emax(host(ma)[p], ref["ang"]))
    del ml, ma
    # Lanczos after 12 iterations: |y_k|^2 = beta0^2 alpha_1 = W^T M W while V stays orthonormal
    yl, ya = _run_k(sol, W, 12)
    y = _flat(yl, ya)
    rn = abs(float(y @ y) / ref["wmw"] - 1.0)
    say(f"  M W sampled e_max {e4:.3e}; |y_12|^2 / (W^T M W)_oracle - 1 = {rn:.2e}")
    assert e4 <= 1e-5
    assert rn <= 1e-5
    sol.close()

"""GPU parity of the symmetric pair mode (each unordered pair evaluated once
and applied in both directions; tile configuration targets_per_lane = 0,
adjoint mode 2) through the C interface: Mdot against the float64 oracle
(bars 1e-12 / 1e-5) at sizes around the 512-particle block and 64-source
chunk edges, with 1 to 3 source blocks per task, translational and
angular; agreement with the ordinary kernel; the Lanczos square root
through the same mode; the adjoint against the oracle's gradient and the
one-sided kernel; partials produced and reduced in several slabs of target
blocks (forced small by RPY_SYM_SLAB_BLOCKS) against one slab and the
oracle; sampled rows above N = 2^18; the mode checks."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import lanczos, mobility
from tests.gpu_util import emax, host, rounded, say, to_dev, tol_for

pytestmark = pytest.mark.gpu
DTYPES = [torch.float64, torch.float32]


def _solver(angular, a=1.1, eta=0.8):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver("open", "open", "open")
    s.initialize(viscosity=eta, hydrodynamicRadius=a, includeAngular=angular)
    return s


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("n,span", [(1, 0), (5, 1), (64, 0), (511, 0), (512, 1), (513, 1), (1100, 0),
                                    (1100, 1), (2047, 3), (2900, 2)])
def test_symmetric_mode_against_oracle(dtype, angular, n, span):
    say(f"case symmetric n={n} span={span} angular={angular} {dtype}")
    rng = np.random.default_rng(900 + n + span)
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.2, 1.1)    # overlapping pairs present
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3)) if angular else None
    sol = _solver(angular)
    sol.setPositions(to_dev(x, dtype))
    Fd, Td = to_dev(F, dtype), to_dev(T, dtype)
    l0, a0 = sol.Mdot(Fd, Td)
    sol.setTileConfig(angular, 0, span)
    assert sol.tileConfig(angular) == (0, span)
    l1, a1 = sol.Mdot(Fd, Td)
    xr = rounded(x, dtype)
    u, w = mobility.mdot_dense(xr, rounded(F, dtype), rounded(T, dtype) if angular else None, 1.1, 0.8)
    e = emax(host(l1), u)
    d = emax(host(l1), host(l0))
    if angular:
        e = max(e, emax(host(a1), w))
        d = max(d, emax(host(a1), host(a0)))
    say(f"  e_max vs oracle {e:.2e}, vs the ordinary kernel {d:.2e}")
    assert e <= tol_for(dtype)
    assert d <= 2 * tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_symmetric_mode_lanczos_and_repeatability(dtype):
    """sqrtMdotW through the symmetric mode against the oracle's Lanczos at the
    reported iteration count, and two products bitwise equal."""
    say(f"case symmetric Lanczos {dtype}")
    s = workloads.uniform_cube(1500, 0.15, 901, torques=True, w=True, angular_w=True)
    sol = _solver(True, s.radius, s.viscosity)
    sol.setPositions(to_dev(s.pos, dtype))
    sol.setTileConfig(True, 0, 1)
    lin, ang = sol.sqrtMdotW(to_dev(s.w, dtype), prefactor=0.9, tol=1e-6)
    k = sol.last_iterations
    xr, wr = rounded(s.pos, dtype), rounded(s.w, dtype)
    m = mobility.grand_mobility(xr, s.radius, s.viscosity, True)
    y_ref, _ = lanczos.lanczos_sqrt(lambda v: m @ v, wr, iters=k, prefactor=0.9)
    y = np.concatenate([host(lin).reshape(-1), host(ang).reshape(-1)])
    e = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
    say(f"  iterations {k}, matched-iteration max rel {e:.2e}")
    assert e <= (1e-12 if dtype == torch.float64 else 1e-5)
    F, T = to_dev(s.forces, dtype), to_dev(s.torques, dtype)
    a1, b1 = sol.Mdot(F, T)
    a2, b2 = sol.Mdot(F, T)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("slab_blocks", [1, 2])
def test_symmetric_mode_slabs(dtype, angular, slab_blocks, monkeypatch):
    """Partials of at most `slab_blocks` target blocks at a time (the running
    sums carried between slabs): forward product and adjoint against the
    oracle and against the same products in one slab."""
    from oracle import gradient
    n = 2900
    say(f"case symmetric slabs of {slab_blocks} blocks n={n} angular={angular} {dtype}")
    rng = np.random.default_rng(960 + slab_blocks)
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.2, 1.1)
    F, GU = rng.standard_normal((2, n, 3))
    T, GW = (rng.standard_normal((2, n, 3)) if angular else (None, None))
    sol = _solver(angular)
    sol.setPositions(to_dev(x, dtype))
    args = [to_dev(v, dtype) for v in (F, T, GU, GW)]
    sol.setTileConfig(angular, 0, 1)
    sol.setAdjointMode(2)
    monkeypatch.delenv("RPY_SYM_SLAB_BLOCKS", raising=False)
    one_f = sol.Mdot(args[0], args[1])
    one_b = sol.Mdot_backward(*args)
    monkeypatch.setenv("RPY_SYM_SLAB_BLOCKS", str(slab_blocks))
    many_f = sol.Mdot(args[0], args[1])
    many_b = sol.Mdot_backward(*args)
    monkeypatch.delenv("RPY_SYM_SLAB_BLOCKS")
    xr = rounded(x, dtype)
    fr, tr, gur, gwr = (rounded(v, dtype) if v is not None else None for v in (F, T, GU, GW))
    u, w = mobility.mdot_dense(xr, fr, tr, 1.1, 0.8)
    gx = gradient.grad_positions(xr, fr, tr, gur, gwr, 1.1, 0.8)
    mg_u, mg_w = mobility.mdot_dense(xr, gur, gwr, 1.1, 0.8)
    e = max(emax(host(many_f[0]), u), emax(host(many_b[0]), gx), emax(host(many_b[1]), mg_u))
    d = max(emax(host(many_f[0]), host(one_f[0])), emax(host(many_b[0]), host(one_b[0])),
            emax(host(many_b[1]), host(one_b[1])))
    if angular:
        e = max(e, emax(host(many_f[1]), w), emax(host(many_b[2]), mg_w))
        d = max(d, emax(host(many_f[1]), host(one_f[1])), emax(host(many_b[2]), host(one_b[2])))
    say(f"  e_max vs oracle {e:.2e}, vs one slab {d:.2e}")
    assert e <= tol_for(dtype)
    assert d <= 2 * tol_for(dtype)


def test_symmetric_mode_above_2_18_sampled_rows():
    """N = 2^18 + 1 (float32, translational) through the symmetric forward
    product and the symmetric adjoint, whose partials exceed one slab's
    workspace here: sampled rows against the oracle."""
    from oracle import gradient, pairloop
    n = (1 << 18) + 1
    say(f"case symmetric mode n={n}")
    rng = np.random.default_rng(970)
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.1)
    F, GU = rng.standard_normal((2, n, 3))
    f32 = torch.float32
    sol = _solver(False, 1.0, 1.0 / (6 * math.pi))
    sol.setPositions(to_dev(x, f32))
    sol.setTileConfig(False, 0, 0)
    sol.setAdjointMode(2)
    lin, _ = sol.Mdot(to_dev(F, f32))
    gp, gf, _ = sol.Mdot_backward(to_dev(F, f32), None, to_dev(GU, f32), None)
    rows = np.sort(rng.choice(n, 16, replace=False))
    xr, fr, gr = rounded(x, f32), rounded(F, f32), rounded(GU, f32)
    u, _ = pairloop.mdot_rows(xr, rows, fr, None, 1.0, 1.0 / (6 * math.pi))
    mg, _ = pairloop.mdot_rows(xr, rows, gr, None, 1.0, 1.0 / (6 * math.pi))
    dx = gradient.grad_positions(xr, fr, None, gr, None, 1.0, 1.0 / (6 * math.pi), rows=rows[:4], chunk=1)
    e = max(emax(host(lin)[rows], u), emax(host(gf)[rows], mg), emax(host(gp)[rows[:4]], dx))
    say(f"  sampled e_max {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("n", [7, 300, 700, 1300])
def test_symmetric_adjoint_against_oracle(dtype, angular, n):
    """Mdot_backward in the symmetric mode (each unordered pair once, its
    position-gradient term added to one particle and subtracted from the
    other) against the oracle's analytic gradient and M g, and against the
    one-sided kernel."""
    from oracle import gradient
    say(f"case symmetric adjoint n={n} angular={angular} {dtype}")
    rng = np.random.default_rng(950 + n)
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.25)
    F, GU = rng.standard_normal((2, n, 3))
    T, GW = (rng.standard_normal((2, n, 3)) if angular else (None, None))
    sol = _solver(angular, 1.2, 0.9)
    sol.setPositions(to_dev(x, dtype))
    args = [to_dev(v, dtype) for v in (F, T, GU, GW)]
    sol.setAdjointMode(1)
    one = sol.Mdot_backward(*args)
    sol.setAdjointMode(2)
    sym = sol.Mdot_backward(*args)
    xr = rounded(x, dtype)
    fr, tr, gur, gwr = (rounded(v, dtype) if v is not None else None for v in (F, T, GU, GW))
    gx = gradient.grad_positions(xr, fr, tr, gur, gwr, 1.2, 0.9)
    mg_u, mg_w = mobility.mdot_dense(xr, gur, gwr, 1.2, 0.9)
    e = max(emax(host(sym[0]), gx), emax(host(sym[1]), mg_u))
    d = max(emax(host(sym[0]), host(one[0])), emax(host(sym[1]), host(one[1])))
    if angular:
        e = max(e, emax(host(sym[2]), mg_w))
        d = max(d, emax(host(sym[2]), host(one[2])))
    say(f"  e_max vs oracle {e:.2e}, vs the one-sided kernel {d:.2e}")
    assert e <= tol_for(dtype)
    assert d <= 2 * tol_for(dtype)


def test_adjoint_mode_checks():
    import paper_2510_02135_amd as rpy
    say("case adjoint mode checks")
    sol = _solver(False)
    for bad in (-1, 3):
        with pytest.raises(rpy.RpyError):
            sol.setAdjointMode(bad)

"""GPU parity of Mdot and divM against the float64 oracle (through the C
interface).  float32 runs are compared with the oracle evaluated on the same
float32-rounded inputs; bars: 1e-12 (float64) and 1e-5 (float32) in
e_max = max_i |dU_i| / max_i |U_ref,i|."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import mobility, pairloop
from tests.gpu_util import emax, host, rounded, say, to_dev, tol_for

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


def _solver(angular, a=1.0, eta=1 / (6 * math.pi)):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver("open", "open", "open")
    s.initialize(viscosity=eta, hydrodynamicRadius=a, includeAngular=angular)
    return s


def _check(sol, x, F, T, dtype, a, eta, want_ang):
    xr, Fr = rounded(x, dtype), rounded(F, dtype)
    Tr = rounded(T, dtype) if T is not None else (np.zeros_like(xr) if want_ang else None)
    sol.setPositions(to_dev(x, dtype))
    lin, ang = sol.Mdot(forces=to_dev(F, dtype), torques=to_dev(T, dtype))
    torch.cuda.synchronize()
    u_ref, w_ref = mobility.mdot_dense(xr, Fr, Tr, a, eta)
    e = emax(host(lin), u_ref)
    if want_ang:
        e = max(e, emax(host(ang), w_ref))
    return e


def test_c1_float64_translational():
    s = workloads.c1_small_fp64()
    say("case c1 N=1024 fp64 linear")
    sol = _solver(False)
    e = _check(sol, s.pos, s.forces, None, torch.float64, s.radius, s.viscosity, False)
    say(f"  e_max {e:.3e}")
    assert e <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 63, 255, 256, 257, 511, 700, 1100])
def test_small_sizes_and_ragged_tails(dtype, angular, n):
    say(f"case random n={n} angular={angular} {dtype}")
    rng = np.random.default_rng(100 + n)
    side = workloads.cube_side(n, 0.15)
    x = (rng.random((n, 3)) - 0.5) * side
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3)) if angular else None
    a, eta = 1.3, 0.9
    sol = _solver(angular, a, eta)
    e = _check(sol, x, F, T, dtype, a, eta, angular)
    say(f"  e_max {e:.3e}")
    assert e <= tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_torque_only_and_force_only_with_angular_output(dtype):
    say(f"case torque-only / force-only {dtype}")
    rng = np.random.default_rng(5)
    n = 300
    x = (rng.random((n, 3)) - 0.5) * 12
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3))
    sol = _solver(True)
    a, eta = 1.0, 1 / (6 * math.pi)
    xr = rounded(x, dtype)
    sol.setPositions(to_dev(x, dtype))
    lin, ang = sol.Mdot(torques=to_dev(T, dtype))
    u, w = mobility.mdot_dense(xr, None, rounded(T, dtype), a, eta)
    assert max(emax(host(lin), u), emax(host(ang), w)) <= tol_for(dtype)
    lin, ang = sol.Mdot(forces=to_dev(F, dtype))
    u, w = mobility.mdot_dense(xr, rounded(F, dtype), np.zeros_like(xr), a, eta)
    assert max(emax(host(lin), u), emax(host(ang), w)) <= tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_degenerate_geometries(dtype):
    """Coincident particles, pairs exactly at contact and 1 ulp either side,
    and a pair far apart (self-mobility limit)."""
    say(f"case degenerate geometries {dtype}")
    a, eta = 1.0, 1 / (6 * math.pi)
    np_t = np.float32 if dtype == torch.float32 else np.float64
    two = np_t(2.0)
    x = np.array([[0, 0, 0], [0, 0, 0],                                   # coincident
                  [0, 20, 0], [float(two), 20, 0],                        # exactly 2a
                  [0, 40, 0], [float(np.nextafter(two, np_t(0))), 40, 0],  # 1 ulp inside
                  [0, 60, 0], [float(np.nextafter(two, np_t(9))), 60, 0],  # 1 ulp outside
                  [1e5, 0, 0], [-1e5, 3, 4]], dtype=np.float64)
    rng = np.random.default_rng(6)
    F = rng.standard_normal(x.shape)
    T = rng.standard_normal(x.shape)
    sol = _solver(True, a, eta)
    e = _check(sol, x, F, T, dtype, a, eta, True)
    say(f"  e_max {e:.3e}")
    assert e <= tol_for(dtype)


def test_div_m_is_zero_and_outputs_are_overwritten():
    say("case divM")
    sol = _solver(True)
    x = np.random.default_rng(1).random((50, 3)) * 5
    sol.setPositions(to_dev(x, torch.float32))
    lin, ang = sol.divM()
    assert not lin.any() and not ang.any() and lin.shape == (50, 3)


@pytest.mark.parametrize("dtype", DTYPES)
def test_repeated_calls_are_bitwise_deterministic(dtype):
    say(f"case determinism {dtype}")
    s = workloads.uniform_cube(3000, 0.1, 77, torques=True)
    sol = _solver(True)
    sol.setPositions(to_dev(s.pos, dtype))
    F, T = to_dev(s.forces, dtype), to_dev(s.torques, dtype)
    a1, b1 = sol.Mdot(F, T)
    a2, b2 = sol.Mdot(F, T)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


@pytest.mark.parametrize("dtype", DTYPES)
def test_c2_full_size_sampled_rows(dtype):
    """N = 65,536 at volume fraction 0.1 with the default tiles and in the
    launch configuration the benchmark's autotuner picks at this size (the
    symmetric mode, one source block per task); the oracle evaluates 512
    sampled target rows."""
    s = workloads.c2_suspension()
    rows = s.extra["subset"][::8]
    xr, Fr = rounded(s.pos, dtype), rounded(s.forces, dtype)
    for cfg in (None, (0, 1)):
        say(f"case c2 N={s.n} {dtype} rows={len(rows)} tiles={cfg or 'default'}")
        sol = _solver(True)
        sol.setPositions(to_dev(s.pos, dtype))
        if cfg:
            sol.setTileConfig(True, *cfg)
            sol.setTileConfig(False, *cfg)
        for torques in (None, s.torques):
            lin, ang = sol.Mdot(forces=to_dev(s.forces, dtype), torques=to_dev(torques, dtype))
            Tr = rounded(torques, dtype) if torques is not None else np.zeros_like(xr)
            u, w = pairloop.mdot_rows(xr, rows, Fr, Tr, s.radius, s.viscosity)
            e = max(emax(host(lin)[rows], u), emax(host(ang)[rows], w))
            say(f"  torques={torques is not None} e_max {e:.3e}")
            assert e <= tol_for(dtype)
        # translational-only solver
        sol2 = _solver(False)
        sol2.setPositions(to_dev(s.pos, dtype))
        if cfg:
            sol2.setTileConfig(False, *cfg)
        lin, _ = sol2.Mdot(forces=to_dev(s.forces, dtype))
        u, _ = pairloop.mdot_rows(xr, rows, Fr, None, s.radius, s.viscosity)
        e = emax(host(lin)[rows], u)
        say(f"  linear-only e_max {e:.3e}")
        assert e <= tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_every_tile_config_and_autotune_keep_parity(dtype, tmp_path):
    """Results stay within the parity bar for every tile configuration the
    autotuner may pick; the tuner's cache file round-trips."""
    import paper_2510_02135_amd as rpy
    say(f"case tile configs / autotune {dtype}")
    s = workloads.uniform_cube(1500, 0.1, 55, torques=True)
    xr, Fr, Tr = rounded(s.pos, dtype), rounded(s.forces, dtype), rounded(s.torques, dtype)
    u_ref, w_ref = pairloop.mdot(xr, Fr, Tr, s.radius, s.viscosity)
    u_lin, _ = pairloop.mdot(xr, Fr, None, s.radius, s.viscosity)
    sol = _solver(True)
    sol.setPositions(to_dev(s.pos, dtype))
    F, T = to_dev(s.forces, dtype), to_dev(s.torques, dtype)
    sol_lin = _solver(False)
    sol_lin.setPositions(to_dev(s.pos, dtype))
    for tm in (1, 2, 3, 4):
        for sp in ((0,) if tm == 3 else (0, 1, 3, 6)):
            sol.setTileConfig(True, tm, sp)
            lin, ang = sol.Mdot(F, T)
            assert max(emax(host(lin), u_ref), emax(host(ang), w_ref)) <= tol_for(dtype), (tm, sp)
            sol_lin.setTileConfig(False, tm, sp)
            lin, _ = sol_lin.Mdot(F)
            assert emax(host(lin), u_lin) <= tol_for(dtype), (tm, sp)
    cache = tmp_path / "tiles.txt"
    cfg_lin, cfg_ang = sol.autotune(str(cache))
    lines = cache.read_text().strip().splitlines()
    say(f"  tuned lin {cfg_lin} ang {cfg_ang}; cache {lines}")
    assert len(lines) == 2
    for cfg in (cfg_lin, cfg_ang):           # a split count, or the fused kernel (no splits)
        assert cfg[1] >= 1 or cfg[0] == 3
    lin, ang = sol.Mdot(F, T)
    assert max(emax(host(lin), u_ref), emax(host(ang), w_ref)) <= tol_for(dtype)
    other = _solver(True)
    other.setPositions(to_dev(s.pos, dtype))
    assert other.autotune(str(cache)) == (cfg_lin, cfg_ang)
    for bad in (5, -1):
        with pytest.raises(rpy.RpyError):
            sol.setTileConfig(False, bad, 0)


def test_untuned_default_and_untimed_choice_above_2_18(tmp_path):
    """An untouched configuration reports two targets per lane below
    N = 32768 and the symmetric mode from there on, and its products are
    those of that mode bit for bit; above N = 2^18 the autotuner takes the
    symmetric mode without timing anything (no cache line is written)."""
    say("case untuned default / untimed choice above 2^18")
    for n, want in ((32767, (2, 0)), (32768, (0, 0))):
        s = workloads.uniform_cube(n, 0.1, 57, torques=True)
        sol = _solver(True)
        sol.setPositions(to_dev(s.pos, torch.float32))
        assert sol.tileConfig(False) == want and sol.tileConfig(True) == want, n
        F, T = to_dev(s.forces, torch.float32), to_dev(s.torques, torch.float32)
        lin0, ang0 = sol.Mdot(F, T)
        sol.setTileConfig(True, *want)
        lin1, ang1 = sol.Mdot(F, T)
        assert torch.equal(lin0, lin1) and torch.equal(ang0, ang1), n
    big = _solver(True)
    big.setPositions(to_dev(workloads.uniform_cube((1 << 18) + 1, 0.1, 58).pos, torch.float32))
    cache = tmp_path / "tiles.txt"
    assert big.autotune(str(cache)) == ((0, 0), (0, 0))
    assert not cache.exists() or not cache.read_text().strip()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 63, 64, 65, 1000, 4097])
def test_fused_small_n_kernel(dtype, angular, n):
    """Tile mode 3 (one launch reading the caller's arrays): every size from
    one particle through partial workgroups and uneven source sixteenths."""
    say(f"case fused n={n} angular={angular} {dtype}")
    rng = np.random.default_rng(700 + n)
    x = (rng.random((n, 3)) - 0.5) * workloads.cube_side(n, 0.2)
    F = rng.standard_normal((n, 3))
    T = rng.standard_normal((n, 3)) if angular else None
    a, eta = 1.1, 0.7
    sol = _solver(angular, a, eta)
    sol.setTileConfig(angular, 3, 0)
    e = _check(sol, x, F, T, dtype, a, eta, angular)
    say(f"  e_max {e:.3e}")
    assert e <= tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fused_kernel_lanczos_torque_only_and_missing_angular_output(dtype):
    from oracle import lanczos
    from paper_2510_02135_amd import _lib
    say(f"case fused lanczos / torque only {dtype}")
    s = workloads.uniform_cube(400, 0.15, 78, torques=True, w=True, angular_w=True)
    sol = _solver(True)
    sol.setTileConfig(True, 3, 0)
    sol.setTileConfig(False, 3, 0)
    sol.setPositions(to_dev(s.pos, dtype))
    xr, wr = rounded(s.pos, dtype), rounded(s.w, dtype)
    lin, ang = sol.sqrtMdotW(to_dev(s.w, dtype), tol=1e-6)
    k = sol.last_iterations
    m = mobility.grand_mobility(xr, s.radius, s.viscosity, True)
    y_ref, _ = lanczos.lanczos_sqrt(lambda v: m @ v, wr, iters=k)
    y = np.concatenate([host(lin).reshape(-1), host(ang).reshape(-1)])
    e = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
    say(f"  lanczos {k} iterations, matched max rel {e:.3e}")
    assert e <= (1e-12 if dtype == torch.float64 else 1e-5)
    # torques with no angular output through the C call: linear rows only
    T = to_dev(s.torques, dtype)
    out = torch.empty((s.n, 3), dtype=dtype, device="cuda")
    _lib.rpy_mdot(sol._h, None, T, out, None, dtype, s.n)
    u, _ = mobility.mdot_dense(xr, None, rounded(s.torques, dtype), s.radius, s.viscosity)
    assert emax(host(out), u) <= tol_for(dtype)
    # fixed summation order: repeated calls agree bit for bit
    assert torch.equal(sol.Mdot(None, T)[0], sol.Mdot(None, T)[0])


def test_error_paths_through_the_binding():
    """Status codes of the C interface surface as exceptions: non-finite
    positions (nothing stored), dtype mismatch, torques without the angular
    blocks, missing inputs."""
    import paper_2510_02135_amd as rpy
    say("case error paths")
    sol = _solver(False)
    x = np.random.default_rng(3).random((20, 3)) * 5
    bad = x.copy()
    bad[4, 1] = np.inf
    with pytest.raises(rpy.RpyError) as ei:
        sol.setPositions(to_dev(bad, torch.float64))
    assert ei.value.status == rpy.Status.NONFINITE
    with pytest.raises(rpy.RpyError) as ei:
        sol.Mdot(forces=to_dev(x, torch.float64))
    assert ei.value.status == rpy.Status.NO_POSITIONS
    sol.setPositions(to_dev(x, torch.float64))
    with pytest.raises(ValueError):
        sol.Mdot(forces=to_dev(x, torch.float32))
    with pytest.raises(rpy.RpyError) as ei:
        sol.Mdot(forces=to_dev(x, torch.float64), torques=to_dev(x, torch.float64))
    assert ei.value.status == rpy.Status.ANGULAR_DISABLED
    with pytest.raises(rpy.RpyError) as ei:
        sol.Mdot()
    assert ei.value.status == rpy.Status.INVALID_ARG
    with pytest.raises(rpy.RpyError) as ei:
        rpy.Solver("open", "open", "two_walls")
    assert ei.value.status == rpy.Status.UNSUPPORTED_GEOMETRY
    with pytest.raises(rpy.RpyError):
        sol.setParameters(wallHeight=0.0)

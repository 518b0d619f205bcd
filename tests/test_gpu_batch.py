"""GPU parity of the batched solver (many independent systems in one
launch: the block mode, each system's unordered pairs once, and the
one-sided persistent kernel; Lanczos replayed from captured HIP graphs)
against the float64 oracle, per system, through the C interface; with and
without angular blocks."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import lanczos, mobility, pairloop
from tests.gpu_util import emax, host, rounded, say, tol_for

pytestmark = pytest.mark.gpu
DTYPES = [torch.float64, torch.float32]


def _systems(sizes, seed, phi=0.15):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        side = workloads.cube_side(n, phi)
        x = (rng.random((n, 3)) - 0.5) * side
        out.append((x, rng.standard_normal((n, 3)), rng.standard_normal(3 * n)))
    return out


def _batch(systems, dtype, eta=None, radius=None, angular=False, tm=None):
    import paper_2510_02135_amd as rpy
    ns = [len(s[0]) for s in systems]
    off = np.concatenate([[0], np.cumsum(ns)])
    eta = np.full(len(ns), 1 / (6 * math.pi)) if eta is None else eta
    radius = np.ones(len(ns)) if radius is None else radius
    b = rpy.Batch(off, eta, radius, dtype, includeAngular=angular)
    if tm is not None:
        b.setTileConfig(tm, 8)
    pos = torch.tensor(np.concatenate([s[0] for s in systems]), dtype=dtype, device="cuda")
    b.setPositions(pos)
    return b, off


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("tm", [0, 1])
def test_batched_mdot_per_system(dtype, tm):
    sizes = [1, 2, 3, 64, 65, 130, 257, 300, 17, 511, 512, 513, 1100, 1600]
    say(f"case batch mdot sizes={sizes} tm={tm} {dtype}")
    systems = _systems(sizes, 11)
    eta = np.linspace(0.5, 1.5, len(sizes))
    rad = np.linspace(0.7, 1.4, len(sizes))
    b, off = _batch(systems, dtype, eta, rad, tm=tm)
    F = torch.tensor(np.concatenate([s[1] for s in systems]), dtype=dtype, device="cuda")
    U = host(b.Mdot(F))
    worst = 0.0
    for k, (x, f, _) in enumerate(systems):
        u_ref, _ = mobility.mdot_dense(rounded(x, dtype), rounded(f, dtype), None, rad[k], eta[k])
        e = emax(U[off[k]:off[k + 1]], u_ref)
        worst = max(worst, e)
    say(f"  worst system e_max {worst:.3e}")
    assert worst <= tol_for(dtype)
    # deterministic: a repeated product is bitwise equal
    np.testing.assert_array_equal(U, host(b.Mdot(F)))


@pytest.mark.parametrize("dtype", DTYPES)
def test_batched_angular_mdot_per_system(dtype):
    sizes = [1, 2, 70, 300, 511, 513, 1030, 40]
    say(f"case batch angular mdot sizes={sizes} {dtype}")
    systems = _systems(sizes, 21, phi=0.2)
    rng = np.random.default_rng(22)
    eta = np.linspace(0.6, 1.3, len(sizes))
    rad = np.linspace(0.8, 1.2, len(sizes))
    b, off = _batch(systems, dtype, eta, rad, angular=True)
    F = np.concatenate([s[1] for s in systems])
    T = rng.standard_normal(F.shape)
    t = lambda v: torch.tensor(v, dtype=dtype, device="cuda")
    U, Om = (host(v) for v in b.Mdot(t(F), t(T)))
    Ut, Omt = (host(v) for v in b.Mdot(None, t(T)))
    worst = 0.0
    for k, (x, f, _) in enumerate(systems):
        sl = slice(off[k], off[k + 1])
        xr, fr, tr = rounded(x, dtype), rounded(f, dtype), rounded(T[sl], dtype)
        u_ref, w_ref = mobility.mdot_dense(xr, fr, tr, rad[k], eta[k])
        ut_ref, wt_ref = mobility.mdot_dense(xr, None, tr, rad[k], eta[k])
        worst = max(worst, emax(U[sl], u_ref), emax(Om[sl], w_ref), emax(Ut[sl], ut_ref), emax(Omt[sl], wt_ref))
    say(f"  worst system e_max {worst:.3e}")
    assert worst <= tol_for(dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_batched_mdot_every_tile_config_and_autotune(dtype):
    """Every (targets per lane, workgroups per CU) of the batched pair kernel,
    and the autotuner's choice, against the oracle per system; bad
    configurations are rejected."""
    import paper_2510_02135_amd as rpy
    sizes = [1, 63, 64, 65, 127, 128, 129, 300, 2, 511]
    say(f"case batch tile configs sizes={sizes} {dtype}")
    systems = _systems(sizes, 14)
    b, off = _batch(systems, dtype)
    F = torch.tensor(np.concatenate([s[1] for s in systems]), dtype=dtype, device="cuda")
    refs = [mobility.mdot_dense(rounded(x, dtype), rounded(f, dtype), None, 1.0, 1 / (6 * math.pi))[0]
            for x, f, _ in systems]

    def check(tag):
        U = host(b.Mdot(F))
        worst = max(emax(U[off[k]:off[k + 1]], refs[k]) for k in range(len(systems)))
        say(f"  {tag}: worst system e_max {worst:.3e}")
        assert worst <= tol_for(dtype)

    for tm in (0, 1, 2):
        for wg in (1, 4, 16, 32):
            b.setTileConfig(tm, wg)
            assert b.tileConfig() == (tm, wg)
            check(f"tm={tm} wg={wg}")
    chosen = b.autotune()
    assert chosen[0] in (0, 1, 2) and chosen[1] in (4, 8, 16)
    check(f"autotuned {chosen}")
    for bad in ((-1, 8), (3, 8), (1, 0), (1, 33)):
        with pytest.raises(rpy.RpyError):
            b.setTileConfig(*bad)
    assert b.tileConfig() == chosen


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("tm", [0, 1])
def test_batched_lanczos_matched_iterations_and_eager_replay(dtype, tm, monkeypatch):
    """Each system stops where the oracle's Lanczos stops (float64; float32
    within one iteration, since float32 products can move an increment that
    lies within rounding of tol), matches the oracle's Lanczos at the
    iteration count the batch reports, and the eager single-system solver
    stopped at that iteration (every replay of the captured graph
    contributes).  The host poll interval changes nothing; the exact test at
    every iteration changes nothing but the rounding of s_k."""
    import paper_2510_02135_amd as rpy
    sizes = [1, 5, 40, 97, 200, 333, 600]
    say(f"case batch lanczos sizes={sizes} tm={tm} {dtype}")
    systems = _systems(sizes, 12, phi=0.2)
    b, off = _batch(systems, dtype, tm=tm)
    W = torch.tensor(np.concatenate([s[2] for s in systems]), dtype=dtype, device="cuda")
    Y = host(b.sqrtMdotW(W, prefactor=0.7, tol=1e-6, checkEvery=3)).reshape(-1)
    iters = list(b.last_iterations)
    say(f"  iterations {iters}")
    Y1 = host(b.sqrtMdotW(W, prefactor=0.7, tol=1e-6, checkEvery=1)).reshape(-1)
    assert list(b.last_iterations) == iters
    np.testing.assert_array_equal(Y, Y1)
    monkeypatch.setenv("RPY_LANCZOS_CHECK", "every")
    Ye = host(b.sqrtMdotW(W, prefactor=0.7, tol=1e-6, checkEvery=5)).reshape(-1)
    monkeypatch.delenv("RPY_LANCZOS_CHECK")
    assert list(b.last_iterations) == iters
    # the default takes s_k from the quadrature estimate (exact to rounding),
    # the every-iteration test from the eigensolver
    scale = np.abs(Ye).max()
    assert np.abs(Y - Ye).max() <= (1e-13 if dtype == torch.float64 else 4 * 2.0 ** -24) * scale
    a, eta = 1.0, 1 / (6 * math.pi)
    for k, (x, f, w) in enumerate(systems):
        xr, wr = rounded(x, dtype), rounded(w, dtype)
        m = mobility.grand_mobility(xr, a, eta)
        _, info = lanczos.lanczos_sqrt(lambda v: m @ v, wr, tol=1e-6)
        say(f"  system {k}: N={len(x)} oracle stops at {info.iters}, batch at {iters[k]}")
        if dtype == torch.float64:
            assert iters[k] == info.iters
        else:
            assert abs(iters[k] - info.iters) <= 1
        y_ref, _ = lanczos.lanczos_sqrt(lambda v: m @ v, wr, iters=iters[k], prefactor=0.7)
        y = Y[3 * off[k]:3 * off[k + 1]]
        e = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
        assert e <= (1e-12 if dtype == torch.float64 else 1e-5), (k, e)
        exact = lanczos.exact_sqrt_mdot_w(m, wr, 0.7)
        assert np.linalg.norm(y - exact) / np.linalg.norm(exact) <= 1e-5
        # eager single-system solver stopped at the same iteration
        sol = rpy.Solver()
        sol.initialize(viscosity=eta, hydrodynamicRadius=a)
        sol.setPositions(torch.tensor(x, dtype=dtype, device="cuda"))
        try:
            lin, _ = sol.sqrtMdotW(torch.tensor(w, dtype=dtype, device="cuda"), prefactor=0.7, tol=1e-15,
                                   maxIter=iters[k])
        except rpy.NotConvergedError as err:
            lin = err.result[0]
        ye = host(lin).reshape(-1)
        e2 = float(np.abs(y - ye).max() / np.abs(ye).max())
        assert e2 <= (1e-12 if dtype == torch.float64 else 1e-5), (k, e2)


def test_batched_repeated_calls_zero_noise_and_errors():
    import paper_2510_02135_amd as rpy
    say("case batch repeated / edge cases")
    systems = _systems([30, 80, 12], 13)
    b, off = _batch(systems, torch.float64)
    rng = np.random.default_rng(1)
    W1 = rng.standard_normal(3 * off[-1])
    W2 = rng.standard_normal(3 * off[-1])
    W2[3 * off[1]:3 * off[2]] = 0.0            # second system: zero noise -> zero output
    t = lambda v: torch.tensor(v, dtype=torch.float64, device="cuda")
    Y1 = host(b.sqrtMdotW(t(W1))).reshape(-1)
    Y2 = host(b.sqrtMdotW(t(W2))).reshape(-1)
    it2 = list(b.last_iterations)
    Y1b = host(b.sqrtMdotW(t(W1))).reshape(-1)
    np.testing.assert_array_equal(Y1, Y1b)
    assert not Y2[3 * off[1]:3 * off[2]].any()
    assert it2[1] == 0 and it2[0] > 0 and it2[2] > 0
    for k in (0, 2):
        x = systems[k][0]
        m = mobility.grand_mobility(x, 1.0, 1 / (6 * math.pi))
        y_ref, _ = lanczos.lanczos_sqrt(lambda v: m @ v, W2[3 * off[k]:3 * off[k + 1]], iters=it2[k])
        assert np.abs(Y2[3 * off[k]:3 * off[k + 1]] - y_ref).max() <= 1e-12 * np.abs(y_ref).max()
    with pytest.raises(rpy.NotConvergedError):
        b.sqrtMdotW(t(W1), tol=1e-14, maxIter=4, checkEvery=2)
    bad = W1.copy()
    bad[7] = np.nan
    with pytest.raises(rpy.RpyError):
        b.sqrtMdotW(t(bad))
    with pytest.raises(rpy.RpyError):
        rpy.Batch([0, 5, 5], [1.0, 1.0], [1.0, 1.0])          # empty system


def test_c4_512_systems_sampled():
    """The 512-system workload (N log-uniform in [64, 8192], phi in
    [0.05, 0.3]): batched Mdot on sampled rows of sampled systems against the
    C oracle, and batched Lanczos on sampled systems against the oracle's
    Lanczos (pair-loop products) at the reported iteration count."""
    import paper_2510_02135_amd as rpy
    syss = workloads.c4_systems()
    ns = np.array([s.n for s in syss])
    off = np.concatenate([[0], np.cumsum(ns)])
    say(f"case c4 systems={len(syss)} total={off[-1]} sum N^2={float((ns ** 2).sum()):.3e}")
    dt = torch.float32
    b = rpy.Batch(off, 1 / (6 * math.pi), 1.0, dt)
    b.setPositions(torch.tensor(np.concatenate([s.pos for s in syss]), dtype=dt, device="cuda"))
    F = np.concatenate([s.forces for s in syss])
    W = np.concatenate([s.w for s in syss])
    U = host(b.Mdot(torch.tensor(F, dtype=dt, device="cuda")))
    Y = host(b.sqrtMdotW(torch.tensor(W, dtype=dt, device="cuda"), tol=1e-6)).reshape(-1)
    iters = np.array(b.last_iterations)
    say(f"  iterations min {iters.min()} median {int(np.median(iters))} max {iters.max()}")
    pick = [int(np.argmin(ns)), int(np.argmax(ns)), 5, 77, 300]
    for k in pick:
        s = syss[k]
        xr = rounded(s.pos, dt)
        rows = np.arange(0, s.n, max(1, s.n // 64))
        u, _ = pairloop.mdot_rows(xr, rows, rounded(s.forces, dt), None, s.radius, s.viscosity)
        e = emax(U[off[k]:off[k + 1]][rows], u)
        assert e <= 1e-5, (k, e)
        if s.n <= 3000:
            wr = rounded(s.w, dt)
            mv = lambda v: pairloop.mdot(xr, v.reshape(-1, 3), None, s.radius, s.viscosity)[0].reshape(-1)
            y_ref, _ = lanczos.lanczos_sqrt(mv, wr, iters=int(iters[k]))
            _, info = lanczos.lanczos_sqrt(mv, wr, tol=1e-6)
            y = Y[3 * off[k]:3 * off[k + 1]]
            e2 = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
            say(f"  system {k} N={s.n} it={iters[k]} (oracle stops at {info.iters}) mdot {e:.2e} lanczos {e2:.2e}")
            assert e2 <= 1e-5
            assert abs(int(iters[k]) - info.iters) <= 1


@pytest.mark.parametrize("dtype", DTYPES)
def test_batched_angular_lanczos_matched_iterations(dtype):
    """With angular blocks each system's noise vector holds its 3 n_s linear
    entries, then its 3 n_s angular ones; each system stops where the
    oracle's Lanczos on its 6 n_s x 6 n_s grand mobility stops and matches
    it at that iteration."""
    sizes = [3, 60, 250, 520]
    say(f"case batch angular lanczos sizes={sizes} {dtype}")
    systems = _systems(sizes, 31, phi=0.2)
    b, off = _batch(systems, dtype, angular=True)
    rng = np.random.default_rng(32)
    Ws = [rng.standard_normal(6 * len(x)) for x, _, _ in systems]
    W = torch.tensor(np.concatenate(Ws), dtype=dtype, device="cuda")
    lin, ang = b.sqrtMdotW(W, prefactor=0.5, tol=1e-6, checkEvery=2)
    lin, ang = host(lin), host(ang)
    iters = list(b.last_iterations)
    say(f"  iterations {iters}")
    a, eta = 1.0, 1 / (6 * math.pi)
    for k, (x, _, _) in enumerate(systems):
        xr, wr = rounded(x, dtype), rounded(Ws[k], dtype)
        m = mobility.grand_mobility(xr, a, eta, angular=True)
        _, info = lanczos.lanczos_sqrt(lambda v: m @ v, wr, tol=1e-6)
        if dtype == torch.float64:
            assert iters[k] == info.iters
        else:
            assert abs(iters[k] - info.iters) <= 1
        y_ref, _ = lanczos.lanczos_sqrt(lambda v: m @ v, wr, iters=iters[k], prefactor=0.5)
        sl = slice(off[k], off[k + 1])
        y = np.concatenate([lin[sl].reshape(-1), ang[sl].reshape(-1)])
        e = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
        say(f"  system {k}: N={len(x)} it={iters[k]} (oracle {info.iters}) max rel {e:.2e}")
        assert e <= (1e-12 if dtype == torch.float64 else 1e-5)

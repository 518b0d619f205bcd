"""GPU parity of the random-finite-difference drift (eq. (rfd), Sec. 3.4)
against the float64 oracle, and the open-space invariant d_X . M = 0 checked
by averaging random finite differences on the 16,384-particle workload
(phi = 0.2), through the C interface.

Tolerance of one sample: each of the two products M(X +- delta/2 W_X) W is
held to the Mdot bar (e_max 1e-12 in float64, 1e-5 in float32, relative to
the largest particle norm of the product); their difference divided by delta
inherits 2 x bar x max|M W| / delta as an absolute bound.  The float32 side
sees W rounded to float32 and displaced positions formed in float64 and
rounded once to float32; the oracle is evaluated on exactly those values.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import drift, mobility, pairloop
from tests.gpu_util import host, rounded, say, tol_for

pytestmark = pytest.mark.gpu
DTYPES = [torch.float64, torch.float32]


def _solver(angular):
    import paper_2510_02135_amd as rpy
    s = rpy.Solver()
    s.initialize(viscosity=workloads.VISCOSITY, hydrodynamicRadius=workloads.RADIUS, includeAngular=angular)
    return s


def _round_fn(dtype):
    if dtype == torch.float32:
        return lambda v: v.astype(np.float32).astype(np.float64)
    return None


def _bound(dtype, xr, w, delta, angular, rf):
    """2 x bar x max particle norm of M(X +- delta/2 W_X) W, divided by delta."""
    n = xr.shape[0]
    wp = w[:3 * n].reshape(n, 3)
    wt = w[3 * n:].reshape(n, 3) if angular else None
    big = 0.0
    for sgn in (1.0, -1.0):
        xd = xr + sgn * 0.5 * delta * wp
        if rf is not None:
            xd = rf(xd)
        u, om = mobility.mdot_dense(xd, wp, wt, workloads.RADIUS, workloads.VISCOSITY)
        big = max(big, np.linalg.norm(u, axis=1).max())
        if om is not None:
            big = max(big, np.linalg.norm(om, axis=1).max())
    return 2 * tol_for(dtype) * big / delta


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("angular", [False, True])
@pytest.mark.parametrize("n", [300, 1000])
def test_rfd_sample_against_oracle(dtype, angular, n):
    say(f"case rfd sample N={n} angular={angular} {dtype}")
    s = workloads.uniform_cube(n, 0.15, 300 + n, torques=angular, w=True, angular_w=angular)
    delta = 1e-3 if dtype == torch.float32 else 1e-4
    sol = _solver(angular)
    sol.setPositions(torch.tensor(s.pos, dtype=dtype, device="cuda"))
    lin, ang = sol.divM_rfd(torch.tensor(s.w, dtype=dtype, device="cuda"), delta=delta)
    xr, wr = rounded(s.pos, dtype), rounded(s.w, dtype)
    rf = _round_fn(dtype)
    ref_l, ref_a = drift.rfd_sample(xr, wr, delta, workloads.RADIUS, workloads.VISCOSITY, angular,
                                    round_positions=rf)
    bound = _bound(dtype, xr, wr, delta, angular, rf)
    err = np.abs(host(lin) - ref_l).max()
    if angular:
        err = max(err, np.abs(host(ang) - ref_a).max())
    scale = max(np.abs(ref_l).max(), np.abs(ref_a).max() if angular else 0.0)
    say(f"  max abs error {err:.3e} (bound {bound:.3e}; sample magnitude {scale:.3e})")
    assert err <= bound


def test_rfd_argument_checks():
    import paper_2510_02135_amd as rpy
    say("case rfd argument checks")
    sol = _solver(False)
    x = torch.tensor(workloads.uniform_cube(20, 0.1, 5).pos, device="cuda")
    sol.setPositions(x)
    w = torch.zeros(60, dtype=torch.float64, device="cuda")
    for bad in (0.0, -1e-4, float("nan"), float("inf")):
        with pytest.raises(rpy.RpyError):
            sol.divM_rfd(w, delta=bad)
    lin, _ = sol.divM_rfd(w, delta=1e-4)          # W = 0: no displacement, zero product
    assert not host(lin).any()


@pytest.mark.timeout(300)
def test_c3_rfd_average_vanishes_and_sampled_rows():
    """d_X . M = 0 in open space by random finite differences on the
    differentiation workload (N = 16,384, phi = 0.2, float64, delta = 1e-4 a,
    256 samples): every component of the sample mean lies within 6 standard
    errors of zero (family-wise false-alarm rate about 1e-4 over the 49,152
    components), and one sample matches the C oracle on sampled rows."""
    s = workloads.c3_gradient()
    n = s.n
    say(f"case c3 rfd N={n}")
    dt = torch.float64
    sol = _solver(False)
    sol.setPositions(torch.tensor(s.pos, dtype=dt, device="cuda"))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1003)
    delta = 1e-4 * workloads.RADIUS
    acc = torch.zeros(3 * n, dtype=dt, device="cuda")
    acc2 = torch.zeros(3 * n, dtype=dt, device="cuda")
    m = 256
    first = None
    for k in range(m):
        W = torch.randn(3 * n, dtype=dt, device="cuda", generator=gen)
        lin, _ = sol.divM_rfd(W, delta=delta)
        v = lin.reshape(-1)
        acc += v
        acc2 += v * v
        if k == 0:
            first = (host(W), host(lin))
    mean = host(acc) / m
    var = (host(acc2) - m * mean ** 2) / (m - 1)
    se = np.sqrt(var / m)
    z = np.abs(mean) / se
    say(f"  max |mean| / se over {3 * n} components: {z.max():.2f}; max |mean| {np.abs(mean).max():.3e}")
    assert z.max() <= 6.0
    # one sample against the oracle on sampled rows (C pair loop)
    w0, lin0 = first
    rows = s.extra["subset"][:32] if "subset" in s.extra else np.arange(0, n, n // 32)

    def rows_mdot(x, f, t, a, eta):
        u, _ = pairloop.mdot_rows(x, rows, f, None, a, eta)
        full = np.zeros((x.shape[0], 3))
        full[rows] = u
        return full, None

    ref, _ = drift.rfd_sample(s.pos, w0, delta, s.radius, s.viscosity, False, mdot=rows_mdot)
    wp = w0.reshape(n, 3)
    big = max(np.linalg.norm(pairloop.mdot_rows(s.pos + sg * 0.5 * delta * wp, rows, wp, None, s.radius,
                                                s.viscosity)[0], axis=1).max() for sg in (1.0, -1.0))
    err = np.abs(lin0[rows] - ref[rows]).max()
    bound = 2 * tol_for(dt) * big / delta
    say(f"  sampled rows max abs error {err:.3e} (bound {bound:.3e})")
    assert err <= bound

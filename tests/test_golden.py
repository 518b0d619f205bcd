"""CPU checks of the stored oracle results in tests/golden/ against what
holds for them independently of how they were computed."""
import numpy as np
import pytest

import workloads
from oracle import gradient
from tests.golden import load as golden


@pytest.mark.parametrize("tag", ["f32", "f64"])
def test_c2_lanczos_golden_identities(tag):
    """|y_k|^2 = beta_0^2 alpha_1 = W^T M W for an orthonormal Lanczos basis
    (Sec. 3.3), and beta_0^2 = |W|^2 of the workload's (rounded) W."""
    g = golden.c2_lanczos(tag)
    assert g["k"] == 20 and len(g["alphas"]) == 20 and len(g["betas"]) == 19
    assert abs(g["ynorm2"] / g["wmw"] - 1) <= 1e-12
    assert abs(g["alphas"][0] * g["beta0sq"] / g["wmw"] - 1) <= 1e-12
    s = workloads.c2_suspension()
    w = s.w if tag == "f64" else np.asarray(s.w, np.float32).astype(np.float64)
    assert abs(float(w @ w) / g["beta0sq"] - 1) <= 1e-13
    assert np.array_equal(g["particles"], s.extra["subset"][:g["rows"]])
    assert np.all(g["betas"] > 0)


def test_c3_fd_golden_against_oracle_gradient(pairloop):
    """The stored central differences agree with the oracle's analytic
    gradient (complex-step pinned) to the truncation error of h = 1e-4."""
    s = workloads.c3_gradient()
    coords, fd = golden.c3_fd()
    assert np.array_equal(coords, s.extra["fd_pos"])
    x = np.asarray(s.pos, np.float32).astype(np.float64)
    f = np.asarray(s.forces, np.float32).astype(np.float64)
    u, _ = pairloop.mdot(x, f, None, s.radius, s.viscosity)
    us, _ = pairloop.mdot(x + s.extra["delta"], f, None, s.radius, s.viscosity)
    gx = gradient.grad_positions(x, f, None, u - us, None, s.radius, s.viscosity, rows=coords // 3)
    ad = gx[np.arange(len(coords)), coords % 3]
    assert np.abs(fd - ad).max() <= 1e-7 * np.abs(fd).max()


def test_c5_golden_header():
    g = golden.c5_wmw()
    if g is None:
        pytest.skip("c5_wmw.txt not written yet")
    s = workloads.c5_chains()
    assert np.array_equal(g["particles"], s.extra["subset"][:g["rows"]])
    assert g["wmw"] > 0

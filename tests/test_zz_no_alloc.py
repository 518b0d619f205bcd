"""rpy_mdot_noalloc (the product without device allocation) against rpy_mdot,
through the C interface: two calls in a row on one solver, the second with
fewer particles, float32 and float64, with and without the angular blocks;
and a size beyond the fixed workspace rejected with a clear error."""
import ctypes
import math

import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import emax, host, say

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2510_02135_amd import _lib as L
    lib = L.load()
    vp = ctypes.c_void_p
    lib.rpy_mdot_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.rpy_mdot_noalloc.restype = ctypes.c_int
    return L, lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("angular", [False, True])
def test_noalloc_matches_mdot_on_two_calls(dtype, angular):
    import paper_2510_02135_amd as rpy
    L, lib = _lib()
    bar = 1e-5 if dtype == torch.float32 else 1e-12
    sol = rpy.Solver()
    sol.initialize(viscosity=workloads.VISCOSITY, hydrodynamicRadius=workloads.RADIUS, includeAngular=angular)
    for n, seed in ((5000, 71), (777, 72)):
        say(f"case noalloc n={n} angular={angular} {dtype}")
        s = workloads.uniform_cube(n, 0.2, seed, torques=angular)
        sol.setPositions(torch.tensor(s.pos, dtype=dtype, device="cuda"))
        F = torch.tensor(s.forces, dtype=dtype, device="cuda")
        T = torch.tensor(s.torques, dtype=dtype, device="cuda") if angular else None
        lin_ref, ang_ref = sol.Mdot(F, T)
        lin = torch.full((n, 3), float("nan"), dtype=dtype, device="cuda")
        ang = torch.full((n, 3), float("nan"), dtype=dtype, device="cuda") if angular else None
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.rpy_mdot_noalloc(sol._h, _p(F), _p(T), _p(lin), _p(ang), st)
        assert rc == 0, lib.rpy_last_error(sol._h)
        torch.cuda.synchronize()
        e = emax(host(lin), host(lin_ref))
        if angular:
            e = max(e, emax(host(ang), host(ang_ref)))
        say(f"  e_max against rpy_mdot {e:.2e}")
        assert math.isfinite(e) and e <= bar
    sol.close()


def test_noalloc_rejects_sizes_beyond_its_workspace():
    import paper_2510_02135_amd as rpy
    L, lib = _lib()
    say("case noalloc too large")
    n = 700_000   # float64 with torques: 2 x 32 B staged + 48 B partials per particle > 64 MiB
    sol = rpy.Solver()
    sol.initialize(viscosity=1.0, hydrodynamicRadius=1.0, includeAngular=True)
    x = torch.rand((n, 3), dtype=torch.float64, device="cuda") * 1000.0
    sol.setPositions(x)
    F = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    lin = torch.zeros_like(F)
    ang = torch.zeros_like(F)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.rpy_mdot_noalloc(sol._h, _p(F), _p(F), _p(lin), _p(ang), st)
    assert rc == L.Status.INVALID_ARG
    assert b"workspace" in lib.rpy_last_error(sol._h)
    sol.close()

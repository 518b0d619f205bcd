"""The C interface without a GPU: the library loads, exports every entry
point that include/rpy.h declares, and rejects bad arguments before it
touches HIP (status codes of the header; API error tests as in Sec. 4)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2510_02135_amd", "librpy.so")
HEADER = os.path.join(ROOT, "include", "rpy.h")

OK, INVALID, GEOM, NOT_INIT, NO_POS, DTYPE, ANG = 0, 1, 2, 3, 4, 6, 7


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__._load_build_module().build_library()
    lib = ctypes.CDLL(LIB)
    lib.rpy_initialize.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.rpy_set_parameter.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_double]
    lib.rpy_set_positions.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    lib.rpy_sqrt_mdot_w.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
    lib.rpy_last_error.restype = ctypes.c_char_p
    lib.rpy_last_error.argtypes = [ctypes.c_void_p]
    lib.rpy_destroy.argtypes = [ctypes.c_void_p]
    return lib


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|void|rpy_status)\s*\**\s*(rpy_\w+)\s*\(", text, re.M)))


def test_header_declares_the_interface():
    names = declared_symbols()
    for must in ["rpy_create", "rpy_set_parameter", "rpy_initialize", "rpy_set_positions", "rpy_mdot",
                 "rpy_sqrt_mdot_w", "rpy_div_m", "rpy_mdot_backward", "rpy_last_error", "rpy_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def _solver(lib):
    h = ctypes.c_void_p()
    assert lib.rpy_create(1, 1, 1, ctypes.byref(h)) == OK
    return h


def test_geometry_checks(lib):
    out = ctypes.c_void_p(123)
    assert lib.rpy_create(1, 1, 2, ctypes.byref(out)) == OK and out.value   # open, open, single_wall
    lib.rpy_destroy(out)
    out = ctypes.c_void_p(123)
    assert lib.rpy_create(2, 1, 1, ctypes.byref(out)) == GEOM and not out.value
    assert lib.rpy_create(0, 0, 1, ctypes.byref(out)) == GEOM and not out.value
    assert lib.rpy_create(0, 1, 0, ctypes.byref(out)) == GEOM
    assert lib.rpy_create(1, 1, 3, ctypes.byref(out)) == GEOM
    assert lib.rpy_create(1, 1, 7, ctypes.byref(out)) == INVALID
    assert lib.rpy_create(1, 1, 1, None) == INVALID
    h = _solver(lib)
    lib.rpy_destroy(h)
    lib.rpy_destroy(None)


def test_periodic_geometry_host_checks(lib):
    """(periodic, periodic, periodic): parameters and initialize are host-side."""
    out = ctypes.c_void_p(0)
    assert lib.rpy_create(0, 0, 0, ctypes.byref(out)) == OK and out.value
    h = out
    try:
        for key, val in ((b"Lx", 10.0), (b"Ly", 11.0), (b"Lz", 12.0), (b"boxSize", 9.0), (b"psi", 0.0),
                         (b"psi", 1.5), (b"tolerance", 1e-6)):
            assert lib.rpy_set_parameter(h, key, val) == OK
        for key, val in ((b"Lx", 0.0), (b"Lz", -1.0), (b"psi", -0.1), (b"tolerance", 0.1), (b"tolerance", 1e-15),
                         (b"wallHeight", 0.0), (b"Lx", float("nan"))):
            assert lib.rpy_set_parameter(h, key, val) == INVALID
        assert b"periodic" in lib.rpy_last_error(h) or b"finite" in lib.rpy_last_error(h)
        assert lib.rpy_initialize(h, 1.0, 1.0, 1) == GEOM          # forces only
        assert lib.rpy_initialize(h, 1.0, 1.0, 0) == OK
    finally:
        lib.rpy_destroy(h)


def test_parameter_and_initialize_checks(lib):
    h = _solver(lib)
    try:
        assert lib.rpy_set_parameter(h, b"wallHeight", 0.0) == INVALID
        assert b"wallHeight" in lib.rpy_last_error(h)
        assert lib.rpy_initialize(h, 0.0, 1.0, 0) == INVALID
        assert lib.rpy_initialize(h, 1.0, -2.0, 0) == INVALID
        assert lib.rpy_initialize(h, float("nan"), 1.0, 0) == INVALID
        assert lib.rpy_initialize(h, 1.0, float("inf"), 0) == INVALID
        assert lib.rpy_initialize(None, 1.0, 1.0, 0) == INVALID
    finally:
        lib.rpy_destroy(h)


def test_call_order_checks(lib):
    h = _solver(lib)
    buf = ctypes.c_void_p(16)   # never dereferenced: every call below fails validation first
    assert lib.rpy_set_adjoint_mode(h, 3) == INVALID and lib.rpy_set_adjoint_mode(h, 2) == OK
    lib.rpy_mdot_multi.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    try:
        assert lib.rpy_set_positions(h, buf, 4, 0, None) == NOT_INIT
        assert lib.rpy_mdot(h, buf, None, buf, None, None) == NOT_INIT
        assert lib.rpy_mdot_multi(h, buf, None, 2, buf, None, None) == NOT_INIT
        assert lib.rpy_initialize(h, 1.0, 1.0, 0) == OK
        assert lib.rpy_mdot(h, buf, None, buf, None, None) == NO_POS
        assert lib.rpy_div_m(h, buf, None, None) == NO_POS
        assert lib.rpy_mdot_backward(h, buf, None, buf, None, buf, None, None, None) == NO_POS
        assert lib.rpy_sqrt_mdot_w(h, buf, 1.0, 1e-6, 10, buf, None, None, None, None) == NO_POS
        assert lib.rpy_mdot_multi(h, buf, None, 2, buf, None, None) == NO_POS
        assert lib.rpy_set_multi_config(h, 3) == INVALID and lib.rpy_set_multi_config(h, -1) == INVALID
        assert lib.rpy_set_multi_config(h, 2) == OK
        assert lib.rpy_set_positions(h, None, 4, 0, None) == INVALID
        assert lib.rpy_set_positions(h, buf, 0, 0, None) == INVALID
        assert lib.rpy_set_positions(h, buf, -3, 1, None) == INVALID
        assert lib.rpy_set_positions(h, buf, 4, 5, None) == DTYPE
        assert b"dtype" in lib.rpy_last_error(h)
    finally:
        lib.rpy_destroy(h)


def test_tile_config_accessors(lib):
    lib.rpy_set_tile_config.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.rpy_get_tile_config.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int)]
    lib.rpy_autotune.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p]
    h = _solver(lib)
    try:
        tm, sp = ctypes.c_int(), ctypes.c_int()
        assert lib.rpy_get_tile_config(h, 0, ctypes.byref(tm), ctypes.byref(sp)) == OK and (tm.value, sp.value) == (2, 0)
        assert lib.rpy_set_tile_config(h, 1, 4, 9) == OK
        assert lib.rpy_get_tile_config(h, 1, ctypes.byref(tm), ctypes.byref(sp)) == OK and (tm.value, sp.value) == (4, 9)
        assert lib.rpy_set_tile_config(h, 0, 5, 0) == INVALID and lib.rpy_set_tile_config(h, 0, 3, 0) == OK
        assert lib.rpy_set_tile_config(h, 0, 0, 2) == OK and lib.rpy_set_tile_config(h, 0, -1, 0) == INVALID
        assert lib.rpy_set_tile_config(h, 0, 2, -1) == INVALID
        assert lib.rpy_autotune(h, None, None) == NOT_INIT
        assert lib.rpy_initialize(h, 1.0, 1.0, 1) == OK
        assert lib.rpy_autotune(h, None, None) == NO_POS
    finally:
        lib.rpy_destroy(h)


def test_timing_accessors(lib):
    """Instrumentation classes 0..3 (pair, adjoint, Lanczos Gram-Schmidt,
    multi-vector pair) report nothing before any launch; other classes are
    rejected."""
    h = _solver(lib)
    lib.rpy_kernel_time.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    assert lib.rpy_enable_timing(h, 1) == OK
    for kind in (0, 1, 2, 3):
        ms, n, work = ctypes.c_double(-1), ctypes.c_int64(-1), ctypes.c_double(-1)
        assert lib.rpy_kernel_time(h, kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(work)) == OK
        assert (ms.value, n.value, work.value) == (0.0, 0, 0.0)
    for kind in (-1, 4):
        assert lib.rpy_kernel_time(h, kind, None, None, None) == INVALID
    assert lib.rpy_enable_timing(h, 0) == OK
    lib.rpy_destroy(h)


def test_batch_create_checks(lib):
    import numpy as np
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    lib.rpy_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_void_p)]
    one = np.ones(2)
    out = ctypes.c_void_p()
    create = lambda off, eta, rad, ang, dt: lib.rpy_batch_create(2, P(off, ctypes.c_int64), P(eta, ctypes.c_double),
                                                                 P(rad, ctypes.c_double), ang, dt, ctypes.byref(out))
    bad_off = np.array([0, 3, 3], dtype=np.int64)
    assert create(bad_off, one, one, 0, 0) == 5
    off = np.array([1, 3, 4], dtype=np.int64)
    assert create(off, one, one, 1, 0) == 5
    off = np.array([0, 3, 4], dtype=np.int64)
    neg = np.array([1.0, -1.0])
    assert create(off, neg, one, 0, 0) == INVALID
    assert create(off, one, one, 1, 7) == DTYPE
    assert lib.rpy_batch_create(0, P(off, ctypes.c_int64), P(one, ctypes.c_double), P(one, ctypes.c_double), 0, 0,
                                ctypes.byref(out)) == INVALID


def test_python_binding_module_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    import paper_2510_02135_amd._lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.load()
    importlib.reload(L)

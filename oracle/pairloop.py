"""Oracle: ctypes wrapper of the plain C float64 pair loop (``pairloop.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

``build()`` compiles the loop with ``gcc -O2 -fopenmp`` (no fast-math, no
vector intrinsics) into ``oracle/liboracle_pairloop.so``; ``load()`` builds it
when it is missing.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pairloop.c")
LIB = os.path.join(HERE, "liboracle_pairloop.so")

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_rpy_mdot.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_double,
                                        ctypes.c_double, dp, dp]
        lib.oracle_rpy_mdot_rows.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64), dp, dp]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _inputs(x, forces, torques):
    """Contiguous float64 copies, each checked to be N x 3 (the C loop reads
    3 N values of every array it is given)."""
    x, f, t = _c64(x), _c64(forces), _c64(torques)
    if x.ndim != 2 or x.shape[1] != 3:
        raise ValueError(f"positions must be N x 3, got shape {x.shape}")
    for name, v in (("forces", f), ("torques", t)):
        if v is not None and v.shape != x.shape:
            raise ValueError(f"{name} must have the positions' shape {x.shape}, got {v.shape}")
    return x, f, t


def threads() -> int:
    return int(load().oracle_threads())


def mdot(x, forces=None, torques=None, a: float = 1.0, eta: float = 1.0 / (6 * math.pi)):
    """(U, Omega) for every particle; Omega is None without torques."""
    lib = load()
    x, f, t = _inputs(x, forces, torques)
    n = x.shape[0]
    u = np.empty((n, 3))
    w = np.empty((n, 3)) if t is not None else None
    lib.oracle_rpy_mdot(n, _ptr(x), _ptr(f), _ptr(t), a, eta, _ptr(u), _ptr(w))
    return u, w


def mdot_rows(x, rows, forces=None, torques=None, a: float = 1.0,
              eta: float = 1.0 / (6 * math.pi)):
    """(U, Omega) for the target particles ``rows`` only (in that order)."""
    lib = load()
    x, f, t = _inputs(x, forces, torques)
    rows = np.asarray(rows)
    if rows.ndim != 1 or (rows.size and not np.issubdtype(rows.dtype, np.integer)):
        raise ValueError("rows must be a 1-D array of particle indices")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= x.shape[0]):
        raise ValueError(f"rows must lie in [0, {x.shape[0]})")
    m = rows.shape[0]
    u = np.empty((m, 3))
    w = np.empty((m, 3)) if t is not None else None
    lib.oracle_rpy_mdot_rows(x.shape[0], _ptr(x), _ptr(f), _ptr(t), a, eta, m,
                             rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             _ptr(u), _ptr(w))
    return u, w

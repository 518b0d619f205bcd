"""ctypes binding of librpy (include/rpy.h): argument marshalling only.

Each ``rpy_*`` function here has the name and meaning of the C entry point
it calls; it turns torch device tensors into device pointers, passes torch's
current HIP stream, and turns a non-OK status into an exception.  Nothing
here computes: every step runs in the HIP library, and importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import enum
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librpy.so")


class Status(enum.IntEnum):
    OK = 0
    INVALID_ARG = 1
    UNSUPPORTED_GEOMETRY = 2
    NOT_INITIALIZED = 3
    NO_POSITIONS = 4
    SIZE_MISMATCH = 5
    DTYPE_MISMATCH = 6
    ANGULAR_DISABLED = 7
    NONFINITE = 8
    NOT_CONVERGED = 9
    NOT_SPD = 10
    OUT_OF_MEMORY = 11
    HIP = 12


PERIODICITY = {"periodic": 0, "open": 1, "single_wall": 2, "two_walls": 3}
DTYPE = {torch.float32: 0, torch.float64: 1}


class RpyError(RuntimeError):
    """A non-OK status from librpy; ``status`` holds the code."""

    def __init__(self, status: int, message: str):
        self.status = Status(status)
        super().__init__(f"{self.status.name}: {message}")


class NotConvergedError(RpyError):
    """Lanczos hit max_iter; ``result`` holds the last iterate written."""

    def __init__(self, status, message, result=None, iters=0, increment=float("nan")):
        super().__init__(status, message)
        self.result = result
        self.iters = iters
        self.increment = increment


_lib = None


def load() -> ctypes.CDLL:
    """The loaded librpy; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"librpy.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2510_02135_amd.build` or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "rpy_create": ([i, i, i, ctypes.POINTER(vp)], i),
        "rpy_set_parameter": ([vp, ctypes.c_char_p, d], i),
        "rpy_initialize": ([vp, d, d, i], i),
        "rpy_set_positions": ([vp, vp, i64, i, vp], i),
        "rpy_mdot": ([vp, vp, vp, vp, vp, vp], i),
        "rpy_mdot_noalloc": ([vp, vp, vp, vp, vp, vp], i),
        "rpy_mdot_multi": ([vp, vp, vp, i, vp, vp, vp], i),
        "rpy_set_multi_config": ([vp, i], i),
        "rpy_sqrt_mdot_w": ([vp, vp, d, d, i, vp, vp, ctypes.POINTER(i), ctypes.POINTER(d), vp], i),
        "rpy_sqrt_mdot_w_multi": ([vp, vp, i, d, d, i, vp, vp, ctypes.POINTER(i), ctypes.POINTER(d), vp], i),
        "rpy_sqrt_mdot_w_precond": ([vp, vp, i64, d, d, i, vp, vp, ctypes.POINTER(i), ctypes.POINTER(d), vp], i),
        "rpy_pse_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(d)], i),
        "rpy_pse_sqrt_mdot_w": ([vp, vp, vp, d, d, i, vp, ctypes.POINTER(i), ctypes.POINTER(d), vp], i),
        "rpy_mobility_solve": ([vp, vp, vp, i, d, i, vp, vp, ctypes.POINTER(i), ctypes.POINTER(d), vp], i),
        "rpy_div_m": ([vp, vp, vp, vp], i),
        "rpy_div_m_rfd": ([vp, vp, d, vp, vp, vp], i),
        "rpy_langevin_velocities": ([vp, vp, vp, vp, d, d, d, i, vp, vp, ctypes.POINTER(i), vp], i),
        "rpy_ab2_step": ([vp, vp, vp, vp, d, d, d, i, vp, i, vp, vp, ctypes.POINTER(i), vp], i),
        "rpy_mdot_backward": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i),
        "rpy_set_adjoint_mode": ([vp, i], i),
        "rpy_batch_create": ([ctypes.c_int32, ctypes.POINTER(i64), ctypes.POINTER(d), ctypes.POINTER(d), i, i,
                              ctypes.POINTER(vp)], i),
        "rpy_batch_set_positions": ([vp, vp, vp], i),
        "rpy_batch_mdot": ([vp, vp, vp, vp, vp, vp], i),
        "rpy_batch_sqrt_mdot_w": ([vp, vp, d, d, i, i, vp, vp, ctypes.POINTER(i), vp], i),
        "rpy_batch_last_error": ([vp], ctypes.c_char_p),
        "rpy_batch_set_tile_config": ([vp, i, i], i),
        "rpy_batch_get_tile_config": ([vp, ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "rpy_batch_autotune": ([vp, vp], i),
        "rpy_batch_destroy": ([vp], None),
        "rpy_set_tile_config": ([vp, i, i, i], i),
        "rpy_get_tile_config": ([vp, i, ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "rpy_autotune": ([vp, ctypes.c_char_p, vp], i),
        "rpy_enable_timing": ([vp, i], i),
        "rpy_kernel_time": ([vp, i, ctypes.POINTER(d), ctypes.POINTER(i64), ctypes.POINTER(d)], i),
        "rpy_last_error": ([vp], ctypes.c_char_p),
        "rpy_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _stream(t: torch.Tensor | None = None):
    dev = t.device if t is not None else torch.device("cuda", torch.cuda.current_device())
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: torch.Tensor | None, dtype: torch.dtype | None = None, numel: int | None = None,
         name: str = "tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"DTYPE_MISMATCH: {name} is {t.dtype}, the solver works in {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _check(h, status: int):
    if status != 0:
        raise RpyError(status, load().rpy_last_error(h).decode() if h else "")


def rpy_create(x: str = "open", y: str = "open", z: str = "open"):
    lib = load()
    out = ctypes.c_void_p()
    try:
        codes = [PERIODICITY[p] for p in (x, y, z)]
    except KeyError as e:
        raise ValueError(f"unknown periodicity {e.args[0]!r}; one of {sorted(PERIODICITY)}") from None
    st = lib.rpy_create(*codes, ctypes.byref(out))
    if st != 0:
        raise RpyError(st, f"rpy_create({x}, {y}, {z})")
    return out


def rpy_set_parameter(h, key: str, value: float):
    _check(h, load().rpy_set_parameter(h, key.encode(), float(value)))


def rpy_initialize(h, viscosity: float, radius: float, include_angular: bool):
    _check(h, load().rpy_initialize(h, float(viscosity), float(radius), int(bool(include_angular))))


def rpy_set_positions(h, pos: torch.Tensor):
    if pos.dtype not in DTYPE:
        raise ValueError(f"DTYPE_MISMATCH: positions must be float32 or float64, got {pos.dtype}")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("positions must have shape (N, 3)")
    p = _ptr(pos, name="positions")
    _check(h, load().rpy_set_positions(h, p, pos.shape[0], DTYPE[pos.dtype], _stream(pos)))


def rpy_mdot(h, forces, torques, lin_out, ang_out, dtype, n):
    _check(h, load().rpy_mdot(h, _ptr(forces, dtype, 3 * n, "forces"), _ptr(torques, dtype, 3 * n, "torques"),
                              _ptr(lin_out, dtype, 3 * n, "lin_out"), _ptr(ang_out, dtype, 3 * n, "ang_out"),
                              _stream(lin_out)))


def rpy_mdot_noalloc(h, forces, torques, lin_out, ang_out, dtype, n):
    _check(h, load().rpy_mdot_noalloc(h, _ptr(forces, dtype, 3 * n, "forces"), _ptr(torques, dtype, 3 * n, "torques"),
                                      _ptr(lin_out, dtype, 3 * n, "lin_out"), _ptr(ang_out, dtype, 3 * n, "ang_out"),
                                      _stream(lin_out)))


def rpy_mdot_multi(h, forces, torques, nrhs, lin_out, ang_out, dtype, n):
    m = 3 * n * nrhs
    _check(h, load().rpy_mdot_multi(h, _ptr(forces, dtype, m, "forces"), _ptr(torques, dtype, m, "torques"),
                                    int(nrhs), _ptr(lin_out, dtype, m, "lin_out"), _ptr(ang_out, dtype, m, "ang_out"),
                                    _stream(lin_out)))


def rpy_set_adjoint_mode(h, mode):
    _check(h, load().rpy_set_adjoint_mode(h, int(mode)))


def rpy_set_multi_config(h, targets_per_lane):
    _check(h, load().rpy_set_multi_config(h, int(targets_per_lane)))


def rpy_sqrt_mdot_w(h, w, prefactor, tol, max_iter, lin_out, ang_out, dtype, n, angular):
    iters = ctypes.c_int(0)
    incr = ctypes.c_double(0.0)
    st = load().rpy_sqrt_mdot_w(h, _ptr(w, dtype, (6 if angular else 3) * n, "W"), float(prefactor),
                                float(tol), int(max_iter), _ptr(lin_out, dtype, 3 * n, "lin_out"),
                                _ptr(ang_out, dtype, 3 * n, "ang_out"), ctypes.byref(iters),
                                ctypes.byref(incr), _stream(lin_out))
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_last_error(h).decode(), (lin_out, ang_out),
                                iters.value, incr.value)
    _check(h, st)
    return iters.value, incr.value


def rpy_sqrt_mdot_w_precond(h, w, group_size, prefactor, tol, max_iter, lin_out, ang_out, dtype, n, angular):
    iters = ctypes.c_int(0)
    incr = ctypes.c_double(0.0)
    st = load().rpy_sqrt_mdot_w_precond(h, _ptr(w, dtype, (6 if angular else 3) * n, "W"), int(group_size),
                                        float(prefactor), float(tol), int(max_iter),
                                        _ptr(lin_out, dtype, 3 * n, "lin_out"), _ptr(ang_out, dtype, 3 * n, "ang_out"),
                                        ctypes.byref(iters), ctypes.byref(incr), _stream(lin_out))
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_last_error(h).decode(), (lin_out, ang_out),
                                iters.value, incr.value)
    _check(h, st)
    return iters.value, incr.value


def rpy_pse_info(h):
    """(grid (Nx, Ny, Nz), xi, rc, sigma, support P, wave cutoff kc) of a periodic solver."""
    grid = (ctypes.c_int64 * 3)()
    info = (ctypes.c_double * 5)()
    _check(h, load().rpy_pse_info(h, grid, info))
    return tuple(int(g) for g in grid), info[0], info[1], info[2], int(info[3]), info[4]


def rpy_pse_sqrt_mdot_w(h, w, noise, noise_count, prefactor, tol, max_iter, lin_out, dtype, n):
    iters = ctypes.c_int(0)
    incr = ctypes.c_double(0.0)
    st = load().rpy_pse_sqrt_mdot_w(h, _ptr(w, dtype, 3 * n, "W"), _ptr(noise, dtype, noise_count, "wave noise"),
                                    float(prefactor), float(tol), int(max_iter), _ptr(lin_out, dtype, 3 * n, "lin_out"),
                                    ctypes.byref(iters), ctypes.byref(incr), _stream(lin_out))
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_last_error(h).decode(), (lin_out, None), iters.value, incr.value)
    _check(h, st)
    return iters.value, incr.value


def rpy_sqrt_mdot_w_multi(h, w, nrhs, prefactor, tol, max_iter, lin_out, ang_out, dtype, n, angular):
    """Per-vector (iterations, increments) lists; NotConvergedError carries them too."""
    iters = (ctypes.c_int * nrhs)()
    incr = (ctypes.c_double * nrhs)()
    m = 3 * n * nrhs
    st = load().rpy_sqrt_mdot_w_multi(h, _ptr(w, dtype, (2 if angular else 1) * m, "W"), int(nrhs),
                                      float(prefactor), float(tol), int(max_iter), _ptr(lin_out, dtype, m, "lin_out"),
                                      _ptr(ang_out, dtype, m, "ang_out"), iters, incr, _stream(lin_out))
    its, incs = list(iters), list(incr)
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_last_error(h).decode(), (lin_out, ang_out), its, incs)
    _check(h, st)
    return its, incs


def rpy_mobility_solve(h, u_lin, u_ang, nrhs, tol, max_iter, f_out, t_out, dtype, n):
    """Per right-hand side (iterations, relative residuals) lists."""
    iters = (ctypes.c_int * nrhs)()
    resid = (ctypes.c_double * nrhs)()
    m = 3 * n * nrhs
    st = load().rpy_mobility_solve(h, _ptr(u_lin, dtype, m, "U"), _ptr(u_ang, dtype, m, "Omega"), int(nrhs),
                                   float(tol), int(max_iter), _ptr(f_out, dtype, m, "f_out"),
                                   _ptr(t_out, dtype, m, "t_out"), iters, resid, _stream(f_out))
    its, res = list(iters), list(resid)
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_last_error(h).decode(), (f_out, t_out), its, res)
    _check(h, st)
    return its, res


def rpy_div_m(h, lin_out, ang_out, dtype, n):
    _check(h, load().rpy_div_m(h, _ptr(lin_out, dtype, 3 * n, "lin_out"),
                               _ptr(ang_out, dtype, 3 * n, "ang_out"), _stream(lin_out)))


def rpy_div_m_rfd(h, w, delta, lin_out, ang_out, dtype, n, angular):
    _check(h, load().rpy_div_m_rfd(h, _ptr(w, dtype, (6 if angular else 3) * n, "W"), float(delta),
                                   _ptr(lin_out, dtype, 3 * n, "lin_out"), _ptr(ang_out, dtype, 3 * n, "ang_out"),
                                   _stream(lin_out)))


def _step_status(h, st, outs, iters):
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_last_error(h).decode(), outs, iters, float("nan"))
    _check(h, st)
    return iters


def rpy_langevin_velocities(h, forces, torques, w, dt, kbt, tol, max_iter, lin_out, ang_out, dtype, n, angular):
    iters = ctypes.c_int(0)
    st = load().rpy_langevin_velocities(
        h, _ptr(forces, dtype, 3 * n, "forces"), _ptr(torques, dtype, 3 * n, "torques"),
        _ptr(w, dtype, (6 if angular else 3) * n, "W"), float(dt), float(kbt), float(tol), int(max_iter),
        _ptr(lin_out, dtype, 3 * n, "lin_out"), _ptr(ang_out, dtype, 3 * n, "ang_out"), ctypes.byref(iters),
        _stream(lin_out))
    return _step_status(h, st, (lin_out, ang_out), iters.value)


def rpy_ab2_step(h, forces, torques, w, dt, kbt, tol, max_iter, history, have_history, pos_out, ang_out, dtype, n,
                 angular):
    iters = ctypes.c_int(0)
    st = load().rpy_ab2_step(
        h, _ptr(forces, dtype, 3 * n, "forces"), _ptr(torques, dtype, 3 * n, "torques"),
        _ptr(w, dtype, (6 if angular else 3) * n, "W"), float(dt), float(kbt), float(tol), int(max_iter),
        _ptr(history, dtype, (6 if angular else 3) * n, "history"), int(bool(have_history)),
        _ptr(pos_out, dtype, 3 * n, "pos_out"), _ptr(ang_out, dtype, 3 * n, "ang_out"), ctypes.byref(iters),
        _stream(pos_out))
    return _step_status(h, st, (pos_out, ang_out), iters.value)


def rpy_mdot_backward(h, forces, torques, grad_lin, grad_ang, grad_pos, grad_forces, grad_torques, dtype, n):
    ref = next(t for t in (grad_pos, grad_forces, grad_torques, grad_lin) if t is not None)
    _check(h, load().rpy_mdot_backward(
        h, _ptr(forces, dtype, 3 * n, "forces"), _ptr(torques, dtype, 3 * n, "torques"),
        _ptr(grad_lin, dtype, 3 * n, "grad_lin"), _ptr(grad_ang, dtype, 3 * n, "grad_ang"),
        _ptr(grad_pos, dtype, 3 * n, "grad_pos"), _ptr(grad_forces, dtype, 3 * n, "grad_forces"),
        _ptr(grad_torques, dtype, 3 * n, "grad_torques"), _stream(ref)))


def rpy_batch_set_tile_config(h, targets_per_lane: int, workgroups_per_cu: int):
    _bcheck(h, load().rpy_batch_set_tile_config(h, int(targets_per_lane), int(workgroups_per_cu)))


def rpy_batch_get_tile_config(h):
    tm, wg = ctypes.c_int(0), ctypes.c_int(0)
    _bcheck(h, load().rpy_batch_get_tile_config(h, ctypes.byref(tm), ctypes.byref(wg)))
    return tm.value, wg.value


def rpy_batch_autotune(h):
    _bcheck(h, load().rpy_batch_autotune(h, _stream()))


def _bcheck(h, status: int):
    if status != 0:
        raise RpyError(status, load().rpy_batch_last_error(h).decode() if h else "")


def rpy_batch_create(offsets, viscosity, radius, dtype: torch.dtype, include_angular: bool = False):
    """Batch of independent systems; offsets has n_systems + 1 entries."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    eta = np.ascontiguousarray(viscosity, dtype=np.float64)
    rad = np.ascontiguousarray(radius, dtype=np.float64)
    ns = off.shape[0] - 1
    if ns < 1 or eta.shape[0] != ns or rad.shape[0] != ns:
        raise ValueError("offsets must have n_systems + 1 entries and viscosity/radius n_systems")
    if dtype not in DTYPE:
        raise ValueError(f"DTYPE_MISMATCH: dtype must be float32 or float64, got {dtype}")
    out = ctypes.c_void_p()
    st = load().rpy_batch_create(ns, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 eta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 rad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(bool(include_angular)),
                                 DTYPE[dtype],
                                 ctypes.byref(out))
    if st != 0:
        raise RpyError(st, "rpy_batch_create")
    return out


def rpy_batch_set_positions(h, pos, dtype, total):
    _bcheck(h, load().rpy_batch_set_positions(h, _ptr(pos, dtype, 3 * total, "positions"), _stream(pos)))


def rpy_batch_mdot(h, forces, torques, lin_out, ang_out, dtype, total):
    m = 3 * total
    _bcheck(h, load().rpy_batch_mdot(h, _ptr(forces, dtype, m, "forces"), _ptr(torques, dtype, m, "torques"),
                                     _ptr(lin_out, dtype, m, "lin_out"), _ptr(ang_out, dtype, m, "ang_out"),
                                     _stream(lin_out)))


def rpy_batch_sqrt_mdot_w(h, w, prefactor, tol, max_iter, check_every, lin_out, ang_out, dtype, total, n_systems):
    iters = (ctypes.c_int * n_systems)()
    wn = (6 if ang_out is not None else 3) * total
    st = load().rpy_batch_sqrt_mdot_w(h, _ptr(w, dtype, wn, "W"), float(prefactor), float(tol),
                                      int(max_iter), int(check_every), _ptr(lin_out, dtype, 3 * total, "lin_out"),
                                      _ptr(ang_out, dtype, 3 * total, "ang_out"), iters, _stream(lin_out))
    it = list(iters)
    if st == Status.NOT_CONVERGED:
        raise NotConvergedError(st, load().rpy_batch_last_error(h).decode(),
                                lin_out if ang_out is None else (lin_out, ang_out), it, float("nan"))
    _bcheck(h, st)
    return it


def rpy_batch_destroy(h):
    if h:
        load().rpy_batch_destroy(h)


def rpy_set_tile_config(h, angular: bool, targets_per_lane: int, source_splits: int):
    _check(h, load().rpy_set_tile_config(h, int(bool(angular)), int(targets_per_lane), int(source_splits)))


def rpy_get_tile_config(h, angular: bool):
    tm = ctypes.c_int(0)
    sp = ctypes.c_int(0)
    _check(h, load().rpy_get_tile_config(h, int(bool(angular)), ctypes.byref(tm), ctypes.byref(sp)))
    return tm.value, sp.value


def rpy_autotune(h, cache_path: str | None = None):
    path = None if cache_path is None else os.fspath(cache_path).encode()
    _check(h, load().rpy_autotune(h, path, _stream()))


def rpy_enable_timing(h, enable: bool = True):
    _check(h, load().rpy_enable_timing(h, int(bool(enable))))


KERNEL = {"pair": 0, "adjoint": 1, "lanczos_cgs": 2, "pair_multi": 3}


def rpy_kernel_time(h, kernel: str = "pair"):
    """(total milliseconds, records, work) recorded for a kernel class; work
    is ordered pairs for "pair" and "adjoint", pairs times vectors for
    "pair_multi", algorithmic HBM bytes for "lanczos_cgs"."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    work = ctypes.c_double(0.0)
    _check(h, load().rpy_kernel_time(h, KERNEL[kernel], ctypes.byref(ms), ctypes.byref(n), ctypes.byref(work)))
    return ms.value, n.value, work.value


def rpy_last_error(h) -> str:
    return load().rpy_last_error(h).decode()


def rpy_destroy(h):
    if h:
        load().rpy_destroy(h)

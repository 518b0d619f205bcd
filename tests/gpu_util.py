"""Helpers shared by the GPU tests (no method arithmetic here)."""
from __future__ import annotations

import numpy as np

F32_TOL = 1e-5     # float32 pair path, against the oracle on float32-rounded inputs
F64_TOL = 1e-12    # float64 pair path


def emax(got, ref) -> float:
    """max_i |got_i - ref_i|_2 / max_i |ref_i|_2 over particles (rows)."""
    got = np.asarray(got, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    den = np.linalg.norm(ref, axis=1).max()
    num = np.linalg.norm(got - ref, axis=1).max()
    if den == 0.0:   # an exactly zero reference must be matched exactly
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)


def say(*args):
    print(*args, flush=True)


def to_dev(x, dtype):
    import torch
    return None if x is None else torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def host(t):
    return None if t is None else t.detach().cpu().numpy().astype(np.float64)


def tol_for(dtype):
    import torch
    return F64_TOL if dtype == torch.float64 else F32_TOL


def rounded(x, dtype):
    """The values the device sees: float32 rounding for a float32 solver."""
    import torch
    if x is None:
        return None
    if dtype == torch.float32:
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)

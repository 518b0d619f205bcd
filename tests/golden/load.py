"""Readers of the stored expected values in tests/golden/ (text files written
by make_goldens.py from the CPU oracle)."""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _lines(name):
    with open(os.path.join(HERE, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def c2_lanczos(tag: str) -> dict:
    """k, |y_k|^2, beta_0^2, W^T M W, alphas, betas, particle rows and their
    (linear, angular) y_k values from c2_lanczos_k20_<tag>.txt."""
    out, rows, vals = {}, [], []
    for ln in _lines(f"c2_lanczos_k20_{tag}.txt"):
        key = ln[0]
        if key in ("k", "rows"):
            out[key] = int(ln[1])
        elif key in ("ynorm2", "beta0sq", "wmw"):
            out[key] = float(ln[1])
        elif key in ("alphas", "betas"):
            out[key] = np.array([float(v) for v in ln[1:]])
        else:
            rows.append(int(key))
            vals.append([float(v) for v in ln[1:]])
    v = np.array(vals)
    out["particles"] = np.array(rows, dtype=np.int64)
    out["lin"], out["ang"] = v[:, :3], v[:, 3:]
    return out


def c3_fd() -> tuple[np.ndarray, np.ndarray]:
    """(flat coordinates, central-difference dL/dX) from c3_fd.txt."""
    ln = _lines("c3_fd.txt")
    return np.array([int(r[0]) for r in ln], dtype=np.int64), np.array([float(r[1]) for r in ln])


def c5_wmw() -> dict | None:
    """W^T M W and sampled rows of M W for the bead chains, or None when the
    file has not been written."""
    path = os.path.join(HERE, "c5_wmw.txt")
    if not os.path.exists(path):
        return None
    out, rows, vals = {}, [], []
    for ln in _lines("c5_wmw.txt"):
        if ln[0] == "wmw":
            out["wmw"] = float(ln[1])
        elif ln[0] == "rows":
            out["rows"] = int(ln[1])
        else:
            rows.append(int(ln[0]))
            vals.append([float(v) for v in ln[1:]])
    v = np.array(vals)
    out["particles"] = np.array(rows, dtype=np.int64)
    out["lin"], out["ang"] = v[:, :3], v[:, 3:]
    return out

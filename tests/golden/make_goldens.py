"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Every number written here comes from ``oracle/`` (float64 CPU code) applied to
the seeded inputs of ``workloads``; nothing is taken from the HIP library.

    python tests/golden/make_goldens.py c2_lanczos   # ~40 angular products at N = 65,536
    python tests/golden/make_goldens.py c3_fd        # 128 translational products at N = 16,384
    python tests/golden/make_goldens.py c5_wmw       # one angular product at N = 1,048,576

Files (plain text, one header block of '#' lines stating the recipe):

* ``c2_lanczos_k20_f32.txt`` / ``c2_lanczos_k20_f64.txt``: the Lanczos
  iterate y_20 of the square root M^{1/2} W (Sec. 3.3; ``oracle.lanczos``
  run for exactly 20 iterations, products by ``oracle.pairloop``) on the
  N = 65,536 suspension with torques (seed 1002), for the first 1024
  particles of the workload's 4096-particle subset: linear rows, then
  angular rows; also |y_20|^2, beta_0^2 and W^T M W, and the 20 alphas and
  19 betas.  The f32 file evaluates the oracle on the float32-rounded
  positions and W promoted to float64 (the values a float32 solver sees),
  the f64 file on the float64 draws.
* ``c3_fd.txt``: central differences (h = 1e-4, float64) of
  L(X) = 0.5 |M(X) F - U*|^2, U* = M(X + delta) F, on the 64 position
  coordinates of the N = 16,384 gradient workload (seed 1003), evaluated
  with ``oracle.pairloop`` on the float32-rounded X and F.
* ``c5_wmw.txt``: W^T M W for the 4096 x 256 bead chains (seed 1005) with
  torques (6N noise vector), float32-rounded positions and W, one full
  ``oracle.pairloop`` product, summed over particles in index order; also
  M W on the first 32 particles of the workload's subset.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import lanczos, pairloop  # noqa: E402

K_MATCHED = 20
C2_ROWS = 1024


def _r32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _fmt(v):
    return repr(float(v))


def _log(msg):
    print(msg, flush=True)


def c2_lanczos():
    s = workloads.c2_suspension()
    n = s.n
    rows = s.extra["subset"][:C2_ROWS]
    for tag, x, w in (("f32", _r32(s.pos), _r32(s.w)), ("f64", s.pos, s.w)):
        count = [0]

        def mv(v):
            t0 = time.time()
            u, om = pairloop.mdot(x, v[:3 * n].reshape(n, 3), v[3 * n:].reshape(n, 3),
                                  s.radius, s.viscosity)
            count[0] += 1
            _log(f"  {tag} product {count[0]} ({time.time() - t0:.1f} s)")
            return np.concatenate([u.reshape(-1), om.reshape(-1)])

        y, info = lanczos.lanczos_sqrt(mv, w, iters=K_MATCHED)
        # W^T M W from one more product of the oracle (the norm identity's right side)
        wmw = float(w @ mv(w))
        beta0 = float(np.linalg.norm(w))
        lin = y[:3 * n].reshape(n, 3)[rows]
        ang = y[3 * n:].reshape(n, 3)[rows]
        path = os.path.join(HERE, f"c2_lanczos_k{K_MATCHED}_{tag}.txt")
        with open(path, "w") as fh:
            fh.write("# Lanczos iterate y_k of M^{1/2} W (Sec. 3.3), k = 20 exactly, oracle.lanczos with\n")
            fh.write("# oracle.pairloop products; N = 65,536 suspension, phi = 0.1, seed 1002, a = 1,\n")
            fh.write("# eta = 1/(6 pi), torques, W of length 6N; inputs "
                     + ("rounded to float32, promoted to float64\n" if tag == "f32" else "float64 draws\n"))
            fh.write("# written by tests/golden/make_goldens.py c2_lanczos\n")
            fh.write(f"k {K_MATCHED}\n")
            fh.write(f"ynorm2 {_fmt(y @ y)}\n")
            fh.write(f"beta0sq {_fmt(beta0 * beta0)}\n")
            fh.write(f"wmw {_fmt(wmw)}\n")
            fh.write("alphas " + " ".join(_fmt(a) for a in info.alphas) + "\n")
            fh.write("betas " + " ".join(_fmt(b) for b in info.betas) + "\n")
            fh.write(f"rows {len(rows)}\n")
            for i, p in enumerate(rows):
                fh.write(f"{int(p)} " + " ".join(_fmt(v) for v in lin[i]) + " "
                         + " ".join(_fmt(v) for v in ang[i]) + "\n")
        _log(f"wrote {path}: |y|^2 = {y @ y:.12e}, W^T M W = {wmw:.12e}")


def c3_fd():
    s = workloads.c3_gradient()
    x, f = _r32(s.pos), _r32(s.forces)
    ustar, _ = pairloop.mdot(x + s.extra["delta"], f, None, s.radius, s.viscosity)
    h = 1e-4
    coords = s.extra["fd_pos"]
    fd = []
    for k, c in enumerate(coords):
        p, ax = divmod(int(c), 3)
        vals = []
        for sgn in (1.0, -1.0):
            xp = x.copy()
            xp[p, ax] += sgn * h
            u, _ = pairloop.mdot(xp, f, None, s.radius, s.viscosity)
            vals.append(0.5 * float(((u - ustar) ** 2).sum()))
        fd.append((vals[0] - vals[1]) / (2 * h))
        _log(f"  coordinate {k + 1}/64: {fd[-1]:.12e}")
    path = os.path.join(HERE, "c3_fd.txt")
    with open(path, "w") as fh:
        fh.write("# Central differences (h = 1e-4, float64) of L(X) = 0.5 |M(X) F - U*|^2,\n")
        fh.write("# U* = M(X + delta) F; N = 16,384, phi = 0.2, seed 1003, a = 1, eta = 1/(6 pi);\n")
        fh.write("# X and F rounded to float32 and promoted; products by oracle.pairloop\n")
        fh.write("# written by tests/golden/make_goldens.py c3_fd\n")
        fh.write("# columns: flat coordinate index (particle * 3 + axis), dL/dX\n")
        for c, v in zip(coords, fd):
            fh.write(f"{int(c)} {_fmt(v)}\n")
    _log(f"wrote {path}")


def c5_wmw():
    s = workloads.c5_chains()
    n = s.n
    x, w = _r32(s.pos), _r32(s.w)
    wf, wt = w[:3 * n].reshape(n, 3), w[3 * n:].reshape(n, 3)
    total = 0.0
    chunk = 8192
    t0 = time.time()
    for start in range(0, n, chunk):
        rows = np.arange(start, min(n, start + chunk))
        u, om = pairloop.mdot_rows(x, rows, wf, wt, s.radius, s.viscosity)
        total += float((u * wf[rows]).sum() + (om * wt[rows]).sum())
        _log(f"  rows {rows[-1] + 1}/{n} ({time.time() - t0:.0f} s)")
    sub = s.extra["subset"][:32]
    u, om = pairloop.mdot_rows(x, sub, wf, wt, s.radius, s.viscosity)
    path = os.path.join(HERE, "c5_wmw.txt")
    with open(path, "w") as fh:
        fh.write("# W^T M W for the 4096 x 256 bead chains (N = 1,048,576, bond 2.1 a, phi = 0.05,\n")
        fh.write("# seed 1005), a = 1, eta = 1/(6 pi), torques, W of length 6N; positions and W rounded to\n")
        fh.write("# float32 and promoted; one full oracle.pairloop product, particle sums in index order\n")
        fh.write("# written by tests/golden/make_goldens.py c5_wmw\n")
        fh.write(f"wmw {_fmt(total)}\n")
        fh.write(f"rows {len(sub)}\n")
        fh.write("# particle, (M W) linear rows then angular rows\n")
        for i, p in enumerate(sub):
            fh.write(f"{int(p)} " + " ".join(_fmt(v) for v in u[i]) + " "
                     + " ".join(_fmt(v) for v in om[i]) + "\n")
    _log(f"wrote {path}: W^T M W = {total:.12e}")


if __name__ == "__main__":
    pairloop.load()
    _log(f"oracle pair loop on {pairloop.threads()} threads")
    {"c2_lanczos": c2_lanczos, "c3_fd": c3_fd, "c5_wmw": c5_wmw}[sys.argv[1]]()

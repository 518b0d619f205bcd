"""Benchmark of the open-boundary RPY mobility hot path on one MI355X.

One step is one pass of the whole single-system hot path over the
N = 65,536 suspension (uniform cube at volume fraction 0.1, a = 1,
eta = 1/(6 pi), F, T, W ~ N(0, 1), seed 1002), in the float32 pair mode:

    Mdot(F, T)                      linear + angular product
    sqrtMdotW(W), tol 1e-6          Lanczos, float64 basis on the device
    divM()                          thermal drift (zero in open space)
    Mdot_backward(F, T, gU, gW)     adjoint: dL/dX, dL/dF, dL/dT

value = N^2 x (number of M products in the step: 1 + Lanczos iterations)
divided by the step time, in pair-interactions/s (the drift and the backward
pass are inside the timed step but add no M products).  Inputs are resident
in device memory before timing starts.

Also reported (outside the timed steps, same data): float32 and float64
pair-interactions/s of one Mdot (translational, and with torques), the
backward/forward time ratio, the roofline position of the dominant kernel
(the float32 angular pair kernel, timed with HIP events on its own stream
inside the timed steps), the HBM rate of the Lanczos vector operations (the
Gram-Schmidt passes, timed the same way, algorithmic bytes), the max
relative error of each result against the float64 CPU oracle on sampled
particles, the oracle's own rate on a bounded sample of the same workload on
the host cores, the 512-system batch (one persistent launch vs one launch
per system), one angular product of 4096 bead chains x 256 beads, and the
multi-vector calls (eight force sets in one product; four noise vectors in
one lockstep Lanczos) against one call per vector.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RPY pair-interactions/s for M·F, FP32 vs FP64, N=65,536; backward/forward"
PEAK_FP32_TFLOPS = 157.3    # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0       # MI355X HBM3E
FLOPS_PER_PAIR = {"linear": 34, "angular": 84}
# single-wall geometry: the open pair plus the image part of the wall kernel
FLOPS_PER_WALL_PAIR = {"linear": 131, "angular": 305}


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=65536, help="particles (default: the 65,536 workload)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle sample")
    p.add_argument("--no-breakdown", action="store_true", help="skip the per-precision breakdown and oracle check")
    p.add_argument("--no-batch", action="store_true",
                   help="skip the batched-systems and bead-chain measurements")
    p.add_argument("--tile-cache", default=None,
                   help="autotune cache file (read if it has an entry, else written)")
    p.add_argument("--tiles", default=None,
                   help="TM,S: fixed pair-kernel tiles for the step's solver instead of autotuning "
                        "(targets per lane, source splits; 0,B is the symmetric mode with B source blocks per task)")
    p.add_argument("--chains-lanczos-iters", type=int, default=20,
                   help="Lanczos iterations of the fixed-length bead-chain leg")
    p.add_argument("--sweep", action="store_true",
                   help="instead of the step: Mdot time against N = 2^10 .. 2^20 at number densities 0.1 and "
                        "0.001 per a^3 (translational, float32), the axes of the paper's timing figure")
    p.add_argument("--batch-only", nargs="?", const="all", default=None, choices=("all", "mdot", "batched"),
                   help="instead of the step: only the 512 batched systems (one launch against one per system); "
                        "'mdot' stops after the batched products, 'batched' skips the per-system calls")
    p.add_argument("--sweep-sizes", default=None,
                   help="comma-separated particle counts for --sweep (default: 2^10 .. 2^20)")
    p.add_argument("--breakdown-only", action="store_true",
                   help="only the float32/float64 Mdot and backward timings at N (tiles from --tiles, else autotuned)")
    p.add_argument("--pse-only", action="store_true",
                   help="only the triply periodic (PSE) products; one JSON line")
    p.add_argument("--pse-size", default=None,
                   help="N:density of the one periodic workload to run (default: all three)")
    p.add_argument("--chains-solve", action="store_true",
                   help="instead of the step: the converged sqrtMdotW (tol 1e-6, float32 pairs, angular) of the "
                        "4096 x 256-bead chains, plain and preconditioned with one chain per group")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    return p.parse_args()


def emax(got, ref):
    import numpy as np
    got = np.asarray(got, dtype=np.float64).reshape(-1, 3)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    return float(np.linalg.norm(got - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())


def hbm_traffic(kernel: str, n: int, tile):
    """HBM bytes per launch of `kernel` at tile configuration `tile` from the
    committed counter summary (FETCH_SIZE and WRITE_SIZE passes scaled by a
    plain copy), or None when the summary has no entry for that kernel, N
    and tile, or the kernel sources have changed since the counters were
    taken (an entry may name its own sources and hash; the others use the
    summary's)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pair_kernel_f32_angular_n65536_hbm.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None

    def sources_unchanged(files, digest):
        h = hashlib.sha256()
        for f in files:
            try:
                h.update(open(os.path.join(ROOT, f), "rb").read())
            except OSError:
                return False
        return bool(files) and h.hexdigest() == digest

    for e in d.get("entries", []):
        if e.get("kernel") == kernel and e.get("n") == n and list(e.get("tile", [])) == list(tile):
            files = e.get("kernel_sources", d.get("kernel_sources", []))
            digest = e.get("kernel_source_sha256", d.get("kernel_source_sha256"))
            return e.get("traffic_bytes_per_dispatch") if sources_unchanged(files, digest) else None
    return None


def bench_batched(rpy, workloads, dev, stream, timed, mdot_only=False, batched_only=False):
    """512 independent systems (N log-uniform in [64, 8192], phi in [0.05, 0.3],
    seed 1004), float32: Mdot and sqrtMdotW (tol 1e-6) for all systems in one
    batched call vs one single-system solver call per system (batched_only:
    without the per-system calls)."""
    import numpy as np
    import torch
    syss = workloads.c4_systems()
    ns = np.array([s.n for s in syss])
    off = np.concatenate([[0], np.cumsum(ns)])
    f32 = torch.float32
    X = torch.tensor(np.concatenate([s.pos for s in syss]), dtype=f32, device=dev)
    F = torch.tensor(np.concatenate([s.forces for s in syss]), dtype=f32, device=dev)
    W = torch.tensor(np.concatenate([s.w for s in syss]), dtype=f32, device=dev)
    b = rpy.Batch(off, workloads.VISCOSITY, workloads.RADIUS, f32)
    b.setPositions(X)
    batch_tiles = b.autotune()
    b.Mdot(F)
    t_mdot = timed(lambda: b.Mdot(F), 10, stream, warmup=3)
    pairs = float((ns.astype(np.float64) ** 2).sum())
    # the same systems with angular blocks (torques N(0, 1), seed 1009; 6N noise)
    rng_a = np.random.default_rng(1009)
    Ta = torch.tensor(rng_a.standard_normal((int(off[-1]), 3)), dtype=f32, device=dev)
    Wa = torch.tensor(rng_a.standard_normal(6 * int(off[-1])), dtype=f32, device=dev)
    ba = rpy.Batch(off, workloads.VISCOSITY, workloads.RADIUS, f32, includeAngular=True)
    ba.setPositions(X)
    ba.Mdot(F, Ta)
    t_mdot_ang = timed(lambda: ba.Mdot(F, Ta), 10, stream, warmup=3)
    angular = {"mdot_ms": round(t_mdot_ang, 4), "mdot_pairs_per_s": pairs / (t_mdot_ang * 1e-3),
               "tile_config": "block mode"}
    if mdot_only:
        b.close()
        ba.close()
        return {"systems": len(syss), "total_particles": int(off[-1]), "sum_n2": pairs,
                "tile_config": {"targets_per_lane": batch_tiles[0], "workgroups_per_cu": batch_tiles[1]},
                "mdot_ms": round(t_mdot, 4), "mdot_pairs_per_s": pairs / (t_mdot * 1e-3), "angular": angular}
    ba.sqrtMdotW(Wa, tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ba.sqrtMdotW(Wa, tol=1e-6)
    torch.cuda.synchronize()
    angular["sqrt_ms"] = round(1e3 * (time.perf_counter() - t0), 3)
    ita = np.array(ba.last_iterations)
    angular["lanczos_iterations"] = {"min": int(ita.min()), "median": float(np.median(ita)), "max": int(ita.max())}
    ba.close()
    del Ta, Wa
    b.sqrtMdotW(W, tol=1e-6)
    t0 = time.perf_counter()
    b.sqrtMdotW(W, tol=1e-6)
    torch.cuda.synchronize()
    t_sqrt = 1e3 * (time.perf_counter() - t0)
    iters = np.array(b.last_iterations)
    if batched_only:
        b.close()
        return {"systems": len(syss), "total_particles": int(off[-1]), "sum_n2": pairs,
                "tile_config": {"targets_per_lane": batch_tiles[0], "workgroups_per_cu": batch_tiles[1]},
                "mdot_ms": round(t_mdot, 4), "mdot_pairs_per_s": pairs / (t_mdot * 1e-3),
                "sqrt_ms": round(t_sqrt, 3),
                "lanczos_iterations": {"min": int(iters.min()), "median": float(np.median(iters)),
                                       "max": int(iters.max())}, "angular": angular}
    # one solver call per system (each system's arrays already on the device)
    sols = []
    for k, s in enumerate(syss):
        so = rpy.Solver()
        so.initialize(viscosity=s.viscosity, hydrodynamicRadius=s.radius)
        so.setPositions(X[off[k]:off[k + 1]])
        sols.append(so)
    Fs = [F[off[k]:off[k + 1]] for k in range(len(syss))]
    Ws = [W[3 * off[k]:3 * off[k + 1]] for k in range(len(syss))]
    def per_system_mdot():
        for so, f in zip(sols, Fs):
            so.Mdot(f)
    per_system_mdot()
    t_mdot_ps = timed(per_system_mdot, 3, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_ps = []
    for so, w in zip(sols, Ws):
        so.sqrtMdotW(w, tol=1e-6)
        it_ps.append(so.last_iterations)
    torch.cuda.synchronize()
    t_sqrt_ps = 1e3 * (time.perf_counter() - t0)
    for so in sols:
        so.close()
    b.close()
    return {"systems": len(syss), "total_particles": int(off[-1]), "sum_n2": pairs,
            "tile_config": {"targets_per_lane": batch_tiles[0], "workgroups_per_cu": batch_tiles[1]},
            "mdot_ms": round(t_mdot, 4), "mdot_pairs_per_s": pairs / (t_mdot * 1e-3),
            "mdot_per_system_launches_ms": round(t_mdot_ps, 3),
            "sqrt_ms": round(t_sqrt, 3), "sqrt_per_system_launches_ms": round(t_sqrt_ps, 3),
            "lanczos_iterations": {"min": int(iters.min()), "median": float(np.median(iters)),
                                   "max": int(iters.max())},
            "per_system_lanczos_iterations_median": float(np.median(it_ps)), "angular": angular}


def oracle_timings(workloads, pairloop):
    """Seconds of the other oracle routes on the host (context for the
    GPU numbers, not targets): dense float64 assembly + product at N = 1024
    and N = 4096 (translational), the oracle's Lanczos square root at
    N = 1024 (tol 1e-6), and the C pair loop on 1024 sampled rows of the
    1,048,576-bead chains (with torques)."""
    import numpy as np
    from oracle import lanczos as olz, mobility as omob
    out = {}
    c1 = workloads.c1_small_fp64()
    t0 = time.perf_counter()
    m = omob.grand_mobility(c1.pos, c1.radius, c1.viscosity)
    u = m @ c1.forces.reshape(-1)
    out["n1024_dense_assembly_and_product_s"] = round(time.perf_counter() - t0, 3)
    c4096 = workloads.uniform_cube(4096, 0.1, 1001)
    t0 = time.perf_counter()
    m4 = omob.grand_mobility(c4096.pos, c4096.radius, c4096.viscosity)
    u4 = m4 @ c4096.forces.reshape(-1)
    out["n4096_dense_assembly_and_product_s"] = round(time.perf_counter() - t0, 3)
    del m4, u4
    w = np.random.default_rng(1001).standard_normal(3 * c1.n)
    t0 = time.perf_counter()
    _, info = olz.lanczos_sqrt(lambda v: m @ v, w, tol=1e-6)
    out["n1024_lanczos_s"] = round(time.perf_counter() - t0, 3)
    out["n1024_lanczos_iterations"] = info.iters
    c5 = workloads.c5_chains()
    rows = c5.extra["subset"][:1024]
    t0 = time.perf_counter()
    pairloop.mdot_rows(c5.pos, rows, c5.forces, c5.torques, c5.radius, c5.viscosity)
    dt = time.perf_counter() - t0
    out["chains_1024_rows_s"] = round(dt, 3)
    out["chains_rows_pairs_per_s"] = len(rows) * float(c5.n) / dt
    del u
    return out


def host_cpu_model():
    """The host CPU's model name from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def timed(fn, reps, stream, warmup=0):
    """Median milliseconds of fn() over reps runs after `warmup` untimed
    runs, HIP events on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def run_breakdown(args, rpy, s, g_u, g_w, dev_t, stream):
    """float32 and float64 Mdot and backward, translational and angular, on
    suspension s (tiles from --tiles, else autotuned); timings and results."""
    import torch
    n = s.n
    breakdown, results = {}, {}
    for dt, name in (() if args.no_breakdown else ((torch.float32, "fp32"), (torch.float64, "fp64"))):
        Xd, Fd, Td = dev_t(s.pos, dt), dev_t(s.forces, dt), dev_t(s.torques, dt)
        GUd, GWd = dev_t(g_u, dt), dev_t(g_w, dt)
        for ang in (False, True):
            so = rpy.Solver()
            so.initialize(viscosity=s.viscosity, hydrodynamicRadius=s.radius, includeAngular=ang)
            so.setPositions(Xd)
            if args.tiles:
                so.setTileConfig(ang, *(int(v) for v in args.tiles.split(",")))
            else:
                so.autotune(args.tile_cache)
            key = f"{name}_{'angular' if ang else 'linear'}"
            fwd = lambda: so.Mdot(forces=Fd, torques=Td if ang else None)
            bwd = lambda: so.Mdot_backward(Fd, Td if ang else None, GUd, GWd if ang else None)
            tf = timed(fwd, 10, stream, warmup=3)
            tb = timed(bwd, 10, stream, warmup=3)
            breakdown[key] = {"mdot_ms": round(tf, 4), "pairs_per_s": float(n) * n / (tf * 1e-3),
                              "backward_ms": round(tb, 4), "backward_over_forward": round(tb / tf, 3),
                              "tiles": list(so.tileConfig(ang))}
            lin, angv = fwd()
            gp, gf, gt = bwd()
            results[key] = (lin.double().cpu().numpy(), None if angv is None else angv.double().cpu().numpy(),
                            gp.double().cpu().numpy(), gf.double().cpu().numpy())
            so.close()
    return breakdown, results


def bench_pse(rpy, workloads, dev, stream, sizes=((1 << 20, 0.1), (1 << 17, 0.1), (1 << 17, 0.001)), tol=1e-4):
    """Triply periodic products (PSE, forces only) on the paper's timing
    workload: uniform random particles in a cubic box at number density
    rho = N / V (0.1 and 0.001 / a^3), automatic splitting, tolerance 1e-4;
    Mdot and the split fluctuations (Lanczos on the real part, tol 1e-6)."""
    import torch
    out = {"workload": "uniform random particles in a cubic periodic box, a = 1, eta = 1/(6 pi), forces N(0, 1); "
                       "automatic psi, tolerance 1e-4", "tolerance": tol}
    for n, rho in sizes:
        s = workloads.periodic_box(n, 1010, density=rho, w=True, images=False)
        res = {"n": n, "density": rho, "box": round(s.extra["box"][0], 3)}
        for dt, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            so = rpy.Solver("periodic", "periodic", "periodic")
            L = s.extra["box"]
            so.setParameters(Lx=L[0], Ly=L[1], Lz=L[2], tolerance=tol)
            so.initialize(viscosity=s.viscosity, hydrodynamicRadius=s.radius)
            so.setPositions(torch.tensor(s.pos, dtype=dt, device=dev))
            info = so.pseInfo()
            Fd = torch.tensor(s.forces, dtype=dt, device=dev)
            tf = timed(lambda: so.Mdot(forces=Fd), 10, stream, warmup=2)
            r = {"mdot_ms": round(tf, 4), "particles_per_s": n / (tf * 1e-3)}
            if name == "fp32":
                res.update({"grid": list(info["grid"]), "xi": round(info["xi"], 4), "rc": round(info["rc"], 3),
                            "support": info["support"]})
                Wd = torch.tensor(s.w, dtype=dt, device=dev)
                noise = torch.randn(so.waveNoiseShape(), dtype=dt, device=dev)
                t0 = time.perf_counter()
                so.sqrtMdotWSplit(Wd, noise, tol=1e-6)
                torch.cuda.synchronize()
                r.update({"sqrt_split_ms": round(1e3 * (time.perf_counter() - t0), 2),
                          "sqrt_split_real_iterations": so.last_iterations})
            res[name] = r
            so.close()
        out[f"n{n}_rho{rho:g}"] = res
        print(f"bench: pse {res}", file=sys.stderr, flush=True)
    return out


def bench_sweep(rpy, workloads, dev, stream, sizes=None):
    """One translational float32 Mdot per size, N = 2^10 .. 2^20, uniform cubes
    at number density rho = 0.1 and 0.001 per a^3 (volume fractions 0.419 and
    0.0042), forces N(0, 1): median of timed products (at least 3, about
    0.3 s per size) after two warm-ups, with autotuned tiles up to N = 2^16;
    above, where tuning would take longer than the sweep, the faster of the
    default tiles and the symmetric mode (both reported)."""
    import numpy as np
    import torch
    out = []
    for rho in (0.1, 0.001):
        phi = rho * 4.0 / 3.0 * math.pi
        for n in (sizes or [1 << e for e in range(10, 21)]):
            e = max(0, int(n).bit_length() - 1)
            c = workloads.uniform_cube(n, phi, 2000 + e)
            sol = rpy.Solver()
            sol.initialize(viscosity=c.viscosity, hydrodynamicRadius=c.radius, includeAngular=False)
            sol.setPositions(torch.tensor(c.pos, dtype=torch.float32, device=dev))
            F = torch.tensor(c.forces, dtype=torch.float32, device=dev)
            if n <= 1 << 16:
                sol.autotune()
            configs = [sol.tileConfig(False)] + ([(0, 0)] if n > 1 << 16 else [])
            by_cfg = {}
            for cfg in configs:
                sol.setTileConfig(False, *cfg)
                t1 = timed(lambda: sol.Mdot(forces=F), 1, stream, warmup=2)
                reps = int(min(50, max(3, 300.0 / max(t1, 1e-3))))
                by_cfg[tuple(cfg)] = (timed(lambda: sol.Mdot(forces=F), reps, stream), reps)
            best = min(by_cfg, key=lambda k: by_cfg[k][0])
            t, reps = by_cfg[best]
            row = {"n": n, "rho": rho, "phi": round(phi, 5), "mdot_ms": round(t, 4), "tiles": list(best),
                   "pairs_per_s": float(n) * n / (t * 1e-3), "reps": reps,
                   "guide_4e-12_n2_ms": round(4e-12 * n * n * 1e3, 4)}
            if len(by_cfg) > 1:
                row["mdot_ms_by_tiles"] = {f"{k[0]},{k[1]}": round(v[0], 4) for k, v in by_cfg.items()}
            out.append(row)
            print(f"bench: sweep rho={rho} N={n}: {t:.3f} ms", file=sys.stderr, flush=True)
            sol.close()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: the solver runs on a single GPU (asked for {args.gpus}); "
              "sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_02135_amd as rpy
    from paper_2510_02135_amd import _lib
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    if args.sweep:
        sweep = bench_sweep(rpy, workloads, dev, stream,
                            [int(v) for v in args.sweep_sizes.split(",")] if args.sweep_sizes else None)
        print(json.dumps({"metric": "Mdot time against N (translational, float32)", "unit": "ms",
                          "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "uniform cubes, N = 2^10 .. 2^20, number density 0.1 and 0.001 "
                                                 "per a^3, a = 1, eta = 1/(6 pi), seeds 2010 .. 2020"},
                          "sweep": sweep}), flush=True)
        return
    if args.chains_solve:
        c5 = workloads.c5_chains()
        sc = rpy.Solver()
        sc.initialize(viscosity=c5.viscosity, hydrodynamicRadius=c5.radius, includeAngular=True)
        sc.setPositions(torch.tensor(c5.pos, dtype=torch.float32, device=dev))
        sc.setTileConfig(True, 0, 0)
        Wc = torch.tensor(c5.w, dtype=torch.float32, device=dev)
        res = {}
        for name in ("preconditioned", "plain"):
            print(f"bench: chains sqrtMdotW {name}", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "plain":
                sc.sqrtMdotW(Wc, tol=1e-6, maxIter=1000)
            else:
                sc.sqrtMdotWPrecond(Wc, groupSize=256, tol=1e-6, maxIter=1000)
            torch.cuda.synchronize()
            res[name] = {"seconds": round(time.perf_counter() - t0, 2), "iterations": sc.last_iterations,
                         "increment": sc.last_increment}
            print(f"bench: {name} {res[name]}", file=sys.stderr, flush=True)
        print(json.dumps({"metric": "sqrtMdotW of the bead chains, converged (tol 1e-6)", "unit": "s",
                          "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "4096 random-walk chains x 256 beads (N = 1,048,576), bond 2.1a, "
                                                 "phi 0.05, seed 1005, torques, 6N noise; symmetric pair mode; "
                                                 "preconditioner: one chain (256 beads) per group"},
                          "chains_solve": res}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"metric": "batched systems: Mdot and sqrtMdotW time (float32)", "unit": "ms",
                          "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "512 systems, N log-uniform in [64, 8192], phi in [0.05, 0.3], "
                                                 "seed 1004"},
                          "batched": bench_batched(rpy, workloads, dev, stream, timed,
                                                   mdot_only=args.batch_only == "mdot",
                                                   batched_only=args.batch_only == "batched")}), flush=True)
        return
    pse_kw = {}
    if args.pse_size:
        n_s, rho_s = args.pse_size.split(":")
        pse_kw["sizes"] = ((int(n_s), float(rho_s)),)
    if args.pse_only:
        print(json.dumps({"metric": "periodic (PSE) Mdot throughput", "unit": "particles/s",
                          "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "uniform random particles, cubic periodic box, density 0.1 and "
                                                 "0.001 / a^3, tolerance 1e-4, automatic psi"},
                          "periodic_pse": bench_pse(rpy, workloads, dev, stream, **pse_kw)}), flush=True)
        return
    s = workloads.c2_suspension(args.n)
    n = s.n
    rng = np.random.default_rng(4242)
    g_u, g_w = rng.standard_normal((2, n, 3))

    def dev_t(x, dt):
        return torch.tensor(np.asarray(x), dtype=dt, device=dev)

    if args.breakdown_only:
        bd, _ = run_breakdown(args, rpy, s, g_u, g_w, dev_t, stream)
        print(json.dumps({"metric": "Mdot and backward times, float32 and float64", "unit": "ms",
                          "higher_is_better": False, "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic",
                          "config": {"workload": f"uniform-cube suspension N={n}, phi=0.1, seed 1002",
                                     "tiles": args.tiles or "autotuned"},
                          "breakdown": bd}), flush=True)
        return
    f32 = torch.float32
    X, F, T, W = (dev_t(v, f32) for v in (s.pos, s.forces, s.torques, s.w))
    GU, GW = dev_t(g_u, f32), dev_t(g_w, f32)
    sol = rpy.Solver("open", "open", "open")
    sol.initialize(viscosity=s.viscosity, hydrodynamicRadius=s.radius, includeAngular=True)
    sol.setPositions(X)
    if args.tiles:
        fixed = tuple(int(v) for v in args.tiles.split(","))
        sol.setTileConfig(False, *fixed)
        sol.setTileConfig(True, *fixed)
        tiles = (fixed, fixed)
    else:
        print("bench: autotuning the pair kernel tiles", file=sys.stderr, flush=True)
        tiles = sol.autotune(args.tile_cache)
    if tiles[1][0] == 0:   # the symmetric pair mode (each unordered pair once)
        kernel_name = "sym_kernel<float, FwdPairs<float, true>>"
        span = tiles[1][1]
        span_text = ("automatic span" if span == 0 else
                     f"{span} source block{'s' if span > 1 else ''} per task")
        kernel_label = f"{kernel_name} (angular, symmetric mode, {span_text})"
    else:
        kernel_name = f"pair_kernel<float, true, {tiles[1][0]}>"
        kernel_label = f"{kernel_name} (angular, {tiles[1][1]} source splits)"

    iters = []

    def step():
        sol.Mdot(forces=F, torques=T)
        sol.sqrtMdotW(W, prefactor=1.0, tol=1e-6, maxIter=500)
        iters.append(sol.last_iterations)
        sol.divM()
        sol.Mdot_backward(F, T, GU, GW)

    print(f"bench: N={n} warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    iters.clear()
    _lib.rpy_enable_timing(sol._h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        print(f"bench: step {k + 1}/{args.steps} done ({iters[-1]} Lanczos iterations)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pair_ms, pair_launches, pair_pairs = _lib.rpy_kernel_time(sol._h, "pair")
    adj_ms, adj_launches, _ = _lib.rpy_kernel_time(sol._h, "adjoint")
    cgs_ms, cgs_records, cgs_bytes = _lib.rpy_kernel_time(sol._h, "lanczos_cgs")
    _lib.rpy_enable_timing(sol._h, False)
    ms_per_step = 1e3 * elapsed / args.steps
    products = sum(1 + k for k in iters)
    value = float(n) * float(n) * products / elapsed

    # dominant kernel: the float32 angular pair kernel (every M product of the step)
    avg_pair_ms = pair_ms / max(pair_launches, 1)
    achieved = FLOPS_PER_PAIR["angular"] * float(n) * float(n) / (avg_pair_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": hbm_traffic(kernel_name, n, tiles[1]),
                "kernel": kernel_label,
                "avg_launch_ms": round(avg_pair_ms, 4),
                "launches": pair_launches, "flops_per_pair": FLOPS_PER_PAIR["angular"],
                "flops_counted_per": "ordered pair of the direct formulation (N^2 per product)"}
    if tiles[1][0] == 0:
        roofline["note"] = ("symmetric mode: each unordered pair's geometry is evaluated once, so the kernel "
                            "executes fewer flops than counted; achieved is its effective rate")

    # Lanczos vector operations: the two classical Gram-Schmidt passes of
    # every iteration (HBM-bound), algorithmic bytes over their event time
    cgs_gbps = cgs_bytes / (cgs_ms * 1e-3) / 1e9 if cgs_ms > 0 else None
    lanczos_cgs = {"bound": "hbm", "achieved": None if cgs_gbps is None else round(cgs_gbps, 1),
                   "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                   "frac": None if cgs_gbps is None else round(cgs_gbps / PEAK_HBM_GBPS, 4),
                   "iterations_timed": cgs_records, "ms_per_step": round(cgs_ms / args.steps, 3),
                   "bytes_per_step": cgs_bytes / args.steps}

    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- breakdown outside the timed steps -------------------------------
    print("bench: breakdown (fp32/fp64 Mdot, backward)", file=sys.stderr, flush=True)
    breakdown, results = run_breakdown(args, rpy, s, g_u, g_w, dev_t, stream)

    # ---- the N = 16,384, phi = 0.2 gradient workload: loss
    # 0.5 |M(X) F - M(X + delta) F|^2, its backward against the forward
    grad_c3 = None
    if not args.no_breakdown:
        print("bench: N=16384 phi=0.2 backward vs forward", file=sys.stderr, flush=True)
        c3 = workloads.c3_gradient()
        grad_c3 = {"workload": f"{c3.name}: uniform cube, seed 1003, translational, target M(X + delta) F"}
        for dt, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            so = rpy.Solver()
            so.initialize(viscosity=c3.viscosity, hydrodynamicRadius=c3.radius, includeAngular=False)
            Fd = dev_t(c3.forces, dt)
            so.setPositions(dev_t(c3.pos + c3.extra["delta"], dt))
            target = so.Mdot(forces=Fd)[0].clone()
            so.setPositions(dev_t(c3.pos, dt))
            so.autotune(args.tile_cache)
            g = (so.Mdot(forces=Fd)[0] - target).contiguous()
            tf = timed(lambda: so.Mdot(forces=Fd), 10, stream, warmup=3)
            tb = timed(lambda: so.Mdot_backward(Fd, None, g, None), 10, stream, warmup=3)
            grad_c3[name] = {"mdot_ms": round(tf, 4), "backward_ms": round(tb, 4),
                              "backward_over_forward": round(tb / tf, 3)}
            so.close()

    # ---- single wall (NBody with a no-slip wall): N = 32,768 particles in a
    # layer above the wall (the size of the paper's rollers example) ------
    wall_res = None
    if not args.no_breakdown:
        print("bench: single-wall products N=32768", file=sys.stderr, flush=True)
        ws = workloads.wall_suspension(32768, 1008, hg=1.5, phi2d=0.35, torques=True, w=True, angular_w=True)
        wall_res = {"workload": f"{ws.name}: in-plane packing 0.35, heights a + Exp(0.5a), 5 % overlapping the wall",
                    "n": ws.n, "flops_per_pair": FLOPS_PER_WALL_PAIR}
        for dt, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            for ang in (False, True):
                so = rpy.Solver("open", "open", "single_wall")
                so.setParameters(wallHeight=0.0)
                so.initialize(viscosity=ws.viscosity, hydrodynamicRadius=ws.radius, includeAngular=ang)
                so.setPositions(dev_t(ws.pos, dt))
                Fd = dev_t(ws.forces, dt)
                Td = dev_t(ws.torques, dt) if ang else None
                tf = timed(lambda: so.Mdot(forces=Fd, torques=Td), 10, stream, warmup=2)
                key = f"{name}_{'angular' if ang else 'linear'}"
                fl = FLOPS_PER_WALL_PAIR["angular" if ang else "linear"]
                pk = PEAK_FP32_TFLOPS if dt == torch.float32 else PEAK_FP64_TFLOPS
                tfl = fl * float(ws.n) ** 2 / (tf * 1e-3) / 1e12
                wall_res[key] = {"mdot_ms": round(tf, 4), "pairs_per_s": float(ws.n) ** 2 / (tf * 1e-3),
                                 "tflops": round(tfl, 2), "frac_of_peak": round(tfl / pk, 4)}
                if ang and dt == torch.float32:
                    t0 = time.perf_counter()
                    so.sqrtMdotW(dev_t(ws.w, dt), tol=1e-6)
                    torch.cuda.synchronize()
                    wall_res[key].update({"sqrt_ms": round(1e3 * (time.perf_counter() - t0), 1),
                                          "sqrt_iterations": so.last_iterations})
                so.close()

    # ---- triply periodic box (PSE) on the paper's timing workload ----------
    pse = None
    if not args.no_breakdown:
        print("bench: periodic products", file=sys.stderr, flush=True)
        pse = bench_pse(rpy, workloads, dev, stream)

    # ---- several vectors at one geometry (float32, 8 force sets; 4 noise
    # vectors) against one call per vector --------------------------------
    multi = None
    if not args.no_breakdown:
        print("bench: multi-vector products", file=sys.stderr, flush=True)
        multi = {"nrhs_mdot": 8, "nrhs_sqrt": 4}
        rng = np.random.default_rng(1006)
        Xd = dev_t(s.pos, torch.float32)
        for ang in (False, True):
            so = rpy.Solver()
            so.initialize(viscosity=s.viscosity, hydrodynamicRadius=s.radius, includeAngular=ang)
            so.setPositions(Xd)
            so.autotune(args.tile_cache)
            Fm = dev_t(rng.standard_normal((8, n, 3)), torch.float32)
            Tm = dev_t(rng.standard_normal((8, n, 3)), torch.float32) if ang else None
            tm = timed(lambda: so.MdotMulti(Fm, Tm), 5, stream, warmup=2) / 8
            single = breakdown["fp32_" + ("angular" if ang else "linear")]["mdot_ms"]
            key = "angular" if ang else "linear"
            multi[f"mdot_{key}_ms_per_vector"] = round(tm, 4)
            multi[f"mdot_{key}_pair_vectors_per_s"] = float(n) * n / (tm * 1e-3)
            multi[f"mdot_{key}_speedup_vs_single"] = round(single / tm, 3)
            if ang:
                Wm = dev_t(rng.standard_normal((4, 6 * n)), torch.float32)
                t0 = time.perf_counter()
                its_single = []
                for r in range(4):
                    so.sqrtMdotW(Wm[r], tol=1e-6)
                    its_single.append(so.last_iterations)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                so.sqrtMdotWMulti(Wm, tol=1e-6)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                multi.update({"sqrt_angular_singles_ms": round(1e3 * (t1 - t0), 1),
                              "sqrt_angular_multi_ms": round(1e3 * (t2 - t1), 1),
                              "sqrt_iterations": so.last_iterations, "sqrt_iterations_single": its_single})
            so.close()
            del Fm, Tm

    # ---- bead chains, N = 1,048,576: one angular float32 product, with the
    # default tiles and with the symmetric mode (tuning would take longer
    # than the product), the faster reported --------------------------------
    chains = None
    if not args.no_batch:
        print("bench: bead chains N=1048576", file=sys.stderr, flush=True)
        c5 = workloads.c5_chains()
        sc = rpy.Solver()
        sc.initialize(viscosity=c5.viscosity, hydrodynamicRadius=c5.radius, includeAngular=True)
        sc.setPositions(dev_t(c5.pos, torch.float32))
        Fc, Tc = dev_t(c5.forces, torch.float32), dev_t(c5.torques, torch.float32)
        by_cfg = {}
        for cfg in (tuple(sc.tileConfig(True)), (0, 0)):
            sc.setTileConfig(True, *cfg)
            by_cfg[cfg] = timed(lambda: sc.Mdot(forces=Fc, torques=Tc), 2, stream, warmup=1)
        best = min(by_cfg, key=by_cfg.get)
        tc = by_cfg[best]
        sc.setTileConfig(True, *best)
        chains = {"n": c5.n, "workload": "4096 random-walk chains x 256 beads, bond 2.1a, phi 0.05, seed 1005",
                  "mdot_angular_fp32_ms": round(tc, 3), "pairs_per_s": float(c5.n) ** 2 / (tc * 1e-3),
                  "tiles": list(best), "mdot_ms_by_tiles": {f"{k[0]},{k[1]}": round(v, 3) for k, v in by_cfg.items()}}
        # one backward pass (cotangents N(0, 1), seed 1007)
        print("bench: bead chains backward", file=sys.stderr, flush=True)
        gcu, gcw = (dev_t(v, torch.float32) for v in np.random.default_rng(1007).standard_normal((2, c5.n, 3)))
        tb = timed(lambda: sc.Mdot_backward(Fc, Tc, gcu, gcw), 1, stream, warmup=1)
        chains.update({"backward_ms": round(tb, 3), "backward_over_forward": round(tb / tc, 3)})
        del gcu, gcw
        # Lanczos run for a fixed number of iterations (the tol-1e-6 solve takes
        # hundreds): time per iteration, and the bytes of its Gram-Schmidt passes
        kfix = args.chains_lanczos_iters
        print(f"bench: bead chains Lanczos, {kfix} iterations", file=sys.stderr, flush=True)
        Wc = dev_t(c5.w, torch.float32)
        _lib.rpy_enable_timing(sc._h, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            sc.sqrtMdotW(Wc, tol=1e-15, maxIter=kfix)
        except rpy.NotConvergedError:
            pass
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        cp_ms, cp_n, _ = _lib.rpy_kernel_time(sc._h, "pair")
        cg_ms, cg_rec, cg_bytes = _lib.rpy_kernel_time(sc._h, "lanczos_cgs")
        _lib.rpy_enable_timing(sc._h, False)
        chains.update({"lanczos_iterations": kfix, "lanczos_ms": round(1e3 * tl, 1),
                       "lanczos_ms_per_iteration": round(1e3 * tl / kfix, 2),
                       "lanczos_pair_kernel_ms_per_product": round(cp_ms / max(cp_n, 1), 2),
                       "lanczos_cgs_ms": round(cg_ms, 2), "lanczos_cgs_bytes": cg_bytes,
                       "lanczos_cgs_gbps": round(cg_bytes / (cg_ms * 1e-3) / 1e9, 1) if cg_ms > 0 else None})
        sc.close()
        del Fc, Tc, Wc

    # ---- batched systems: one persistent launch vs one launch per system ----
    batched = None
    if not args.no_batch:
        print("bench: batched systems", file=sys.stderr, flush=True)
        batched = bench_batched(rpy, workloads, dev, stream, timed)

    # ---- accuracy against the float64 oracle on sampled particles --------
    print("bench: oracle check on sampled rows", file=sys.stderr, flush=True)
    from oracle import gradient, pairloop
    rows = s.extra["subset"][:256]
    acc = {}
    for key, (lin, angv, gp, gf) in results.items():
        dt = np.float32 if key.startswith("fp32") else np.float64
        xr = s.pos.astype(dt).astype(np.float64)
        fr = s.forces.astype(dt).astype(np.float64)
        tr = s.torques.astype(dt).astype(np.float64) if angv is not None else None
        u, w = pairloop.mdot_rows(xr, rows, fr, tr, s.radius, s.viscosity)
        e = emax(lin[rows], u)
        if angv is not None:
            e = max(e, emax(angv[rows], w))
        gur = g_u.astype(dt).astype(np.float64)
        gwr = g_w.astype(dt).astype(np.float64) if angv is not None else None
        mg, _ = pairloop.mdot_rows(xr, rows[:64], gur, gwr, s.radius, s.viscosity)
        gx = gradient.grad_positions(xr, fr, tr, gur, gwr, s.radius, s.viscosity, rows=rows[:8])
        acc[key] = {"mdot_emax": e, "backward_dF_emax": emax(gf[rows[:64]], mg),
                    "backward_dX_emax": emax(gp[rows[:8]], gx)}

    # sqrtMdotW against the oracle at N = 1024 (phi = 0.1, with torques), where
    # the oracle's Lanczos and the exact root are affordable on the host
    if not args.no_breakdown:
        from oracle import lanczos as olz, mobility as omob
        small = workloads.uniform_cube(1024, 0.1, 1001, torques=True, w=True, angular_w=True)
        for dt, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            so = rpy.Solver()
            so.initialize(viscosity=small.viscosity, hydrodynamicRadius=small.radius, includeAngular=True)
            so.setPositions(dev_t(small.pos, dt))
            ylin, yang = so.sqrtMdotW(dev_t(small.w, dt), tol=1e-6)
            k = so.last_iterations
            y = np.concatenate([ylin.double().cpu().numpy().reshape(-1), yang.double().cpu().numpy().reshape(-1)])
            npd = np.float32 if dt == torch.float32 else np.float64
            xr = small.pos.astype(npd).astype(np.float64)
            wr = small.w.astype(npd).astype(np.float64)
            m = omob.grand_mobility(xr, small.radius, small.viscosity, angular=True)
            y_ref, _ = olz.lanczos_sqrt(lambda v: m @ v, wr, iters=k)
            exact = olz.exact_sqrt_mdot_w(m, wr)
            acc.setdefault(f"{name}_sqrtMdotW_n1024", {})
            acc[f"{name}_sqrtMdotW_n1024"] = {
                "iterations": k,
                "matched_iteration_emax": emax(y.reshape(-1, 3), y_ref.reshape(-1, 3)),
                "vs_exact_root_rel": float(np.linalg.norm(y - exact) / np.linalg.norm(exact))}
            so.close()

    # ---- CPU oracle baseline on a bounded sample --------------------------
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        probe = s.extra["subset"][:64]
        t1 = time.perf_counter()
        pairloop.mdot_rows(s.pos, probe, s.forces, s.torques, s.radius, s.viscosity)
        rate = len(probe) * n / (time.perf_counter() - t1)
        m = int(min(n, max(64, args.cpu_seconds * rate / n)))
        sample = np.sort(np.random.default_rng(7).choice(n, size=m, replace=False))
        reps = 0
        t1 = time.perf_counter()
        while True:   # whole passes over the sample until cpu_seconds have passed
            pairloop.mdot_rows(s.pos, sample, s.forces, s.torques, s.radius, s.viscosity)
            reps += 1
            dt_cpu = time.perf_counter() - t1
            if dt_cpu >= args.cpu_seconds:
                break
        cpu = {"value": reps * m * float(n) / dt_cpu, "unit": "pair-interactions/s", "cores": pairloop.threads(),
               "kind": "oracle",
               "sample": f"{reps} x ({m} target rows x {n} sources) of the same workload, linear+angular Mdot, "
                         f"float64 C/OpenMP pair loop ({dt_cpu:.1f} s)",
               "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count()}
        cpu["other_oracle_timings"] = oracle_timings(workloads, pairloop)
        # the step's products at the oracle's rate (extrapolated from the sample, not run)
        cpu["other_oracle_timings"]["step_products_extrapolated_s"] = round(products / args.steps * float(n) * n
                                                                            / cpu["value"], 1)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"uniform-cube suspension N={n}, phi=0.1, a=1, eta=1/(6 pi), seed 1002; "
                               "float32 pairs: Mdot(F,T) + sqrtMdotW(W, tol 1e-6, float64 Lanczos) + divM + "
                               "Mdot_backward(F,T,gU,gW)",
                   "n": n, "lanczos_iterations": iters, "m_products_per_step": products / args.steps},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "lanczos_vector_ops": lanczos_cgs,
        "breakdown": breakdown,
        "gradient_n16384": grad_c3,
        "single_wall_n32768": wall_res,
        "periodic_pse": pse,
        "accuracy_vs_fp64_oracle": acc,
        "batched": batched,
        "chains": chains,
        "multi_vector": multi,
        "tiles": {"linear": tiles[0], "angular": tiles[1]},
        "adjoint_kernel_avg_ms": round(adj_ms / max(adj_launches, 1), 4),
    }
    sol.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

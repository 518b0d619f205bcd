"""Seeded synthetic inputs for the open-boundary RPY mobility path.

This module only draws random numbers and lays them out; it holds none of the
mobility arithmetic.  Both the HIP path (through its tests and the benchmark)
and the CPU oracle are fed from here, so the two sides always see the same
numbers.

Recipe shared by every workload:

* generator ``numpy.random.default_rng(seed)`` (PCG64);
* draw order: positions, then forces, then torques, then the noise vector W,
  then any subset / perturbation indices;
* particles of radius ``a`` are placed uniformly in a cube centred at the
  origin, ``[-L/2, L/2)^3`` with ``L = (N (4/3) pi a^3 / phi)^(1/3)``;
  overlaps are allowed, as in the paper's timing benchmark (Sec. 5.5);
* forces, torques and W are i.i.d. standard normal;
* float32 arrays are the float64 draws rounded once.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Unit choice of every workload: radius 1 and viscosity 1/(6 pi), so that the
# single-particle translational mobility 1/(6 pi eta a) equals 1.
RADIUS = 1.0
VISCOSITY = 1.0 / (6.0 * math.pi)


def cube_side(n: int, phi: float, a: float = RADIUS) -> float:
    """Side of the cube holding ``n`` spheres of radius ``a`` at volume fraction ``phi``."""
    return (n * (4.0 / 3.0) * math.pi * a ** 3 / phi) ** (1.0 / 3.0)


@dataclass
class Suspension:
    """One synthetic system: the float64 draws (float32 users round them once)."""
    name: str
    pos: np.ndarray                       # (N, 3) float64
    forces: np.ndarray                    # (N, 3) float64
    torques: np.ndarray | None = None     # (N, 3) float64
    w: np.ndarray | None = None           # (3N,) or (6N,) float64
    radius: float = RADIUS
    viscosity: float = VISCOSITY
    box: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def uniform_cube(n: int, phi: float, seed: int, *, torques: bool = False,
                 w: bool = False, angular_w: bool = False,
                 a: float = RADIUS, name: str = "") -> Suspension:
    """Uniform random suspension; draw order positions, forces, torques, W."""
    rng = np.random.default_rng(seed)
    side = cube_side(n, phi, a)
    pos = (rng.random((n, 3)) - 0.5) * side
    forces = rng.standard_normal((n, 3))
    tq = rng.standard_normal((n, 3)) if torques else None
    wv = rng.standard_normal(6 * n if angular_w else 3 * n) if w else None
    s = Suspension(name or f"cube_n{n}_phi{phi}_s{seed}", pos, forces, tq, wv,
                   radius=a, box=side)
    s.extra["rng"] = rng
    return s


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def c1_small_fp64() -> Suspension:
    """N=1024, phi=0.1, seed 1001: translational product in float64."""
    return uniform_cube(1024, 0.1, 1001, name="c1_n1024_phi0.1")


def c2_suspension(n: int = 65536) -> Suspension:
    """N=65,536, phi=0.1, seed 1002: forces, torques and a 6N noise vector.

    ``extra['subset']`` holds 4096 target indices drawn without replacement
    (drawn last, after W).
    """
    s = uniform_cube(n, 0.1, 1002, torques=True, w=True, angular_w=True,
                     name=f"c2_n{n}_phi0.1")
    rng = s.extra.pop("rng")
    s.extra["subset"] = np.sort(rng.choice(n, size=min(4096, n), replace=False))
    return s


def c3_gradient(n: int = 16384) -> Suspension:
    """N=16,384, phi=0.2, seed 1003: loss 0.5*||M(X)F - U*||^2.

    After positions and forces the generator draws the perturbation
    ``delta ~ N(0, (0.1 a)^2)`` (N x 3) that defines the target configuration
    X + delta, then 64 (particle, axis) coordinates and 64 force coordinates
    (flat indices into N x 3, without replacement).
    """
    rng = np.random.default_rng(1003)
    side = cube_side(n, 0.2)
    pos = (rng.random((n, 3)) - 0.5) * side
    forces = rng.standard_normal((n, 3))
    delta = 0.1 * RADIUS * rng.standard_normal((n, 3))
    fd_pos = rng.choice(3 * n, size=64, replace=False)
    fd_force = rng.choice(3 * n, size=64, replace=False)
    s = Suspension(f"c3_n{n}_phi0.2", pos, forces, None, None, box=side)
    s.extra.update(delta=delta, fd_pos=fd_pos, fd_force=fd_force)
    return s


def c4_systems(n_systems: int = 512, seed: int = 1004,
               n_min: int = 64, n_max: int = 8192) -> list[Suspension]:
    """Independent systems with N log-uniform in [n_min, n_max] and phi in [0.05, 0.3].

    One generator draws, in order: every N_s, every phi_s, then for each
    system its positions, forces and 3N noise vector.
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_systems))).astype(np.int64)
    phis = rng.uniform(0.05, 0.3, n_systems)
    out = []
    for k in range(n_systems):
        n = int(ns[k])
        side = cube_side(n, float(phis[k]))
        pos = (rng.random((n, 3)) - 0.5) * side
        forces = rng.standard_normal((n, 3))
        wv = rng.standard_normal(3 * n)
        s = Suspension(f"c4_sys{k}_n{n}", pos, forces, None, wv, box=side)
        s.extra["phi"] = float(phis[k])
        out.append(s)
    return out


def c5_chains(n_chains: int = 4096, beads: int = 256, bond: float = 2.1,
              phi: float = 0.05, seed: int = 1005) -> Suspension:
    """Random-walk bead chains: 4096 x 256 beads at bead volume fraction 0.05.

    Bond vectors have length ``bond`` (2.1 a) and directions from normalised
    N(0, I3) draws; each chain is centred on its centroid and then shifted to
    a centre uniform in the cube.  Draw order: bond directions, chain
    centres, forces, torques, W (6N).
    """
    rng = np.random.default_rng(seed)
    n = n_chains * beads
    side = cube_side(n, phi)
    dirs = rng.standard_normal((n_chains, beads - 1, 3))
    dirs /= np.linalg.norm(dirs, axis=2, keepdims=True)
    chain = np.concatenate([np.zeros((n_chains, 1, 3)), np.cumsum(bond * dirs, axis=1)], axis=1)
    chain -= chain.mean(axis=1, keepdims=True)
    centres = (rng.random((n_chains, 1, 3)) - 0.5) * side
    pos = (chain + centres).reshape(n, 3)
    forces = rng.standard_normal((n, 3))
    tq = rng.standard_normal((n, 3))
    wv = rng.standard_normal(6 * n)
    s = Suspension(f"c5_chains{n_chains}x{beads}", pos, forces, tq, wv, box=side)
    s.extra["subset"] = np.sort(rng.choice(n, size=min(4096, n), replace=False))
    return s



def wall_suspension(n: int, seed: int, *, hg: float = 1.5, phi2d: float = 0.11, overlap: float = 0.05,
                    torques: bool = False, w: bool = False, angular_w: bool = False,
                    wall_height: float = 0.0) -> Suspension:
    """Particles above a no-slip wall at z = wall_height (a monolayer-like
    layer, as in the paper's rollers and wall-diffusion examples).

    In-plane positions uniform in a square of side L = sqrt(N pi a^2 / phi2d)
    (in-plane packing fraction phi2d, centred at the origin); heights above
    the wall a + Exp(hg - a), the Gibbs-Boltzmann distribution of a
    sedimented sphere with gravitational height hg (the paper's rollers use
    hg = 1.5a and 6.1a), except a fraction ``overlap`` of the particles,
    chosen at random, whose heights are uniform in (0, a): they overlap the
    wall.  Draw order: in-plane positions, heights, overlap flags and their
    heights, forces, torques, W.
    """
    rng = np.random.default_rng(seed)
    side = math.sqrt(n * math.pi * RADIUS ** 2 / phi2d)
    xy = (rng.random((n, 2)) - 0.5) * side
    h = RADIUS + rng.exponential((hg - 1.0) * RADIUS, n)
    low = rng.random(n) < overlap
    h = np.where(low, rng.random(n) * RADIUS, h)
    pos = np.column_stack([xy, wall_height + h])
    forces = rng.standard_normal((n, 3))
    tq = rng.standard_normal((n, 3)) if torques else None
    wv = rng.standard_normal(6 * n if angular_w else 3 * n) if w else None
    s = Suspension(f"wall_n{n}_hg{hg}_s{seed}", pos, forces, tq, wv, box=side)
    s.extra.update(wall_height=wall_height)
    return s


def periodic_box(n: int, seed: int, *, box=None, density: float = 0.1, w: bool = False,
                 images: bool = True, name: str = "") -> Suspension:
    """Periodic suspension: positions uniform in the box [0, Lx) x [0, Ly) x
    [0, Lz) (cubic with side (N / density)^(1/3) when `box` is not given,
    the number density of the paper's timing benchmark, Sec. 5.5), then,
    with `images`, every particle moved by a random whole number of box
    lengths in -2..2 per axis (the same suspension, unwrapped); draw order
    positions, image shifts, forces, W (3N)."""
    rng = np.random.default_rng(seed)
    if box is None:
        side = (n / density) ** (1.0 / 3.0)
        box = (side, side, side)
    L = np.asarray(box, dtype=np.float64)
    pos = rng.random((n, 3)) * L
    shifts = rng.integers(-2, 3, (n, 3))
    if images:
        pos = pos + shifts * L
    forces = rng.standard_normal((n, 3))
    wv = rng.standard_normal(3 * n) if w else None
    s = Suspension(name or f"periodic_n{n}_s{seed}", pos, forces, None, wv, box=float(L[0]))
    s.extra["box"] = tuple(float(v) for v in L)
    return s


def wave_noise(shape, seed: int) -> np.ndarray:
    """Standard normal Fourier-space noise of the given shape (the periodic
    solver's split fluctuations), from its own generator."""
    return np.random.default_rng(seed).standard_normal(tuple(shape))

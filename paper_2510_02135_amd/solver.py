"""Python front-end with the paper's solver interface (Sec. 3.2).

``Solver`` mirrors the libMobility solver classes: constructor with per-axis
periodicity, ``setParameters``, ``initialize``, ``setPositions``, ``Mdot``,
``sqrtMdotW``, ``divM`` and ``LangevinVelocities``, each returning (linear,
angular), plus ``divM_rfd`` (one random finite difference of the drift,
eq. (rfd)).  ``AdamsBashforth`` steps eq. (bdhi) with the scheme of
Sec. 5.1.  Only torch device tensors are accepted; results are new tensors
of the input dtype on the same device.  ``mdot`` is the differentiable form:
a ``torch.autograd.Function`` whose backward calls the library's adjoint.
"""
from __future__ import annotations

import math

import torch

from . import _lib
from ._lib import NotConvergedError


class Solver:
    """RPY mobility solver on one HIP device: open boundaries;
    ("open", "open", "single_wall") for a no-slip wall at z = wallHeight
    (setParameters(wallHeight=...), default 0); or ("periodic", "periodic",
    "periodic") for a periodic box by the positively split Ewald method
    (setParameters(Lx=..., Ly=..., Lz=... or boxSize=..., psi=..., tolerance=...);
    forces only)."""

    def __init__(self, periodicityX: str = "open", periodicityY: str = "open",
                 periodicityZ: str = "open"):
        self._h = _lib.rpy_create(periodicityX, periodicityY, periodicityZ)
        self.periodicity = (periodicityX, periodicityY, periodicityZ)
        self._n = 0
        self._dtype = None
        self._device = None
        self._angular = False
        self.viscosity = None
        self.hydrodynamicRadius = None
        self.last_iterations = 0
        self.last_increment = float("nan")

    # -- configuration -----------------------------------------------------
    def setParameters(self, **params):
        for k, v in params.items():
            _lib.rpy_set_parameter(self._h, k, v)

    def initialize(self, viscosity: float, hydrodynamicRadius: float, includeAngular: bool = False):
        _lib.rpy_initialize(self._h, viscosity, hydrodynamicRadius, includeAngular)
        self.viscosity = float(viscosity)
        self.hydrodynamicRadius = float(hydrodynamicRadius)
        self._angular = bool(includeAngular)

    def setPositions(self, positions: torch.Tensor):
        pos = positions.reshape(-1, 3)
        _lib.rpy_set_positions(self._h, pos)
        self._n = pos.shape[0]
        self._dtype = pos.dtype
        self._device = pos.device

    @property
    def n(self) -> int:
        return self._n

    @property
    def dtype(self):
        return self._dtype

    @property
    def includeAngular(self) -> bool:
        return self._angular

    def _empty(self):
        return torch.empty((self._n, 3), dtype=self._dtype, device=self._device)

    def _require_positions(self):
        """Let the library report the missing positions (NO_POSITIONS)."""
        if self._n == 0:
            _lib._check(self._h, _lib.load().rpy_mdot(self._h, None, None, None, None, None))

    def _as(self, t, name):
        self._require_positions()
        if t is None:
            return None
        t = t.reshape(-1, 3)
        if t.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: {name} is {t.dtype}, positions are {self._dtype}")
        return t.contiguous()

    # -- the three terms of eq. (bdhi) --------------------------------------
    def Mdot(self, forces: torch.Tensor | None = None, torques: torch.Tensor | None = None):
        """(M_uF F + M_uT T, M_wF F + M_wT T or None)."""
        f, t = self._as(forces, "forces"), self._as(torques, "torques")
        lin = self._empty()
        ang = self._empty() if (self._angular and (t is not None or f is not None)) else None
        _lib.rpy_mdot(self._h, f, t, lin, ang, self._dtype, self._n)
        return lin, ang

    def MdotMulti(self, forces: torch.Tensor | None = None, torques: torch.Tensor | None = None):
        """Mdot for several vectors at the stored positions: forces / torques
        of shape (nrhs, N, 3); returns outputs of the same shape (angular
        None without includeAngular).  Each vector's result equals Mdot's
        (bit for bit without angular terms, to rounding with them)."""
        self._require_positions()
        ref = forces if forces is not None else torques
        if ref is None:
            _lib.rpy_mdot_multi(self._h, None, None, 1, self._empty(), None, self._dtype, self._n)
        nrhs = ref.numel() // (3 * self._n) if ref.numel() % (3 * self._n) == 0 else -1
        if nrhs < 1:
            raise ValueError(f"vectors must have shape (nrhs, {self._n}, 3)")
        f = self._as_multi(forces, "forces", nrhs)
        t = self._as_multi(torques, "torques", nrhs)
        lin = torch.empty((nrhs, self._n, 3), dtype=self._dtype, device=self._device)
        ang = torch.empty_like(lin) if self._angular else None
        _lib.rpy_mdot_multi(self._h, f, t, nrhs, lin, ang, self._dtype, self._n)
        return lin, ang

    def _as_multi(self, t, name, nrhs):
        if t is None:
            return None
        if t.numel() != 3 * self._n * nrhs:
            raise ValueError(f"{name} must have shape ({nrhs}, {self._n}, 3)")
        if t.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: {name} is {t.dtype}, positions are {self._dtype}")
        return t.reshape(nrhs, self._n, 3).contiguous()

    def sqrtMdotW(self, W: torch.Tensor | None = None, prefactor: float = 1.0,
                  tol: float = 1e-6, maxIter: int = 500, generator: torch.Generator | None = None):
        """prefactor * M^{1/2} W by Lanczos; W ~ N(0, I) is drawn when not given."""
        self._require_positions()
        dim = (6 if self._angular else 3) * self._n
        if W is None:
            W = torch.randn(dim, dtype=self._dtype, device=self._device, generator=generator)
        w = W.reshape(-1)
        if w.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: W is {w.dtype}, positions are {self._dtype}")
        w = w.contiguous()
        lin = self._empty()
        ang = self._empty() if self._angular else None
        it, inc = _lib.rpy_sqrt_mdot_w(self._h, w, prefactor, tol, maxIter, lin, ang, self._dtype,
                                       self._n, self._angular)
        self.last_iterations, self.last_increment = it, inc
        return lin, ang

    def pseInfo(self) -> dict:
        """Configuration of a periodic solver: Fourier grid, splitting xi,
        real-space cutoff rc, Gaussian width sigma and support, wave cutoff."""
        grid, xi, rc, sigma, support, kc = _lib.rpy_pse_info(self._h)
        return {"grid": grid, "xi": xi, "rc": rc, "sigma": sigma, "support": support, "kc": kc}

    def waveNoiseShape(self):
        """Shape of the Fourier-space noise of sqrtMdotWSplit: (3, Nx, Ny, Nz//2 + 1, 2)."""
        g = self.pseInfo()["grid"]
        return (3, g[0], g[1], g[2] // 2 + 1, 2)

    def sqrtMdotWSplit(self, W: torch.Tensor | None = None, waveNoise: torch.Tensor | None = None,
                       prefactor: float = 1.0, tol: float = 1e-6, maxIter: int = 500,
                       generator: torch.Generator | None = None):
        """Periodic box: prefactor * (M_real^{1/2} W + a wave-space sample drawn
        from waveNoise), a fluctuating term with covariance M built from the
        positive split (Lanczos on the near-field part only; the far field
        from independent Fourier-space normals, one inverse FFT).  W (3N) and
        waveNoise (waveNoiseShape()) ~ N(0, 1) are drawn when not given."""
        self._require_positions()
        w = self._noise(W, generator)
        shape = self.waveNoiseShape()
        if waveNoise is None:
            waveNoise = torch.randn(shape, dtype=self._dtype, device=self._device, generator=generator)
        if tuple(waveNoise.shape) != shape and waveNoise.numel() != math.prod(shape):
            raise ValueError(f"SIZE_MISMATCH: wave noise needs {shape}, got {tuple(waveNoise.shape)}")
        if waveNoise.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: wave noise is {waveNoise.dtype}, positions are {self._dtype}")
        lin = self._empty()
        it, inc = _lib.rpy_pse_sqrt_mdot_w(self._h, w, waveNoise.contiguous().reshape(-1), math.prod(shape), prefactor,
                                           tol, maxIter, lin, self._dtype, self._n)
        self.last_iterations, self.last_increment = it, inc
        return lin, None

    def sqrtMdotWPrecond(self, W: torch.Tensor | None = None, groupSize: int = 1, prefactor: float = 1.0,
                         tol: float = 1e-6, maxIter: int = 500, generator: torch.Generator | None = None):
        """prefactor * L (L^{-1} M L^{-T})^{1/2} W with L the block Cholesky factor
        of M over groups of groupSize consecutive particles: a fluctuating
        term with covariance M (not the symmetric root) that needs fewer
        Lanczos iterations when the groups hold the stiff couplings (chains,
        rigid bodies)."""
        self._require_positions()
        dim = (6 if self._angular else 3) * self._n
        if W is None:
            W = torch.randn(dim, dtype=self._dtype, device=self._device, generator=generator)
        w = W.reshape(-1)
        if w.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: W is {w.dtype}, positions are {self._dtype}")
        lin = self._empty()
        ang = self._empty() if self._angular else None
        it, inc = _lib.rpy_sqrt_mdot_w_precond(self._h, w.contiguous(), groupSize, prefactor, tol, maxIter, lin, ang,
                                               self._dtype, self._n, self._angular)
        self.last_iterations, self.last_increment = it, inc
        return lin, ang

    def sqrtMdotWMulti(self, W: torch.Tensor, prefactor: float = 1.0, tol: float = 1e-6, maxIter: int = 500):
        """prefactor * M^{1/2} W_r for the rows of W (shape (nrhs, 3N), or
        (nrhs, 6N) with angular terms), one Lanczos recurrence per row
        advanced together; each row's result and iteration count equal
        sqrtMdotW's (exactly without angular terms, to rounding with them).
        Returns outputs of shape (nrhs, N, 3);
        last_iterations becomes the list of iteration counts."""
        self._require_positions()
        dim = (6 if self._angular else 3) * self._n
        if W.numel() % dim != 0 or W.numel() == 0:
            raise ValueError(f"W must have shape (nrhs, {dim})")
        if W.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: W is {W.dtype}, positions are {self._dtype}")
        nrhs = W.numel() // dim
        w = W.reshape(nrhs, dim).contiguous()
        lin = torch.empty((nrhs, self._n, 3), dtype=self._dtype, device=self._device)
        ang = torch.empty_like(lin) if self._angular else None
        it, inc = _lib.rpy_sqrt_mdot_w_multi(self._h, w, nrhs, prefactor, tol, maxIter, lin, ang, self._dtype,
                                             self._n, self._angular)
        self.last_iterations, self.last_increment = it, inc
        return lin, ang

    def solve(self, U: torch.Tensor, Omega: torch.Tensor | None = None, tol: float = 1e-8, maxIter: int = 1000):
        """Forces (and torques) with M [F; T] = [U; Omega] by conjugate
        gradients.  U (and Omega, required with includeAngular) of shape
        (N, 3) or (nrhs, N, 3); returns arrays of the same shape.
        last_iterations / last_residual hold per-right-hand-side lists."""
        self._require_positions()
        single = U.dim() == 2
        nrhs = U.numel() // (3 * self._n) if U.numel() % (3 * self._n) == 0 else -1
        if nrhs < 1:
            raise ValueError(f"U must have shape (N, 3) or (nrhs, {self._n}, 3)")
        if self._angular and Omega is None:
            raise ValueError("includeAngular needs Omega")
        if not self._angular and Omega is not None:
            raise ValueError("Omega needs includeAngular")
        u = self._as_multi(U, "U", nrhs)
        w = self._as_multi(Omega, "Omega", nrhs) if self._angular else None
        f = torch.empty((nrhs, self._n, 3), dtype=self._dtype, device=self._device)
        t = torch.empty_like(f) if self._angular else None
        it, res = _lib.rpy_mobility_solve(self._h, u, w, nrhs, tol, maxIter, f, t, self._dtype, self._n)
        self.last_iterations, self.last_residual = it, res
        if single:
            return f[0], (t[0] if t is not None else None)
        return f, t

    def divM(self, generator: torch.Generator | None = None):
        """Thermal drift d_X . M: zero in an unbounded fluid; above a wall one
        random finite difference (divM_rfd with a drawn W), as the paper's
        default for solvers whose drift does not vanish (Sec. 3.4)."""
        self._require_positions()
        if self.periodicity[2] == "single_wall":
            return self.divM_rfd(generator=generator)
        lin = self._empty()
        ang = self._empty() if self._angular else None
        _lib.rpy_div_m(self._h, lin, ang, self._dtype, self._n)
        return lin, ang

    def divM_rfd(self, W: torch.Tensor | None = None, delta: float | None = None,
                 generator: torch.Generator | None = None):
        """One random finite difference of the drift, eq. (rfd):
        (M(X + delta/2 W_X) W - M(X - delta/2 W_X) W) / delta.  W ~ N(0, I)
        is drawn when not given (3N, or 6N with angular terms); delta
        defaults to 1e-3 a (float32) or 1e-4 a (float64)."""
        self._require_positions()
        dim = (6 if self._angular else 3) * self._n
        if W is None:
            W = torch.randn(dim, dtype=self._dtype, device=self._device, generator=generator)
        w = W.reshape(-1)
        if w.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: W is {w.dtype}, positions are {self._dtype}")
        if delta is None:
            delta = (1e-3 if self._dtype == torch.float32 else 1e-4) * self.hydrodynamicRadius
        lin = self._empty()
        ang = self._empty() if self._angular else None
        _lib.rpy_div_m_rfd(self._h, w.contiguous(), delta, lin, ang, self._dtype, self._n, self._angular)
        return lin, ang

    def LangevinVelocities(self, forces=None, torques=None, dt: float = 1.0, kBT: float = 0.0,
                           W: torch.Tensor | None = None, tol: float = 1e-6, maxIter: int = 500,
                           generator: torch.Generator | None = None):
        """Euler-Maruyama velocities of eq. (bdhi):
        M [F; T] + sqrt(2 kBT / dt) M^{1/2} W + kBT d_X . M (drift zero in
        open space).  W ~ N(0, I) is drawn when kBT > 0 and W is not given."""
        self._require_positions()
        f, t = self._as(forces, "forces"), self._as(torques, "torques")
        w = self._noise(W, generator) if kBT > 0 else None
        lin = self._empty()
        ang = self._empty() if self._angular else None
        self.last_iterations = _lib.rpy_langevin_velocities(self._h, f, t, w, dt, kBT, tol, maxIter, lin, ang,
                                                            self._dtype, self._n, self._angular)
        return lin, ang

    def _noise(self, W, generator):
        dim = (6 if self._angular else 3) * self._n
        if W is None:
            W = torch.randn(dim, dtype=self._dtype, device=self._device, generator=generator)
        w = W.reshape(-1)
        if w.dtype != self._dtype:
            raise ValueError(f"DTYPE_MISMATCH: W is {w.dtype}, positions are {self._dtype}")
        return w.contiguous()

    def Mdot_backward(self, forces, torques, grad_lin, grad_ang=None, need_pos=True,
                      need_forces=True, need_torques=True):
        """(dL/dX, dL/dF, dL/dT) for cotangents of the Mdot outputs."""
        f, t = self._as(forces, "forces"), self._as(torques, "torques")
        gl, ga = self._as(grad_lin, "grad_lin"), self._as(grad_ang, "grad_ang")
        gp = self._empty() if need_pos else None
        gf = self._empty() if need_forces else None
        gt = self._empty() if (need_torques and self._angular) else None
        _lib.rpy_mdot_backward(self._h, f, t, gl, ga, gp, gf, gt, self._dtype, self._n)
        return gp, gf, gt

    # -- tile configuration of the pair kernel ------------------------------
    def autotune(self, cache_path: str | None = None):
        """Time the pair-kernel tile candidates at the current N and keep the fastest."""
        _lib.rpy_autotune(self._h, cache_path)
        return self.tileConfig(False), (self.tileConfig(True) if self._angular else None)

    def tileConfig(self, angular: bool = False):
        """(targets per lane, source splits; 0 = automatic)."""
        return _lib.rpy_get_tile_config(self._h, angular)

    def setTileConfig(self, angular: bool, targets_per_lane: int, source_splits: int = 0):
        _lib.rpy_set_tile_config(self._h, angular, targets_per_lane, source_splits)

    def setAdjointMode(self, mode: int):
        """Pair evaluation of Mdot_backward: 0 automatic, 1 one-sided, 2 symmetric."""
        _lib.rpy_set_adjoint_mode(self._h, mode)

    def setMultiConfig(self, targets_per_lane: int):
        """Targets per lane (0 = automatic, 1 or 2) of the multi-vector pair kernel."""
        _lib.rpy_set_multi_config(self._h, targets_per_lane)

    def close(self):
        if getattr(self, "_h", None):
            _lib.rpy_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent open-boundary systems solved together.

    System s owns rows offsets[s]:offsets[s+1] of the concatenated (total, 3)
    positions / forces / torques / outputs; noise vectors give it entries
    m*offsets[s]:m*offsets[s+1] (m = 3, or 6 with includeAngular: the
    system's linear entries, then its angular ones).
    """

    def __init__(self, offsets, viscosity, radius, dtype=torch.float32, device=None, includeAngular: bool = False):
        import numpy as np
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.n_systems = int(self.offsets.shape[0] - 1)
        self.total = int(self.offsets[-1])
        vis = np.broadcast_to(np.asarray(viscosity, dtype=np.float64), (self.n_systems,))
        rad = np.broadcast_to(np.asarray(radius, dtype=np.float64), (self.n_systems,))
        self._dtype = dtype
        self._angular = bool(includeAngular)
        self._device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._h = _lib.rpy_batch_create(self.offsets, vis, rad, dtype, self._angular)
        self.last_iterations = None

    @property
    def includeAngular(self) -> bool:
        return self._angular

    def setPositions(self, positions: torch.Tensor):
        _lib.rpy_batch_set_positions(self._h, positions.reshape(-1, 3).contiguous(), self._dtype, self.total)

    def _vec(self, t):
        return None if t is None else t.reshape(-1, 3).contiguous()

    def Mdot(self, forces: torch.Tensor | None = None, torques: torch.Tensor | None = None):
        """Linear velocities (total, 3); with includeAngular, (linear, angular)."""
        out = torch.empty((self.total, 3), dtype=self._dtype, device=self._device)
        ang = torch.empty_like(out) if self._angular else None
        _lib.rpy_batch_mdot(self._h, self._vec(forces), self._vec(torques), out, ang, self._dtype, self.total)
        return (out, ang) if self._angular else out

    def autotune(self):
        """Time the batched product's configurations on the current systems
        and keep the fastest; returns (targets per lane (0 = block mode),
        workgroups per CU)."""
        _lib.rpy_batch_autotune(self._h)
        return self.tileConfig()

    def tileConfig(self):
        return _lib.rpy_batch_get_tile_config(self._h)

    def setTileConfig(self, targets_per_lane: int, workgroups_per_cu: int = 8):
        _lib.rpy_batch_set_tile_config(self._h, targets_per_lane, workgroups_per_cu)

    def sqrtMdotW(self, W: torch.Tensor, prefactor: float = 1.0, tol: float = 1e-6, maxIter: int = 500,
                  checkEvery: int = 4):
        """prefactor M_s^{1/2} W_s for every system: (total, 3), or (linear,
        angular) with includeAngular."""
        out = torch.empty((self.total, 3), dtype=self._dtype, device=self._device)
        ang = torch.empty_like(out) if self._angular else None
        self.last_iterations = _lib.rpy_batch_sqrt_mdot_w(self._h, W.reshape(-1).contiguous(), prefactor, tol,
                                                          maxIter, checkEvery, out, ang, self._dtype, self.total,
                                                          self.n_systems)
        return (out, ang) if self._angular else out

    def close(self):
        if getattr(self, "_h", None):
            _lib.rpy_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AdamsBashforth:
    """The stochastic Adams-Bashforth scheme of Sec. 5.1 on a Solver:

        X^{n+1} = X^n + dt (3/2 u^n - 1/2 u^{n-1}) + sqrt(2 kBT dt) (M^n)^{1/2} W^n,
        u^n = M^n [F^n; T^n] + kBT (d_X . M)^n,

    starting with one Euler-Maruyama step.  ``step`` uses the solver's
    current positions, returns (X^{n+1}, rotation increment or None) and
    stores X^{n+1} in the solver for the next step.  The scheme's history
    u^{n-1} lives in a device buffer owned by this object."""

    def __init__(self, solver: "Solver", dt: float, kBT: float = 0.0, tol: float = 1e-6, maxIter: int = 500):
        self.solver, self.dt, self.kBT, self.tol, self.maxIter = solver, float(dt), float(kBT), tol, maxIter
        self._hist = None
        self._have = False
        self.last_iterations = 0
        self.positions = None     # X^{n+1} of the last step (also stored in the solver)

    def reset(self):
        """Forget the history: the next step is an Euler-Maruyama step."""
        self._have = False

    def step(self, forces=None, torques=None, W: torch.Tensor | None = None,
             generator: torch.Generator | None = None):
        s = self.solver
        s._require_positions()
        f, t = s._as(forces, "forces"), s._as(torques, "torques")
        w = s._noise(W, generator) if self.kBT > 0 else None
        dim = (6 if s._angular else 3) * s._n
        if self._hist is None or self._hist.numel() != dim or self._hist.dtype != s._dtype:
            self._hist = torch.empty(dim, dtype=s._dtype, device=s._device)
            self._have = False
        pos = s._empty()
        ang = s._empty() if s._angular else None
        try:
            self.last_iterations = _lib.rpy_ab2_step(s._h, f, t, w, self.dt, self.kBT, self.tol, self.maxIter,
                                                     self._hist, self._have, pos, ang, s._dtype, s._n, s._angular)
        except NotConvergedError:
            # the step was completed with the last Lanczos iterate
            self._have = True
            s.setPositions(pos)
            self.positions = pos
            raise
        self._have = True
        s.setPositions(pos)
        self.positions = pos
        return pos, ang


class _MdotFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, positions, forces, torques):
        solver.setPositions(positions.detach())
        lin, ang = solver.Mdot(forces.detach() if forces is not None else None,
                               torques.detach() if torques is not None else None)
        ctx.solver = solver
        ctx.save_for_backward(positions, forces, torques)
        ctx.has_t = torques is not None
        if ang is None:
            ang = torch.zeros_like(lin)
        return lin, ang

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_lin, g_ang):
        solver = ctx.solver
        positions, forces, torques = ctx.saved_tensors
        solver.setPositions(positions.detach())
        g_ang = g_ang if (solver.includeAngular and g_ang is not None) else None
        gl = g_lin.contiguous() if g_lin is not None else torch.zeros_like(positions)
        gp, gf, gt = solver.Mdot_backward(forces, torques, gl, g_ang,
                                          need_pos=ctx.needs_input_grad[1],
                                          need_forces=ctx.needs_input_grad[2],
                                          need_torques=ctx.needs_input_grad[3] and ctx.has_t)
        gp = gp.reshape_as(positions) if gp is not None else None
        gf = gf.reshape_as(forces) if (gf is not None and forces is not None) else None
        gt = gt.reshape_as(torques) if (gt is not None and ctx.has_t) else None
        return None, gp, gf, gt


def mdot(solver: Solver, positions: torch.Tensor, forces: torch.Tensor | None,
         torques: torch.Tensor | None = None):
    """Differentiable (U, Omega) = M(X) [F; T]; gradients flow to X, F and T."""
    if forces is None and torques is None:
        raise ValueError("need forces or torques")
    lin, ang = _MdotFunction.apply(solver, positions, forces, torques)
    return lin, (ang if solver.includeAngular else None)

"""Oracle: time stepping of eq. (bdhi) for the open-boundary solver, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Sec. 3.2, LangevinVelocities: all three terms of eq. (bdhi) together; a
  solver without a special method takes an Euler-Maruyama step, i.e. the
  velocities
      v = M [F; T] + sqrt(2 kT / dt) M^{1/2} W + kT d_X . M,   W ~ N(0, I),
  so that X + dt v is one Euler-Maruyama step of eq. (bdhi) (dW = sqrt(dt) W).
* Sec. 5.1: the stochastic Adams-Bashforth scheme
      X^{n+1} = X^n + dt [ 3/2 u^n - 1/2 u^{n-1} ] + sqrt(2 kT dt) (M^n)^{1/2} W^n,
      u^n = M^n [F^n; T^n] + kT (d_X . M)^n,
  with the angular rows giving the rotation increment.  The paper does not
  say how the scheme starts; the first step (no u^{n-1}) is read as the
  Euler-Maruyama step (coefficients 1 and 0).
* The drift d_X . M is zero in open space (``drift.div_m_open``).

``sqrt_mdot_w(x, v)`` supplies M(x)^{1/2} v: the exact symmetric root or the
oracle's Lanczos at a matched iteration count.
"""
from __future__ import annotations

import math

import numpy as np

from .drift import div_m_open
from .mobility import mdot_dense


def _split(v, n):
    return v[: 3 * n].reshape(n, 3), (v[3 * n:].reshape(n, 3) if v.size > 3 * n else None)


def deterministic_velocity(x, forces, torques, kt, a, eta, angular: bool = False):
    """u = M [F; T] + kT d_X . M as (linear, angular or None)."""
    n = x.shape[0]
    f = np.zeros((n, 3)) if forces is None else forces
    t = torques if torques is not None else (np.zeros((n, 3)) if angular else None)
    u, om = mdot_dense(x, f, t, a, eta)
    dl, da = div_m_open(n, angular)
    u = u + kt * dl
    if angular:
        om = (np.zeros((n, 3)) if om is None else om) + kt * da
    return u, (om if angular else None)


def langevin_velocities(x, forces, torques, w, dt, kt, a, eta, sqrt_mdot_w, angular: bool = False):
    """Euler-Maruyama velocities of eq. (bdhi); returns (linear, angular)."""
    n = x.shape[0]
    u, om = deterministic_velocity(x, forces, torques, kt, a, eta, angular)
    if kt > 0:
        nl, na = _split(sqrt_mdot_w(x, w) * math.sqrt(2 * kt / dt), n)
        u = u + nl
        if angular:
            om = om + na
    return u, om


def ab2_step(x, forces, torques, w, dt, kt, a, eta, sqrt_mdot_w, u_prev=None, angular: bool = False):
    """One step of the scheme of Sec. 5.1 from positions ``x``.

    ``u_prev`` is the previous step's deterministic velocity as one vector
    (3N, or 6N with angular rows, linear first) or None for the first step.
    Returns (new positions, rotation increment or None, u^n as one vector).
    """
    n = x.shape[0]
    u, om = deterministic_velocity(x, forces, torques, kt, a, eta, angular)
    u_now = np.concatenate([u.reshape(-1), om.reshape(-1)]) if angular else u.reshape(-1)
    if u_prev is None:
        step = dt * u_now
    else:
        step = dt * (1.5 * u_now - 0.5 * u_prev)
    if kt > 0:
        step = step + math.sqrt(2 * kt * dt) * sqrt_mdot_w(x, w)
    dx, dth = _split(step, n)
    return x + dx, (dth if angular else None), u_now

"""Oracle: thermal drift k_B T d_X . M for the open-boundary solver, float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Sec. 2 (after eq. (fdt)): when M is translation invariant and isotropic,
  as in a bulk fluid, the drift vanishes, and it never has an orientational
  part because the particles are spheres.  Sec. 3.4: the default drift is
  zero.  ``div_m_open`` is that zero.
* Sec. 4, "Thermal drift": the deterministic divergence
  (1/delta) sum_j [M(q + delta/2 e_j) e_j - M(q - delta/2 e_j) e_j].  Only
  the 3N positional coordinates of q move the particles; orientation does
  not enter M (Sec. 3.4), so angular columns contribute nothing.
* Eq. (rfd): one random finite difference
  (1/delta) [M(X + delta/2 W) W - M(X - delta/2 W) W], W ~ N(0, I), whose
  average over W is the divergence up to O(delta^2).
"""
from __future__ import annotations

import numpy as np

from .mobility import grand_mobility, mdot_dense


def div_m_open(n: int, angular: bool = False):
    """Zero drift of the open-boundary solver: (linear, angular or None)."""
    return np.zeros((n, 3)), (np.zeros((n, 3)) if angular else None)


def divergence_fd(x, delta, a, eta, angular: bool = False, mobility=None):
    """Deterministic finite-difference divergence of M (the test of Sec. 4).

    Returns the 3N (or 6N, linear rows first) vector sum_j dM_ij/dq_j.
    ``mobility(x, a, eta, angular)`` gives the dense matrix (default: the
    open-boundary one).
    """
    grand_mobility_ = grand_mobility if mobility is None else mobility
    n = x.shape[0]
    dim = 6 * n if angular else 3 * n
    out = np.zeros(dim)
    for j in range(3 * n):
        xp = x.copy()
        xm = x.copy()
        xp.flat[j] += 0.5 * delta
        xm.flat[j] -= 0.5 * delta
        out += (grand_mobility_(xp, a, eta, angular)[:, j]
                - grand_mobility_(xm, a, eta, angular)[:, j]) / delta
    return out


def rfd_sample(x, w, delta, a, eta, angular: bool = False, round_positions=None, mdot=None):
    """One random finite difference of eq. (rfd) for the noise vector ``w``.

    ``w`` has 3N entries (6N with angular terms, linear first); only its
    positional part displaces the particles.  ``round_positions``, when
    given, is applied to the two displaced configurations before M is
    evaluated (to evaluate the sample on positions stored at a lower
    precision).  ``mdot(x, forces, torques, a, eta) -> (U, Omega)`` replaces
    the dense product (e.g. the C pair loop on selected rows).  Returns
    (linear, angular).
    """
    mdot = mdot_dense if mdot is None else mdot
    n = x.shape[0]
    wp = w[: 3 * n].reshape(n, 3)
    wt = w[3 * n:].reshape(n, 3) if angular else None
    xp = x + 0.5 * delta * wp
    xm = x - 0.5 * delta * wp
    if round_positions is not None:
        xp, xm = round_positions(xp), round_positions(xm)
    up, op = mdot(xp, wp, wt, a, eta)
    um, om = mdot(xm, wp, wt, a, eta)
    return (up - um) / delta, (None if not angular else (op - om) / delta)

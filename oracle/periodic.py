"""Oracle: the triply periodic RPY mobility (the PSE solver's problem), float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``); shares no code with the
HIP path.

What the paper fixes (Sec. 3.5, "Positively Split Ewald (PSE)")
---------------------------------------------------------------
For periodic boundaries in x, y and z the library computes the RPY mobility
of the periodic suspension by the positively split Ewald method of Fiore et
al.: a real-space part summed over near neighbours and a wave-space part on
a grid, both positive definite; the solver takes forces only.

Readings
--------
* The free-space RPY tensor (overlap branch and self block included) is the
  inverse Fourier transform of sinc^2(k a) (I - khat khat^T) / (eta k^2)
  (the double sphere-surface average of the Oseen tensor); the periodic
  mobility replaces the integral by the lattice sum, without k = 0 (zero
  mean flow):
      M_ij = (1 / (eta V)) sum_{k != 0} sinc^2(k a) (I - khat khat^T) / k^2 e^{i k (x_i - x_j)}.
* The split uses Hasimoto's function H(k, xi) = (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)},
  0 <= H <= 1:  M = M_real + M_wave with
      M_wave  = the lattice sum above times H(k, xi),
      M_real  = sum over periodic images n of [RPY(r + n L) - Wr(r + n L)],
  Wr the inverse Fourier transform of sinc^2(k a) H(k, xi) (I - khat khat^T)/(eta k^2)
  (a fast-converging radial integral, evaluated here by Gauss-Legendre
  quadrature); RPY - Wr decays like a Gaussian, and its integral (the k = 0
  term) vanishes, so the image sum converges absolutely and the total does
  not depend on xi (tested).
* Fluctuations (the "positive" split): both parts are positive definite, so
  a sample with covariance M is M_real^{1/2} W + (a sample with covariance
  M_wave), the second drawn in Fourier space from independent normals
  (``wave_fluctuation``; its noise layout is stated there).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn

from .mobility import coefficients

__all__ = ["hasimoto", "wave_radial", "real_blocks", "real_matrix", "wave_matrix", "grand_mobility_periodic",
           "mdot_periodic", "wave_vectors", "wave_fluctuation", "wave_rows", "mdot_periodic_rows"]


def hasimoto(k, xi):
    """Hasimoto's splitting function (1 + k^2/(4 xi^2)) exp(-k^2/(4 xi^2))."""
    q = (np.asarray(k) / (2.0 * xi)) ** 2
    return (1.0 + q) * np.exp(-q)


def _sinc2(x):
    return np.sinc(np.asarray(x) / np.pi) ** 2


_GL = {}


def wave_radial(r, a: float, eta: float, xi: float, nodes: int = 384):
    """(f, g) with Wr(r) = f(r) I + g(r) rhat rhat^T: the free-space transform of
    the wave-space kernel, by Gauss-Legendre quadrature on [0, 14 xi]."""
    if nodes not in _GL:
        _GL[nodes] = np.polynomial.legendre.leggauss(nodes)
    t, w = _GL[nodes]
    kmax = 14.0 * xi
    k = 0.5 * kmax * (t + 1.0)
    wk = 0.5 * kmax * w * _sinc2(k * a) * hasimoto(k, xi) / (2.0 * math.pi ** 2 * eta)
    r = np.asarray(r, dtype=np.float64)
    kr = r[..., None] * k
    small = kr < 1e-8
    krs = np.where(small, 1.0, kr)
    j0 = spherical_jn(0, krs)
    j1 = spherical_jn(1, krs)
    j2 = spherical_jn(2, krs)
    a_fun = np.where(small, 2.0 / 3.0, j0 - j1 / krs)
    b_fun = np.where(small, 0.0, j2)
    return (a_fun * wk).sum(-1), (b_fun * wk).sum(-1)


def _box(box):
    b = np.asarray(box, dtype=np.float64).reshape(-1)
    return np.repeat(b, 3) if b.size == 1 else b


def real_blocks(xt, xs, box, a: float, eta: float, xi: float, rcut: float | None = None):
    """Real-space blocks (P, Q, 3, 3): sum over images n of RPY - Wr at
    x_t - x_s + n L with |.| < rcut (default 7.5 / xi)."""
    L = _box(box)
    rcut = 7.5 / xi if rcut is None else rcut
    nmax = [int(math.ceil(rcut / L[d])) + 1 for d in range(3)]
    d0 = np.asarray(xt)[:, None, :] - np.asarray(xs)[None, :, :]
    d0 = d0 - L * np.round(d0 / L)            # nearest image first, so the window covers every image within rcut
    out = np.zeros(d0.shape[:2] + (3, 3))
    eye = np.eye(3)
    for n0 in range(-nmax[0], nmax[0] + 1):
        for n1 in range(-nmax[1], nmax[1] + 1):
            for n2 in range(-nmax[2], nmax[2] + 1):
                d = d0 + np.array([n0 * L[0], n1 * L[1], n2 * L[2]])
                r = np.sqrt((d * d).sum(-1))
                sel = r < rcut
                if not sel.any():
                    continue
                rr = r[sel]
                c1, c2, _, _, _ = coefficients(rr, a, eta)
                fw, gw = wave_radial(rr, a, eta, xi)
                rhat = np.where(rr[:, None] > 0, d[sel] / np.where(rr > 0, rr, 1.0)[:, None], 0.0)
                outer = rhat[:, :, None] * rhat[:, None, :]
                out[sel] += (c1 - fw)[:, None, None] * eye + (c2 - gw)[:, None, None] * outer
    return out


def wave_matrix(x, box, a: float, eta: float, xi: float):
    """Dense 3N x 3N wave-space part: the lattice sum over k != 0 with
    |k| <= 14 xi (where H < 1e-20)."""
    L = _box(box)
    kmax = 14.0 * xi
    nk = [int(math.floor(kmax * L[d] / (2 * math.pi))) for d in range(3)]
    grids = np.meshgrid(*[np.arange(-m, m + 1) for m in nk], indexing="ij")
    kv = np.stack([2 * math.pi * g.reshape(-1) / L[d] for d, g in enumerate(grids)], -1)
    k2 = (kv * kv).sum(-1)
    keep = (k2 > 0) & (k2 <= kmax * kmax)
    kv, k2 = kv[keep], k2[keep]
    kn = np.sqrt(k2)
    coef = _sinc2(kn * a) * hasimoto(kn, xi) / (eta * L.prod() * k2)
    khat = kv / kn[:, None]
    n = x.shape[0]
    m = np.zeros((n, 3, n, 3))
    for s in range(0, kv.shape[0], 2048):
        kk = kv[s:s + 2048]
        ph = np.asarray(x) @ kk.T                      # (N, K): k . x_i
        c, sn = np.cos(ph), np.sin(ph)
        proj = np.eye(3)[None] - khat[s:s + 2048, :, None] * khat[s:s + 2048, None, :]   # (K, 3, 3)
        w = coef[s:s + 2048]
        # sum_k w_k P_k cos(k . (x_i - x_j)) = sum_k w_k P_k (c_i c_j + s_i s_j)
        m += np.einsum("ik,jk,kab->iajb", c * w, c, proj) + np.einsum("ik,jk,kab->iajb", sn * w, sn, proj)
    return m.reshape(3 * n, 3 * n)


def grand_mobility_periodic(x, box, a: float, eta: float, xi: float | None = None):
    """Dense 3N x 3N periodic RPY mobility M_real + M_wave (xi default
    sqrt(pi) / min(L): both parts cheap for small test boxes)."""
    L = _box(box)
    xi = math.sqrt(math.pi) / L.min() if xi is None else xi
    n = x.shape[0]
    mr = real_blocks(x, x, L, a, eta, xi).transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
    return mr + wave_matrix(x, L, a, eta, xi)


def mdot_periodic(x, forces, box, a: float = 1.0, eta: float = 1.0 / (6 * math.pi), xi: float | None = None):
    """U = M F for the periodic suspension (dense)."""
    n = x.shape[0]
    return (grand_mobility_periodic(x, box, a, eta, xi) @ np.asarray(forces).reshape(-1)).reshape(n, 3)


def real_matrix(x, box, a: float, eta: float, xi: float, rcut: float | None = None):
    """Dense 3N x 3N real-space part alone (positive definite by itself)."""
    n = x.shape[0]
    return real_blocks(x, x, box, a, eta, xi, rcut).transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def wave_vectors(box, grid):
    """Wave vectors of an Nx x Ny x Nz Fourier grid: index -> 2 pi m / L_d with
    m the signed frequency (0..N/2-1, then -N/2..-1); (kx, ky, kz) arrays of
    the full grid, and a mask of the Nyquist entries (m = -N/2 for even N)."""
    L = _box(box)
    ks, nyq = [], []
    for d in range(3):
        n = int(grid[d])
        m = np.fft.fftfreq(n, d=1.0 / n)                  # signed integer frequencies
        ks.append(2.0 * math.pi * m / L[d])
        nyq.append((n % 2 == 0) & (np.arange(n) == n // 2))
    kx, ky, kz = np.meshgrid(*ks, indexing="ij")
    nq = nyq[0][:, None, None] | nyq[1][None, :, None] | nyq[2][None, None, :]
    return kx, ky, kz, nq


def _zeta(noise, grid):
    """Complex unit normals zeta_k (3, Nx, Ny, Nz) with zeta_{-k} = conj(zeta_k),
    from the half-spectrum noise (3, Nx, Ny, Nz//2 + 1, 2) of real N(0, 1)
    numbers (last axis: real, imaginary part):
      * 0 < kz-index < Nz/2: zeta = (re + i im) / sqrt(2);
      * the kz-index planes 0 and Nz/2 hold each k together with -k: the one
        of the pair (kx, ky) <= (-kx mod Nx, -ky mod Ny) (lexicographic) uses
        its own numbers as above, the other the conjugate of its partner's;
        a self-conjugate k takes zeta = re (real);
      * the other half of the spectrum is the conjugate of the stored half."""
    nx, ny, nz = (int(g) for g in grid)
    nh = nz // 2 + 1
    nu = np.asarray(noise, dtype=np.float64).reshape(3, nx, ny, nh, 2)
    half = (nu[..., 0] + 1j * nu[..., 1]) / math.sqrt(2.0)
    planes = [0] + ([nz // 2] if nz % 2 == 0 else [])
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    px, py = (-ix) % nx, (-iy) % ny
    own = ix * ny + iy
    mate = px * ny + py
    for q in planes:
        plane = half[:, :, :, q].copy()
        partner = (nu[:, px, py, q, 0] + 1j * nu[:, px, py, q, 1]) / math.sqrt(2.0)
        plane = np.where(own > mate, np.conj(partner), plane)
        plane = np.where(own == mate, nu[:, :, :, q, 0] + 0j, plane)
        half[:, :, :, q] = plane
    full = np.zeros((3, nx, ny, nz), dtype=complex)
    full[..., :nh] = half
    for iz in range(nh, nz):
        full[:, :, :, iz] = np.conj(half[:, (-np.arange(nx)) % nx][:, :, (-np.arange(ny)) % ny, nz - iz])
    return full


def wave_fluctuation(x, box, a: float, eta: float, xi: float, grid, noise):
    """A sample with covariance M_wave (restricted to the wave vectors of the
    grid, k = 0 and Nyquist entries excluded), from the noise array of
    ``_zeta``:  y_i = V^{-1/2} sum_k sqrt(Khat_w(k)) (I - khat khat^T) zeta_k e^{i k . x_i},
    Khat_w(k) = sinc^2(k a) H(k, xi) / (eta k^2)."""
    L = _box(box)
    kx, ky, kz, nyq = wave_vectors(L, grid)
    k2 = kx * kx + ky * ky + kz * kz
    keep = (k2 > 0) & ~nyq
    kv = np.stack([kx[keep], ky[keep], kz[keep]], -1)
    kn = np.sqrt(k2[keep])
    amp = np.sqrt(_sinc2(kn * a) * hasimoto(kn, xi) / (eta * kn * kn))
    z = _zeta(noise, grid)[:, keep].T                                 # (K, 3)
    khat = kv / kn[:, None]
    pz = z - khat * (khat * z).sum(-1, keepdims=True)                  # (I - khat khat^T) zeta
    ph = np.exp(1j * (np.asarray(x) @ kv.T))                           # (N, K)
    y = ph @ (amp[:, None] * pz) / math.sqrt(L.prod())
    return y.real


def wave_rows(x, rows, forces, box, a: float, eta: float, xi: float):
    """Rows `rows` of M_wave F as the lattice sum applied to F directly:
    Fhat(k) = sum_j F_j e^{-i k . x_j}, U_i = (1/(eta V)) sum_k sinc^2 H / k^2
    (I - khat khat^T) Re(Fhat(k) e^{i k . x_i}), k != 0, |k| <= 14 xi."""
    L = _box(box)
    kmax = 14.0 * xi
    nk = [int(math.floor(kmax * L[d] / (2 * math.pi))) for d in range(3)]
    grids = np.meshgrid(*[np.arange(-m, m + 1) for m in nk], indexing="ij")
    kv = np.stack([2 * math.pi * g.reshape(-1) / L[d] for d, g in enumerate(grids)], -1)
    k2 = (kv * kv).sum(-1)
    keep = (k2 > 0) & (k2 <= kmax * kmax)
    kv, k2 = kv[keep], k2[keep]
    kn = np.sqrt(k2)
    coef = _sinc2(kn * a) * hasimoto(kn, xi) / (eta * L.prod() * k2)
    khat = kv / kn[:, None]
    x = np.asarray(x)
    F = np.asarray(forces, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((len(rows), 3))
    for s in range(0, kv.shape[0], 4096):
        kk = kv[s:s + 4096]
        fh = np.exp(-1j * (x @ kk.T)).T @ F                       # (K, 3)
        kh = khat[s:s + 4096]
        pf = fh - kh * (kh * fh).sum(-1, keepdims=True)           # (I - khat khat^T) Fhat
        ph = np.exp(1j * (x[rows] @ kk.T))                        # (R, K)
        out += (ph @ (coef[s:s + 4096, None] * pf)).real
    return out


def mdot_periodic_rows(x, rows, forces, box, a: float, eta: float, xi: float):
    """Rows `rows` of M F (real part by blocks, wave part by ``wave_rows``)."""
    F = np.asarray(forces, dtype=np.float64).reshape(-1, 3)
    rb = real_blocks(np.asarray(x)[rows], x, box, a, eta, xi)          # (R, N, 3, 3)
    return np.einsum("rjab,jb->ra", rb, F) + wave_rows(x, rows, F, box, a, eta, xi)

"""Long-range PM force of the PM-FMM split and a periodic Ewald sum.

Test infrastructure (see the package docstring).  Float64 numpy.

Paper passages followed (Sec. 2): the gravity of a periodic box is split
into a short-range part, the truncated pair force of Eq. (tr), and a
long-range part solved on a mesh with FFTs, whose Green's function is the
Newtonian one multiplied by a Gaussian factor in k.

Readings (the paper states the split but not the mesh details):
  * long-range factor: exp(-k^2 r_s^2), the Fourier transform of
    erf(r / 2 r_s) / r divided by 4 pi / k^2, so that short + long is the
    Newtonian pair force (the printed exponent is read this way; see the
    package's design notes);
  * mesh: N^3 nodes at g L / N (g = 0 .. N-1) in the periodic box, cloud in
    cell (CIC) assignment of the masses and the same CIC interpolation of
    the accelerations, each undone once in k by dividing by
    W(k) = prod_a sinc^2(k_a L / 2N);
  * potential phi(k) = -4 pi G rho(k) exp(-k^2 r_s^2) / k^2 (k = 0 dropped:
    the mean density is subtracted, as in any periodic solver), acceleration
    a(k) = -i k phi(k), with the Nyquist component of each k_a set to zero.

Ewald (``ewald_accel``): the textbook splitting of the periodic 1/r sum
with its own parameter alpha, real-space images up to |n| <= n_img and
reciprocal vectors up to |m| <= m_max; independent of the mesh and of
r_s, it is the reference the full force (short + long) is checked against.

Parity: pinned by tests/test_oracle_pm.py (Ewald against the direct image
sum of a neutralised pair and its own convergence in alpha; PM long +
short pair force against Ewald within the mesh's error; momentum
conservation of the PM force; the PM force of a pair against the
erf-smoothed pair law at separations well inside the box).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

SQRT_PI = math.sqrt(math.pi)


def _cic(pos, box, n):
    """Lower node index (N, 3) and weights of the two nodes per axis."""
    u = np.asarray(pos, np.float64) * (n / box)
    g = np.floor(u)
    f = u - g
    g = g.astype(np.int64) % n
    return g, np.stack([1.0 - f, f], axis=0)      # (2, N, 3)


def cic_deposit(pos, mass, box, n):
    """Mass density on the mesh (N^3 nodes), CIC."""
    rho = np.zeros((n, n, n))
    g, w = _cic(pos, box, n)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                wt = mass * w[dx, :, 0] * w[dy, :, 1] * w[dz, :, 2]
                np.add.at(rho, ((g[:, 0] + dx) % n, (g[:, 1] + dy) % n,
                                (g[:, 2] + dz) % n), wt)
    return rho * (n / box) ** 3


def cic_interp(field, pos, box, n):
    """Mesh field (3, N, N, N) at the particles, CIC."""
    g, w = _cic(pos, box, n)
    out = np.zeros((len(pos), 3))
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                wt = w[dx, :, 0] * w[dy, :, 1] * w[dz, :, 2]
                idx = ((g[:, 0] + dx) % n, (g[:, 1] + dy) % n, (g[:, 2] + dz) % n)
                for a in range(3):
                    out[:, a] += wt * field[a][idx]
    return out


def wavenumbers(box, n):
    """k along one axis in numpy FFT order, with the Nyquist entry."""
    m = np.fft.fftfreq(n, d=1.0 / n)
    return 2.0 * math.pi * m / box


def long_range_accel(pos, mass, box, r_s, n, G=1.0):
    """Long-range accelerations (N, 3) of the split, on an n^3 mesh."""
    rho = cic_deposit(pos, mass, box, n)
    rk = np.fft.fftn(rho)
    k1 = wavenumbers(box, n)
    kx, ky, kz = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    h = box / n

    def sinc(x):
        return np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))

    W = (sinc(kx * h / 2) * sinc(ky * h / 2) * sinc(kz * h / 2)) ** 2
    green = np.zeros_like(k2)
    nz = k2 > 0
    green[nz] = -4.0 * math.pi * G * np.exp(-k2[nz] * r_s * r_s) / k2[nz]
    phik = rk * green / (W * W)
    nyq = n // 2 if n % 2 == 0 else None
    field = []
    for a, ka in enumerate((kx, ky, kz)):
        kk = ka.copy()
        if nyq is not None:
            sl = [slice(None)] * 3
            sl[a] = nyq
            kk[tuple(sl)] = 0.0
        field.append(np.real(np.fft.ifftn(-1j * kk * phik)))
    return cic_interp(field, pos, box, n)


def ewald_accel(pos, mass, box, G=1.0, alpha=None, n_img=2, m_max=10):
    """Periodic Newtonian accelerations (uniform background subtracted) by
    Ewald summation: a_i = G sum_j m_j [real + reciprocal], d = x_j - x_i,
      real  = sum_n (d + nL) / r^3 (erfc(alpha r) + 2 alpha r / sqrt(pi) e^(-alpha^2 r^2)),
              r = |d + nL|, the n = 0 term left out for j = i;
      recip = (4 pi / L^3) sum_{k != 0} (k / k^2) exp(-k^2 / 4 alpha^2) sin(k . d)."""
    pos = np.asarray(pos, np.float64)
    mass = np.asarray(mass, np.float64)
    n = len(pos)
    if alpha is None:
        alpha = 5.0 / box
    acc = np.zeros((n, 3))
    rng = range(-n_img, n_img + 1)
    for i in range(n):
        d0 = pos - pos[i][None, :]
        for nx in rng:
            for ny in rng:
                for nz in rng:
                    d = d0 + np.array([nx, ny, nz], float)[None, :] * box
                    r = np.linalg.norm(d, axis=1)
                    ok = r > 0
                    rr = np.where(ok, r, 1.0)
                    f = (erfc(alpha * rr) + 2.0 * alpha * rr / SQRT_PI
                         * np.exp(-alpha * alpha * rr * rr)) / rr ** 3
                    f = np.where(ok, f, 0.0)
                    acc[i] += np.sum((mass * f)[:, None] * d, axis=0)
    ms = np.arange(-m_max, m_max + 1)
    mx, my, mz = np.meshgrid(ms, ms, ms, indexing="ij")
    kv = (2.0 * math.pi / box) * np.stack([mx.ravel(), my.ravel(), mz.ravel()], 1)
    k2 = np.sum(kv * kv, axis=1)
    keep = k2 > 0
    kv, k2 = kv[keep], k2[keep]
    coef = (4.0 * math.pi / box ** 3) * np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    # sum_j m_j sin(k.(x_j - x_i)) = S_s(k) cos(k.x_i) - S_c(k) sin(k.x_i)
    ph = pos @ kv.T                                   # (N, K)
    Sc = mass @ np.cos(ph)
    Ss = mass @ np.sin(ph)
    s = Ss[None, :] * np.cos(ph) - Sc[None, :] * np.sin(ph)
    acc += (s * coef[None, :]) @ kv
    return G * acc


def short_pair_accel(pos, mass, box, r_s, G=1.0):
    """Short-range accelerations of all minimum-image pairs (no cutoff),
    G m_j T(r / 2 r_s) d / r^3, for the small systems of the PM checks."""
    pos = np.asarray(pos, np.float64)
    acc = np.zeros_like(pos)
    for i in range(len(pos)):
        d = pos - pos[i][None, :]
        d -= box * np.round(d / box)
        r = np.linalg.norm(d, axis=1)
        ok = r > 0
        rr = np.where(ok, r, 1.0)
        x = rr / (2.0 * r_s)
        T = erfc(x) + (2.0 / SQRT_PI) * x * np.exp(-x * x)
        g = np.where(ok, mass * T / rr ** 3, 0.0)
        acc[i] = np.sum(g[:, None] * d, axis=0)
    return G * acc

"""Seeded synthetic particle sets for the short-range gravity path.

This module only draws inputs: positions in a periodic box, equal particle
masses, and the seeded cotangents used by the gradient checks.  It holds none
of the force arithmetic and imports nothing else from the package, so the CPU
oracle checks and the GPU path can both be fed from it.

The paper's own initial conditions come from 2LPTic with a CAMB spectrum
(Sec. 4); neither is available here.  The stand-in is a Zel'dovich-displaced
grid whose density contrast has P(k) proportional to k^-2, plus a fraction of
the particles moved into Plummer spheres, which gives the uneven leaf-pair
lists a clustered cosmological snapshot produces.

Workload recipe (every number is a parameter below):
  * grid points at (i + 1/2) L / n for i = 0..n-1 on each axis;
  * density contrast delta_k = W_k / |k| from unit white noise W, with the
    k = 0 mode and every Nyquist plane set to zero;
  * Zel'dovich displacement psi_k = i k delta_k / k^2, scaled so that the
    3-D rms of |psi| equals ``rms_disp`` grid spacings;
  * a seeded random ``halo_frac`` of the displaced particles is moved into
    ``n_halos`` Plummer spheres of scale ``halo_scale`` grid spacings; halo
    weights are 10**U(0,1) (log-uniform over one decade), particle counts
    per halo by largest remainder, halo centres uniform in the box, radii
    r = a (U^(-2/3) - 1)^(-1/2) redrawn while r > 10 a, isotropic
    directions;
  * everything is wrapped into [0, L).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BOX = 100.0


def wrap(x: np.ndarray, box: float) -> np.ndarray:
    """Map coordinates into [0, box)."""
    y = np.mod(x, box)
    y[y >= box] -= box
    y[y < 0.0] = 0.0
    return y


def uniform(n: int, box: float, seed: int) -> np.ndarray:
    """n i.i.d. uniform points in [0, box)^3, shape (n, 3), float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, box, size=(n, 3))


def zeldovich_grid(n_side: int, box: float, rms_disp: float, rng) -> np.ndarray:
    """Grid displaced by a Gaussian random field with P_delta ~ k^-2.

    ``rms_disp`` is in units of the grid spacing box / n_side.
    """
    n = n_side
    dg = box / n
    noise = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(noise)
    del noise
    f = np.fft.fftfreq(n, d=1.0 / n)          # integer frequencies
    fz = np.fft.rfftfreq(n, d=1.0 / n)
    kx = f[:, None, None]
    ky = f[None, :, None]
    kz = fz[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    zero = (k2 == 0)
    if n % 2 == 0:
        nyq = n // 2
        zero = zero | (np.abs(kx) == nyq) | (np.abs(ky) == nyq) | (kz == nyq)
    k2s = np.where(zero, 1.0, k2)
    delta = wk / np.sqrt(k2s)                 # amplitude ~ k^-1 -> P ~ k^-2
    delta[zero] = 0.0
    del wk
    disp = np.empty((n, n, n, 3))
    for a, ka in enumerate((kx, ky, kz)):
        psi_k = 1j * ka * delta / k2s
        psi_k[zero] = 0.0
        disp[..., a] = np.fft.irfftn(psi_k, s=(n, n, n), axes=(0, 1, 2))
        del psi_k
    del delta
    rms = math.sqrt(float(np.mean(np.sum(disp * disp, axis=-1))))
    if rms > 0.0:
        disp *= (rms_disp * dg) / rms
    g = (np.arange(n) + 0.5) * dg
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1)
    x = (q + disp).reshape(-1, 3)
    return wrap(x, box)


def _largest_remainder(total: int, weights: np.ndarray) -> np.ndarray:
    ideal = total * weights / weights.sum()
    base = np.floor(ideal).astype(np.int64)
    rem = total - int(base.sum())
    order = np.lexsort((np.arange(len(weights)), -(ideal - base)))
    base[order[:rem]] += 1
    return base


def plummer_halos(x: np.ndarray, halo_frac: float, n_halos: int,
                  scale: float, box: float, rng) -> np.ndarray:
    """Move a random ``halo_frac`` of the rows of x into Plummer spheres."""
    n = x.shape[0]
    n_move = int(round(halo_frac * n))
    if n_move == 0 or n_halos == 0:
        return x
    x = x.copy()
    chosen = rng.choice(n, size=n_move, replace=False)
    weights = 10.0 ** rng.uniform(0.0, 1.0, size=n_halos)
    counts = _largest_remainder(n_move, weights)
    centres = rng.uniform(0.0, box, size=(n_halos, 3))
    # radii: inverse CDF of the Plummer cumulative mass, redrawn beyond 10 a
    r = np.empty(n_move)
    todo = np.arange(n_move)
    while todo.size:
        u = rng.uniform(0.0, 1.0, size=todo.size)
        u = np.maximum(u, 1e-300)
        rr = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        ok = rr <= 10.0 * scale
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    v = rng.standard_normal((n_move, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    halo_of = np.repeat(np.arange(n_halos), counts)
    x[chosen] = centres[halo_of] + r[:, None] * v
    return wrap(x, box)


@dataclass
class Workload:
    """One periodic box: positions, masses and the force-split parameters."""
    name: str
    pos: np.ndarray
    mass: np.ndarray
    box: float
    n_pm: int
    r_s: float
    r_cut: float
    max_leaf: int
    order: int
    meta: dict = field(default_factory=dict)


def split_params(box: float, n_pm: int):
    """r_s = 1.2 box / N_PM and r_cut = 4.5 r_s."""
    r_s = 1.2 * box / n_pm
    return r_s, 4.5 * r_s


def clustered(n_side: int, box: float, halo_frac: float, n_halos: int,
              seed, rms_disp: float = 0.5, halo_scale: float = 0.3):
    """Zel'dovich grid plus Plummer halos; ``seed`` is an int or a Generator."""
    rng = seed if isinstance(seed, np.random.Generator) else \
        np.random.default_rng(seed)
    x = zeldovich_grid(n_side, box, rms_disp, rng)
    return plummer_halos(x, halo_frac, n_halos, halo_scale * box / n_side,
                         box, rng)


def _wl(name, pos, n_pm, max_leaf, order, **meta):
    n = pos.shape[0]
    r_s, r_cut = split_params(BOX, n_pm)
    return Workload(name, np.ascontiguousarray(pos), np.full(n, 1.0 / n),
                    BOX, n_pm, r_s, r_cut, max_leaf, order, meta)


def uniform_32k(seed: int = 14009) -> Workload:
    """32^3 uniform particles, N_PM = 32, leaves <= 32, p = 4."""
    return _wl("uniform_32k", uniform(32 ** 3, BOX, seed), 32, 32, 4)


def clustered_2m(seed: int = 14010) -> Workload:
    """128^3 clustered: Zel'dovich + 20 % in 200 Plummer halos, N_PM = 128."""
    return _wl("clustered_2m", clustered(128, BOX, 0.2, 200, seed), 128, 64, 4)


def clustered_16m(seed: int = 14011) -> Workload:
    """256^3 clustered: Zel'dovich + 30 % in 2000 Plummer halos, N_PM = 256."""
    return _wl("clustered_16m", clustered(256, BOX, 0.3, 2000, seed),
               256, 64, 4)


def clustered_262k(seed: int = 14013) -> Workload:
    """64^3 clustered (Zel'dovich + 20 % Plummer), N_PM = 64, gradient case."""
    return _wl("clustered_262k", clustered(64, BOX, 0.2, 25, seed), 64, 64, -1)


def clustered_small(n_side: int, seed, halo_frac: float = 0.2,
                    n_halos: int | None = None, max_leaf: int = 64,
                    order: int = 4) -> Workload:
    """Clustered box of n_side^3 particles with N_PM = n_side."""
    if n_halos is None:
        n_halos = max(4, int(round(200 * n_side ** 3 / 128 ** 3)))
    pos = clustered(n_side, BOX, halo_frac, n_halos, seed)
    return _wl(f"clustered_{n_side}^3", pos, n_side, max_leaf, order,
               n_halos=n_halos)


def batch_side(rng, lo: int = 16, hi: int = 96) -> int:
    """n_side = round(exp U(ln lo, ln hi)): N log-uniform in [lo^3, hi^3]."""
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_64(n_box: int = 64, seed: int = 1400800, max_leaf: int = 64,
             lo: int = 16, hi: int = 96):
    """Independent clustered boxes; box b draws from default_rng(seed + b)."""
    boxes = []
    for b in range(n_box):
        rng = np.random.default_rng(seed + b)
        ns = batch_side(rng, lo, hi)
        boxes.append(clustered_small(ns, rng, max_leaf=max_leaf, order=-1))
    return boxes


def cotangent(n: int, seed: int = 15013) -> np.ndarray:
    """Seeded Gaussian weights w_i (n, 3) for loss = sum_i w_i . a_i."""
    return np.random.default_rng(seed).standard_normal((n, 3))

"""Pins of the oracle's leapfrog and power spectrum."""

import math

import numpy as np

from oracle import stepping
from paper_2107_14008_amd import inputs


class _W:
    """8^3 Zel'dovich-displaced grid particles (no halos: no close pairs,
    so the orbits are smooth) with a 16^3 mesh (r_cut < L / 2)."""

    def __init__(self):
        self.box, self.n_pm = inputs.BOX, 16
        self.pos = inputs.clustered(8, self.box, 0.0, 1, 21)
        self.mass = np.full(len(self.pos), 1.0 / len(self.pos))
        self.r_s, self.r_cut = inputs.split_params(self.box, self.n_pm)


def _system():
    return _W()


def _dt(w):
    """A step that moves the fastest particle ~1 % of a cell in its first step."""
    a = stepping.split_accel(w.pos, w.mass, w.box, w.r_s, w.r_cut, w.n_pm)
    return math.sqrt(0.02 * w.box / w.n_pm / np.abs(a).max())


def test_leapfrog_is_second_order():
    """Error against a 128-step run falls 4x per halving of dt (a wrong kick
    or drift factor makes it first order or O(1))."""
    w = _system()
    dt = _dt(w)
    v0 = np.zeros_like(w.pos)
    T = 2 * dt          # before the first close approaches (no softening)
    ref, _ = stepping.kdk(w.pos, v0, w.mass, w.box, w.r_s, w.r_cut, w.n_pm, T / 128, 128)
    errs = []
    for k in (4, 8, 16):
        x, _ = stepping.kdk(w.pos, v0, w.mass, w.box, w.r_s, w.r_cut, w.n_pm, T / k, k)
        d = x - ref
        d -= w.box * np.round(d / w.box)
        errs.append(np.abs(d).max())
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def test_leapfrog_is_time_reversible_and_keeps_momentum():
    w = _system()
    dt = _dt(w)
    v0 = np.zeros_like(w.pos)
    x, v = stepping.kdk(w.pos, v0, w.mass, w.box, w.r_s, w.r_cut, w.n_pm, dt / 2, 4)
    xb, vb = stepping.kdk(x, -v, w.mass, w.box, w.r_s, w.r_cut, w.n_pm, dt / 2, 4)
    d = xb - w.pos
    d -= w.box * np.round(d / w.box)
    moved = x - w.pos
    moved -= w.box * np.round(moved / w.box)
    assert np.abs(d).max() <= 1e-9 * np.abs(moved).max()
    assert np.abs(vb).max() <= 1e-9 * np.abs(v).max()
    p = (w.mass[:, None] * v).sum(0)
    assert np.abs(p).max() <= 1e-12 * (w.mass[:, None] * np.abs(v)).sum()


def test_power_spectrum_of_one_mode():
    """A lattice displaced by one sine wave: its power sits in the wave's shell
    (amplitude A, delta = -k A cos(kx) to first order, P = (k A)^2 L^3 / 4)."""
    n, box = 32, 100.0
    g = (np.arange(n) + 0.5) * box / n
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    k = 2 * math.pi * 3 / box
    A = 0.01 * box / n
    pos[:, 0] += A * np.sin(k * pos[:, 0])
    ks, P, cnt = stepping.power_spectrum(pos, np.ones(len(pos)), box, n)
    s = int(np.argmin(np.abs(ks - k)))
    expect = (k * A) ** 2 * box ** 3 / 4 * 2 / cnt[s]   # two modes (+k, -k) in the shell
    assert abs(P[s] - expect) <= 0.05 * expect
    others = np.delete(P, s)
    assert others.max() <= 1e-3 * P[s]

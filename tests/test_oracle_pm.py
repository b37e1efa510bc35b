"""Pins of the oracle's long-range PM force and Ewald sum.

The Ewald sum is pinned by its independence of its own splitting parameter
(a wrong factor or sign in the real or reciprocal part shows as a
dependence on alpha) and by the Newtonian pair force at small separation;
the PM force then against Ewald: short (Eq. (tr), every pair) + long (the
mesh) = periodic Newton, within the mesh error, which falls as the mesh is
refined at fixed r_s.  Loosely pinned: the mesh error (~1e-2 at
r_s = 1.2 cells) is the tolerance.
"""

import math

import numpy as np
from scipy.special import erf

from oracle import pm


def _system(n=40, seed=1, box=100.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, box, (n, 3)), rng.uniform(0.5, 1.5, n), box


def test_ewald_does_not_depend_on_alpha():
    pos, m, box = _system()
    a1 = pm.ewald_accel(pos, m, box, alpha=5.0 / box)
    a2 = pm.ewald_accel(pos, m, box, alpha=3.5 / box, n_img=3, m_max=9)
    assert np.abs(a1 - a2).max() <= 1e-11 * np.abs(a1).max()


def test_ewald_close_pair_is_newton():
    box = 100.0
    pos = np.array([[50.0, 50.0, 50.0], [50.3, 50.1, 49.8]])
    m = np.array([1.0, 2.0])
    a = pm.ewald_accel(pos, m, box)
    d = pos[1] - pos[0]
    r = np.linalg.norm(d)
    newton = m[1] * d / r ** 3
    # images and the background change it by ~ (r / L)^3
    assert np.linalg.norm(a[0] - newton) <= 1e-4 * np.linalg.norm(newton)


def test_pm_plus_short_is_periodic_newton():
    pos, m, box = _system()
    ew = pm.ewald_accel(pos, m, box)
    errs = []
    for n in (32, 64):
        r_s = 1.2 * box / 32
        tot = pm.long_range_accel(pos, m, box, r_s, n) + pm.short_pair_accel(pos, m, box, r_s)
        e = np.linalg.norm(tot - ew, axis=1) / np.linalg.norm(ew, axis=1)
        errs.append(np.median(e))
    assert errs[0] < 1e-2
    assert errs[1] < errs[0] / 3          # mesh error ~ h^2 at fixed r_s


def test_pm_momentum_is_conserved():
    pos, m, box = _system(n=100, seed=4)
    a = pm.long_range_accel(pos, m, box, 1.2 * box / 32, 32)
    p = (m[:, None] * a).sum(0)
    assert np.abs(p).max() <= 1e-13 * np.abs(m[:, None] * a).sum()


def test_pm_pair_follows_the_erf_law():
    """Two particles a few r_s apart: the mesh force is the long-range part
    G m (erf(x) - 2 x e^(-x^2) / sqrt(pi)) / r^2, x = r / 2 r_s."""
    box, n = 100.0, 64
    r_s = 1.2 * box / n
    pos = np.array([[40.3, 50.2, 49.7], [40.3 + 3 * r_s, 50.2, 49.7]])
    m = np.array([1.0, 1.0])
    a = pm.long_range_accel(pos, m, box, r_s, n)
    r = 3 * r_s
    x = r / (2 * r_s)
    law = (erf(x) - 2 * x * math.exp(-x * x) / math.sqrt(math.pi)) / r ** 2
    # the periodic images and the background shift it by ~ r / L^3
    assert abs(a[0, 0] - law) <= 2e-2 * law
    assert abs(a[1, 0] + law) <= 2e-2 * law

"""Pins of the oracle's brute-force sum and its gradient.

Checks against routes the brute force does not share: the O(N^2) all-pairs
sum, the two-body closed form in high precision, symmetry (perfect lattice,
translation, momentum), Newton's law in the r_s -> infinity limit, and
central finite differences of the loss for the gradient.
"""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import direct
from paper_2107_14008_amd import inputs


def test_cell_grid_matches_all_pairs_uniform():
    rng = np.random.default_rng(1)
    pos = rng.uniform(0, 100, (1500, 3))
    m = rng.uniform(0.5, 2.0, 1500)
    a1, c1 = direct.all_pairs(pos, m, 100.0, 3.75, 16.875)
    a2, c2 = direct.brute_force(pos, m, 100.0, 3.75, 16.875, workers=1)
    assert np.array_equal(c1, c2)
    scale = np.abs(a1).max()
    assert np.max(np.abs(a1 - a2)) <= 1e-13 * scale


def test_cell_grid_matches_all_pairs_clustered_parallel():
    w = inputs.clustered_small(12, 7, halo_frac=0.4, n_halos=3)
    a1, c1 = direct.all_pairs(w.pos, w.mass, w.box, w.r_s, w.r_cut)
    a2, c2 = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                workers=2)
    assert np.array_equal(c1, c2)
    assert np.max(np.abs(a1 - a2)) <= 1e-13 * np.abs(a1).max()


def test_targets_subset():
    w = inputs.clustered_small(12, 8)
    full, cf = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                  workers=1)
    t = np.array([5, 77, 3, 1000, 1727])
    sub, cs = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                 targets=t, workers=1)
    assert np.array_equal(sub, full[t])
    assert np.array_equal(cs, cf[t])


@pytest.mark.parametrize("r", [0.3, 2.0, 7.5, 16.0])
def test_two_body_closed_form(r):
    """|a| = G m T(r / 2 r_s) / r^2 toward the partner, evaluated in mpmath."""
    box, r_s, r_cut = 100.0, 3.75, 16.875
    # the pair straddles the periodic boundary along x
    pos = np.array([[99.0, 50.0, 50.0], [99.0 + r, 50.0, 50.0]])
    pos = inputs.wrap(pos, box)
    m = np.array([0.7, 1.9])
    G = 2.5
    acc, cnt = direct.all_pairs(pos, m, box, r_s, r_cut, G=G)
    x = mp.mpf(r) / (2 * r_s)
    T = mp.erfc(x) + 2 * x / mp.sqrt(mp.pi) * mp.exp(-x * x)
    mag0 = float(G * m[1] * T / mp.mpf(r) ** 2)
    mag1 = float(G * m[0] * T / mp.mpf(r) ** 2)
    assert acc[0, 0] == pytest.approx(mag0, rel=1e-13)
    assert acc[1, 0] == pytest.approx(-mag1, rel=1e-13)
    assert np.all(acc[:, 1:] == 0.0)
    assert list(cnt) == [1, 1]


def test_pair_outside_cutoff_and_coincident():
    box, r_s, r_cut = 100.0, 3.75, 16.875
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + 16.9, 10.0, 10.0],
                    [40.0, 40.0, 40.0], [40.0, 40.0, 40.0]])
    acc, cnt = direct.all_pairs(pos, np.ones(4), box, r_s, r_cut)
    assert np.all(acc == 0.0)
    assert list(cnt) == [0, 0, 0, 0]


def test_perfect_lattice_has_zero_force():
    n = 12
    box = 100.0
    g = (np.arange(n) + 0.5) * box / n
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    r_s = 1.2 * box / n
    r_cut = 4.5 * r_s
    m = np.full(len(pos), 1.0 / len(pos))
    acc, cnt = direct.brute_force(pos, m, box, r_s, r_cut, workers=1)
    single = m[0] / (box / n) ** 2          # one nearest-neighbour term
    assert np.max(np.abs(acc)) < 1e-12 * single
    assert np.all(cnt == cnt[0])


def test_translation_invariance():
    w = inputs.clustered_small(12, 9)
    a0, c0 = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                workers=1)
    moved = inputs.wrap(w.pos + np.array([31.7, -12.25, 77.0]), w.box)
    a1, c1 = direct.brute_force(moved, w.mass, w.box, w.r_s, w.r_cut,
                                workers=1)
    assert np.array_equal(c0, c1)
    mag = np.linalg.norm(a0, axis=1)
    assert np.max(np.linalg.norm(a1 - a0, axis=1) / mag) < 1e-10


def test_momentum_conservation():
    w = inputs.clustered_small(12, 10)
    m = np.random.default_rng(3).uniform(0.5, 1.5, len(w.pos))
    acc, _ = direct.brute_force(w.pos, m, w.box, w.r_s, w.r_cut, workers=1)
    p = (m[:, None] * acc).sum(0)
    scale = np.sum(m * np.linalg.norm(acc, axis=1))
    assert np.all(np.abs(p) < 1e-14 * scale)


def test_newtonian_limit():
    """r_s much larger than the cluster: the sum tends to plain G m / r^2."""
    rng = np.random.default_rng(4)
    pos = 500.0 + rng.standard_normal((200, 3))
    m = rng.uniform(0.5, 1.5, 200)
    box, r_s = 1000.0, 100.0
    acc, _ = direct.all_pairs(pos, m, box, r_s, 4.5 * r_s)
    d = pos[None, :, :] - pos[:, None, :]
    r = np.linalg.norm(d, axis=-1)
    np.fill_diagonal(r, np.inf)
    newton = np.sum(m[None, :, None] * d / r[..., None] ** 3, axis=1)
    rel = np.linalg.norm(acc - newton, axis=1) / np.linalg.norm(newton, axis=1)
    # T = 1 - O(x^3), x = r / 2 r_s ~ 1e-2 at most here
    assert np.max(rel) < 1e-5


# ------------------------------------------------------------- gradient

@pytest.fixture(scope="module")
def grad_case():
    rng = np.random.default_rng(11)
    n = 400
    box = 20.0
    pos = rng.uniform(0, box, (n, 3))
    # a small clump so that close pairs are present
    pos[:60] = inputs.wrap(7.0 + 0.4 * rng.standard_normal((60, 3)), box)
    m = rng.uniform(0.5, 1.5, n) / n
    w = rng.standard_normal((n, 3))
    r_s = 1.2 * box / 16
    r_cut = 4.5 * r_s
    return pos, m, w, box, r_s, r_cut


def test_gradient_mass_matches_fd(grad_case):
    pos, m, w, box, r_s, r_cut = grad_case
    gx, gm = direct.gradient(pos, m, w, box, r_s, r_cut, workers=1)
    for k in [0, 5, 70, 300]:
        h = 1e-3 * m[k]
        mp_, mm_ = m.copy(), m.copy()
        mp_[k] += h
        mm_[k] -= h
        fd = (direct.loss(pos, mp_, w, box, r_s, r_cut, workers=1)
              - direct.loss(pos, mm_, w, box, r_s, r_cut, workers=1)) / (2 * h)
        assert gm[k] == pytest.approx(fd, rel=1e-8, abs=1e-10 * abs(gm).max())


def test_gradient_position_matches_fd(grad_case):
    pos, m, w, box, r_s, r_cut = grad_case
    gx, _ = direct.gradient(pos, m, w, box, r_s, r_cut, workers=1)
    dg = box / 16
    h = 1e-4 * dg
    checked = 0
    for k in [1, 3, 10, 55, 120, 250, 399]:
        d = direct.image_displacement(pos[k][None, :], pos, box)
        r = np.linalg.norm(d, axis=1)
        if np.any(np.abs(r - r_cut) < 2 * h):
            continue                      # the cutoff's delta function
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, a] += h
            pm[k, a] -= h
            fd = (direct.loss(pp, m, w, box, r_s, r_cut, workers=1)
                  - direct.loss(pm, m, w, box, r_s, r_cut, workers=1)) / (2 * h)
            assert gx[k, a] == pytest.approx(fd, rel=2e-4,
                                             abs=1e-6 * np.abs(gx).max())
            checked += 1
    assert checked >= 12


def test_gradient_targets_subset(grad_case):
    pos, m, w, box, r_s, r_cut = grad_case
    gx, gm = direct.gradient(pos, m, w, box, r_s, r_cut, workers=1)
    t = np.array([9, 2, 333])
    sx, sm = direct.gradient(pos, m, w, box, r_s, r_cut, targets=t, workers=1)
    assert np.allclose(sx, gx[t], rtol=0, atol=0)
    assert np.allclose(sm, gm[t], rtol=0, atol=0)

"""Pins of the oracle's truncated FMM.

P2M/M2M and L2L are checked against direct expansion about the new centre,
M2L/L2P against the brute-force sum (error falling with the order p), and
the whole FMM against brute force on clustered inputs.
"""

import math

import numpy as np
import pytest

from oracle import direct, fmm, metrics
from oracle import truncation as tr
from oracle import tree as T
from paper_2107_14008_amd import inputs


@pytest.fixture(scope="module")
def small():
    return inputs.clustered_small(12, 31, halo_frac=0.5, n_halos=3,
                                  max_leaf=16)


def test_m2m_equals_direct_p2m(small):
    w = small
    p = 4
    tree = T.build_orb(w.pos, 16)
    M = fmm.m2m(tree, fmm.p2m(tree, w.pos, w.mass, p), p)
    c = tree.centre
    for cell in [0, 1, 2, 5, len(tree.lo) // 2]:
        idx = tree.perm[tree.first[cell]:tree.first[cell] + tree.count[cell]]
        v = c[cell][None, :] - w.pos[idx]
        for k in tr.multi_indices(p):
            direct_val = np.sum(w.mass[idx] * np.prod(
                [v[:, a] ** k[a] / math.factorial(k[a]) for a in range(3)], 0))
            scale = np.sum(w.mass[idx] * np.linalg.norm(v, axis=1) ** sum(k))
            assert abs(M[k][cell] - direct_val) <= 1e-12 * scale


def test_l2l_is_exact_translation(small):
    w = small
    p = 4
    tree = T.build_orb(w.pos, 16)
    rng = np.random.default_rng(2)
    mi = tr.multi_indices(p)
    L = {k: np.zeros(len(tree.lo)) for k in mi}
    for k in mi:
        L[k][0] = rng.standard_normal()
    L = fmm.l2l(tree, L, p)
    c = tree.centre
    leaf = tree.leaf_cell[3]
    x = c[leaf] + 0.3 * rng.standard_normal((5, 3))

    def evaluate(cell):
        u = x - c[cell][None, :]
        return sum(L[k][cell] * np.prod([u[:, a] ** k[a] / math.factorial(k[a])
                                         for a in range(3)], 0) for k in mi)
    assert np.allclose(evaluate(leaf), evaluate(0), rtol=1e-11, atol=1e-12)


def _two_clumps():
    rng = np.random.default_rng(5)
    a = 20.0 + 0.15 * rng.standard_normal((300, 3))
    b = 20.0 + np.array([1.6, 0.4, -0.3]) + 0.15 * rng.standard_normal((300, 3))
    pos = np.concatenate([a, b])
    return pos, np.full(600, 1.0 / 600), 50.0, 1.0, 4.5


def test_m2l_error_falls_with_order():
    pos, m, box, r_s, r_cut = _two_clumps()
    ref, _ = direct.all_pairs(pos, m, box, r_s, r_cut)
    errs = []
    for p in range(0, 7):
        acc, near, far, tree, lists = fmm.fmm_forces(
            pos, m, box, r_s, r_cut, 16, p, 0.3, return_parts=True)
        assert len(lists.m2l) > 0
        errs.append(metrics.error_summary(acc, ref)["p99"])
    assert errs[-1] < 1e-5
    for lo, hi in zip(errs[2:], errs[1:-1]):
        assert lo < hi


def test_theta_zero_is_brute_force(small):
    w = small
    ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                workers=1)
    acc = fmm.fmm_forces(w.pos, w.mass, w.box, w.r_s, w.r_cut, 16, 4, 0.0)
    assert metrics.error_summary(acc, ref)["max"] < 1e-13


def test_fmm_accuracy_on_clustered(small):
    w = small
    ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                workers=1)
    errs = []
    for theta in (0.35, 0.3, 0.25):
        acc, near, far, tree, lists = fmm.fmm_forces(
            w.pos, w.mass, w.box, w.r_s, w.r_cut, 16, 4, theta,
            return_parts=True)
        assert len(lists.m2l) > 0
        errs.append(metrics.error_summary(acc, ref)["p999"])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4
    # the far field carries a real share of the force in the halo
    assert np.max(np.linalg.norm(far, axis=1)) > 1e-3 * np.max(
        np.linalg.norm(ref, axis=1))

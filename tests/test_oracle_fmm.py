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


# ---- the oracle's FMM adjoint (tree, lists and centres held fixed)

def _far_loss(pos, mass, w, box, r_s, r_cut, p, tree, lists):
    _, _, far, _, _ = fmm.fmm_forces(pos, mass, box, r_s, r_cut, 16, p, 0.3,
                                     tree=tree, lists=lists, return_parts=True)
    return float(np.sum(w * far))


def test_far_gradient_matches_finite_differences():
    """The far-field force is a polynomial in the positions and linear in
    the masses once the centres are fixed, so central differences pin the
    transposed operators (a dropped term, a sign or a transposed index in
    any of them shows here)."""
    pos, m, box, r_s, r_cut = _two_clumps()
    m = m * np.random.default_rng(3).uniform(0.5, 1.5, len(m))
    p = 3
    tree = T.build_orb(pos, 16)
    lists = T.dual_walk(tree, box, r_cut, 0.3, True)
    assert len(lists.m2l) > 0
    w = np.random.default_rng(4).standard_normal(pos.shape)
    gx, gm = fmm.far_gradient(tree, lists, pos, m, w, box, r_s, p)
    h = 1e-4
    for k in (0, 123, 301, 599):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[k, a] += h
            pm[k, a] -= h
            fd = (_far_loss(pp, m, w, box, r_s, r_cut, p, tree, lists)
                  - _far_loss(pm, m, w, box, r_s, r_cut, p, tree, lists)) / (2 * h)
            assert abs(fd - gx[k, a]) <= 1e-6 * (abs(gx[k, a]) + np.abs(gx).max() * 1e-3), (k, a)
        mp, mm = m.copy(), m.copy()
        mp[k] += 1e-3
        mm[k] -= 1e-3
        fd = (_far_loss(pos, mp, w, box, r_s, r_cut, p, tree, lists)
              - _far_loss(pos, mm, w, box, r_s, r_cut, p, tree, lists)) / 2e-3
        assert abs(fd - gm[k]) <= 1e-9 * (abs(gm[k]) + np.abs(gm).max()), k


def test_p2p_gradient_at_theta_zero_is_brute_force(small):
    """With theta = 0 the P2P lists hold every pair within the cutoff, so the
    list-based transpose equals the cell-list brute-force gradient."""
    w = small
    cot = np.random.default_rng(6).standard_normal(w.pos.shape)
    ref_x, ref_m, sx, sm = direct.gradient(w.pos, w.mass, cot, w.box, w.r_s,
                                           w.r_cut, workers=1, with_scale=True)
    gx, gm = fmm.fmm_gradient(w.pos, w.mass, cot, w.box, w.r_s, w.r_cut, 16,
                              4, 0.0)
    assert np.all(np.abs(gx - ref_x) <= 1e-13 * sx[:, None] + 1e-300)
    assert np.all(np.abs(gm - ref_m) <= 1e-13 * sm + 1e-300)


def test_fmm_gradient_approaches_brute_force():
    """The FMM adjoint converges to the brute-force gradient as p grows."""
    pos, m, box, r_s, r_cut = _two_clumps()
    cot = np.random.default_rng(8).standard_normal(pos.shape)
    ref_x, ref_m = direct.gradient(pos, m, cot, box, r_s, r_cut, workers=1)
    ex, em = [], []
    for p in (1, 3, 5):
        gx, gm, fx, fm, tree, lists = fmm.fmm_gradient(
            pos, m, cot, box, r_s, r_cut, 16, p, 0.3, return_parts=True)
        assert len(lists.m2l) > 0
        ex.append(np.median(np.linalg.norm(gx - ref_x, axis=1)
                            / np.linalg.norm(ref_x, axis=1)))
        em.append(np.median(np.abs(gm - ref_m) / np.abs(ref_m)))
    assert ex[0] > ex[1] > ex[2] and em[0] > em[1] > em[2]
    assert ex[2] < 1e-4 and em[2] < 1e-4
    # the far field carries a real share of the gradient (close pairs,
    # with their 1/r^3 terms, set the largest entries of it)
    assert np.max(np.linalg.norm(fx, axis=1)) > 1e-3 * np.median(np.linalg.norm(ref_x, axis=1))
    assert np.max(np.abs(fm)) > 1e-3 * np.median(np.abs(ref_m))


def test_centre_cut_fmm_converges_to_its_cell_pair_sum():
    """With the literal (centre-distance) cut an M2L task stands for every
    particle pair of its two cells with the untruncated kernel psi_s, and
    an accepted pair beyond r_cut for none: the FMM converges in p to that
    sum, which differs from the truncated pair sum when clumps sit about
    r_cut apart."""
    rng = np.random.default_rng(9)
    a = 20.0 + 0.4 * rng.standard_normal((300, 3))
    b = 20.0 + np.array([4.3, 0.0, 0.0]) + 0.4 * rng.standard_normal((300, 3))
    pos = np.concatenate([a, b])
    m = np.full(600, 1.0 / 600)
    box, r_s, r_cut = 50.0, 1.0, 4.5
    sv = T.shift_vectors() * box
    errs = []
    for p in (1, 3, 5):
        acc, near, far, tree, lists = fmm.fmm_forces(
            pos, m, box, r_s, r_cut, 16, p, 0.35, return_parts=True,
            centre_cut=True)
        assert len(lists.m2l) > 0
        ref = near.copy()
        for t, u, s in lists.m2l:
            ia = tree.perm[tree.first[t]:tree.first[t] + tree.count[t]]
            ib = tree.perm[tree.first[u]:tree.first[u] + tree.count[u]]
            d = (pos[ib][None, :, :] - pos[ia][:, None, :]) + sv[s]
            r = np.linalg.norm(d, axis=-1)
            g = m[ib][None, :] * tr.T_of_r(r, r_s) / r ** 3
            ref[ia] += np.einsum("ij,ijk->ik", g, d)
        errs.append(metrics.error_summary(acc, ref)["median"])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 5e-6
    plain = fmm.fmm_forces(pos, m, box, r_s, r_cut, 16, 5, 0.35)
    brute, _ = direct.all_pairs(pos, m, box, r_s, r_cut)
    # the default cut converges to the truncated pair sum, the centre cut
    # does not (pairs across r_cut inside accepted cell pairs)
    assert metrics.error_summary(plain, brute)["median"] < 1e-6
    assert metrics.error_summary(acc, brute)["median"] > 10 * errs[2]

"""Pins of the oracle's ORB tree and dual walk.

The lists are checked against the brute-force neighbour sets: every particle
pair inside the cutoff must be covered exactly once, either by a P2P task
whose per-pair test accepts it or by an M2L cell pair lying wholly inside
the cutoff.
"""

import numpy as np
import pytest

from oracle import direct
from oracle import tree as T
from paper_2107_14008_amd import inputs


@pytest.fixture(scope="module")
def clustered():
    return inputs.clustered_small(14, 21, halo_frac=0.5, n_halos=3,
                                  max_leaf=16)


def test_tree_invariants(clustered):
    w = clustered
    tr = T.build_orb(w.pos, 16)
    n = len(w.pos)
    assert np.array_equal(np.sort(tr.perm), np.arange(n))
    assert tr.first[0] == 0 and tr.count[0] == n
    for c in range(len(tr.lo)):
        idx = tr.perm[tr.first[c]:tr.first[c] + tr.count[c]]
        assert np.array_equal(tr.lo[c], w.pos[idx].min(0))
        assert np.array_equal(tr.hi[c], w.pos[idx].max(0))
        if tr.leaf_of_cell[c] >= 0:
            assert 1 <= tr.count[c] <= 16
            assert np.all(np.diff(idx) > 0)       # ascending original index
            continue
        l, r = tr.child[c]
        assert l == c + 1                          # pre-order numbering
        assert tr.count[l] == tr.count[c] // 2
        assert tr.count[l] + tr.count[r] == tr.count[c]
        assert tr.first[l] == tr.first[c]
        assert tr.first[r] == tr.first[c] + tr.count[l]
        ext = tr.hi[c] - tr.lo[c]
        ax = int(np.argmax(ext))
        li = tr.perm[tr.first[l]:tr.first[l] + tr.count[l]]
        ri = tr.perm[tr.first[r]:tr.first[r] + tr.count[r]]
        kl = np.max(np.stack([w.pos[li, ax], li], 1).tolist(), axis=0)
        # every left particle precedes every right one by (coordinate, index)
        left_max = max(zip(w.pos[li, ax], li))
        right_min = min(zip(w.pos[ri, ax], ri))
        assert left_max < right_min
    leaves = tr.leaf_cell
    assert np.all(np.diff(tr.first[leaves]) > 0)
    assert tr.first[leaves[-1]] + tr.count[leaves[-1]] == n


def test_power_of_two_gives_full_leaves():
    pos = inputs.uniform(4096, 100.0, 3)
    tr = T.build_orb(pos, 32)
    assert tr.n_leaves == 128
    assert np.all(tr.leaf_count == 32)


def _covered_pairs(w, tr, lists):
    """(i, j) original-index pairs covered by P2P (with the cutoff test) and
    by M2L (whole cell pairs)."""
    pos = w.pos
    rc2 = w.r_cut * w.r_cut
    sv = T.shift_vectors() * w.box
    lf, lc = tr.leaf_first, tr.leaf_count
    p2p_pairs = []
    for i, j, s in lists.p2p:
        a = tr.perm[lf[i]:lf[i] + lc[i]]
        b = tr.perm[lf[j]:lf[j] + lc[j]]
        d = (pos[b][None, :, :] - pos[a][:, None, :]) + sv[s]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ok = (r2 > 0) & (r2 < rc2)
        ii, jj = np.nonzero(ok)
        p2p_pairs.append(np.stack([a[ii], b[jj]], 1))
    m2l_pairs = []
    for t, u, s in lists.m2l:
        a = tr.perm[tr.first[t]:tr.first[t] + tr.count[t]]
        b = tr.perm[tr.first[u]:tr.first[u] + tr.count[u]]
        d = (pos[b][None, :, :] - pos[a][:, None, :]) + sv[s]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        assert np.all((r2 > 0) & (r2 < rc2)), "M2L pair crosses the cutoff"
        ii, jj = np.meshgrid(a, b, indexing="ij")
        m2l_pairs.append(np.stack([ii.ravel(), jj.ravel()], 1))
    p2p_pairs = np.concatenate(p2p_pairs) if p2p_pairs else np.zeros((0, 2), int)
    m2l_pairs = np.concatenate(m2l_pairs) if m2l_pairs else np.zeros((0, 2), int)
    return p2p_pairs, m2l_pairs


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.6])
def test_every_pair_covered_exactly_once(clustered, theta):
    w = clustered
    tr = T.build_orb(w.pos, 16)
    lists = T.dual_walk(tr, w.box, w.r_cut, theta, far_field=True)
    if theta == 0.0:
        assert len(lists.m2l) == 0
    else:
        assert len(lists.m2l) > 0
    p2p_pairs, m2l_pairs = _covered_pairs(w, tr, lists)
    allp = np.concatenate([p2p_pairs, m2l_pairs])
    n = len(w.pos)
    key = allp[:, 0] * n + allp[:, 1]
    assert len(np.unique(key)) == len(key), "a pair is covered twice"
    _, cnt = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                workers=1)
    got = np.bincount(allp[:, 0], minlength=n)
    assert np.array_equal(got, cnt)


def test_lists_are_symmetric(clustered):
    w = clustered
    tr = T.build_orb(w.pos, 16)
    lists = T.dual_walk(tr, w.box, w.r_cut, 0.4, far_field=True)
    neg = 26 - np.arange(27)            # code of -s
    for arr in (lists.p2p, lists.m2l):
        a = {tuple(x) for x in arr.tolist()}
        b = {(j, i, int(neg[s])) for i, j, s in arr.tolist()}
        assert a == b


def test_far_field_off_gives_no_m2l(clustered):
    w = clustered
    tr = T.build_orb(w.pos, 16)
    lists = T.dual_walk(tr, w.box, w.r_cut, 0.5, far_field=False)
    assert len(lists.m2l) == 0
    assert np.all(np.diff(lists.p2p_row) >= 0)
    assert lists.p2p_row[-1] == len(lists.p2p)
    # canonical order
    k = lists.p2p
    order = np.lexsort((k[:, 2], k[:, 1], k[:, 0]))
    assert np.array_equal(order, np.arange(len(k)))


def _pairs_within(w, tr, rows, leaf_ids):
    """Original-index pairs inside the cutoff of the particle pairs of the
    given (t, u, s) rows (leaf ids for P2P rows, cell ids otherwise)."""
    pos = w.pos
    rc2 = w.r_cut * w.r_cut
    sv = T.shift_vectors() * w.box
    out = []
    for t, u, s in rows:
        if leaf_ids:
            a = tr.perm[tr.leaf_first[t]:tr.leaf_first[t] + tr.leaf_count[t]]
            b = tr.perm[tr.leaf_first[u]:tr.leaf_first[u] + tr.leaf_count[u]]
        else:
            a = tr.perm[tr.first[t]:tr.first[t] + tr.count[t]]
            b = tr.perm[tr.first[u]:tr.first[u] + tr.count[u]]
        d = (pos[b][None, :, :] - pos[a][:, None, :]) + sv[s]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ii, jj = np.nonzero((r2 > 0) & (r2 < rc2))
        out.append(np.stack([a[ii], b[jj]], 1))
    return np.concatenate(out) if out else np.zeros((0, 2), int)


@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_centre_cut_covers_every_pair_once(clustered, theta):
    """The literal reading: accepted pairs go to M2L by centre distance or
    are dropped; every particle pair inside the cutoff is then in exactly
    one P2P task, M2L task or dropped pair."""
    w = clustered
    tr = T.build_orb(w.pos, 16)
    dropped = []
    lists = T.dual_walk(tr, w.box, w.r_cut, theta, True, centre_cut=True,
                        dropped=dropped)
    dropped = np.concatenate(dropped) if dropped else np.zeros((0, 3), int)
    assert len(lists.m2l) > 0 and len(dropped) > 0
    c, rad = tr.centre, tr.radius
    sv = T.shift_vectors() * w.box
    rc2 = w.r_cut * w.r_cut
    for rows, inside in ((lists.m2l, True), (dropped, False)):
        t, u, s = rows[:, 0], rows[:, 1], rows[:, 2]
        R = (c[u] - c[t]) + sv[s]
        R2 = (R[:, 0] * R[:, 0] + R[:, 1] * R[:, 1]) + R[:, 2] * R[:, 2]
        lhs = rad[t] + rad[u]
        assert np.all(lhs * lhs < theta * theta * R2)
        assert np.all((R2 < rc2) == inside)
    allp = np.concatenate([_pairs_within(w, tr, lists.p2p, True),
                           _pairs_within(w, tr, lists.m2l, False),
                           _pairs_within(w, tr, dropped, False)])
    n = len(w.pos)
    key = allp[:, 0] * n + allp[:, 1]
    assert len(np.unique(key)) == len(key), "a pair is covered twice"
    _, cnt = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                workers=1)
    assert np.array_equal(np.bincount(allp[:, 0], minlength=n), cnt)
    # the default reading on the same tree sends none of these to M2L
    # without the whole pair inside the cutoff
    plain = T.dual_walk(tr, w.box, w.r_cut, theta, True)
    assert len(plain.m2l) != len(lists.m2l) or not np.array_equal(plain.m2l, lists.m2l)

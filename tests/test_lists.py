"""The host planner's tree and task lists equal the oracle's, integer for
integer and bit for bit (the oracle builds them independently in numpy from
the same written rules).  CPU only: planning touches no GPU."""

import numpy as np
import pytest

from oracle import tree as T
from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs


def host_lists(pos, mass, box, r_s, r_cut, max_leaf, order, theta, threads=0,
               m2l_cut=B.M2L_INSIDE):
    ctx = B.Context(box=box, r_s=r_s, r_cut=r_cut, max_leaf=max_leaf,
                    order=order, theta=theta, threads=threads, m2l_cut=m2l_cut)
    ctx.plan(pos, mass)
    return ctx.lists()


def assert_same(L, tree, lists):
    assert np.array_equal(L["perm"], tree.perm)
    assert L["n_cells"] == len(tree.lo)
    assert np.array_equal(L["cell_first"], tree.first)
    assert np.array_equal(L["cell_count"], tree.count)
    assert np.array_equal(L["cell_child"], tree.child)
    assert np.array_equal(L["cell_lo"], tree.lo)      # bit-exact floats
    assert np.array_equal(L["cell_hi"], tree.hi)
    assert np.array_equal(L["leaf_cell"], tree.leaf_cell)
    assert np.array_equal(L["leaf_first"], tree.leaf_first)
    assert np.array_equal(L["leaf_count"], tree.leaf_count)
    assert np.array_equal(L["p2p_row"], lists.p2p_row)
    assert np.array_equal(L["p2p_j"], lists.p2p[:, 1])
    assert np.array_equal(L["p2p_shift"], lists.p2p[:, 2])
    assert np.array_equal(L["m2l_row"], lists.m2l_row)
    assert np.array_equal(L["m2l_src"], lists.m2l[:, 1])
    assert np.array_equal(L["m2l_shift"], lists.m2l[:, 2])
    assert L["candidate_pairs"] == T.candidate_pairs(tree, lists)


def oracle_lists(pos, box, r_cut, max_leaf, order, theta, centre_cut=False):
    tree = T.build_orb(pos, max_leaf)
    lists = T.dual_walk(tree, box, r_cut, theta, order >= 0, centre_cut)
    return tree, lists


def test_uniform_32k_p2p_only():
    w = inputs.uniform_32k()
    L = host_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, w.max_leaf, -1, 0.0)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, w.max_leaf, -1, 0.0)
    assert len(lists.m2l) == 0
    assert_same(L, tree, lists)
    assert L["n_leaves"] == 1024 and np.all(L["leaf_count"] == 32)


@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_clustered_centre_cut(theta):
    """The literal (centre-distance) M2L cut: same lists as the oracle."""
    w = inputs.clustered_small(20, 41, halo_frac=0.4, n_halos=5, max_leaf=24)
    L = host_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 24, 4, theta,
                   m2l_cut=B.M2L_CENTRE)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 24, 4, theta, True)
    assert len(lists.m2l) > 0
    assert_same(L, tree, lists)


@pytest.mark.parametrize("theta", [0.25, 0.5])
def test_clustered_with_far_field(theta):
    w = inputs.clustered_small(20, 41, halo_frac=0.4, n_halos=5, max_leaf=24)
    L = host_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 24, 4, theta)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 24, 4, theta)
    assert len(lists.m2l) > 0
    assert_same(L, tree, lists)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_thread_count_does_not_change_lists(threads):
    w = inputs.clustered_small(16, 43, max_leaf=16)
    L = host_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 16, 4, 0.3, threads)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 16, 4, 0.3)
    assert_same(L, tree, lists)


@pytest.mark.parametrize("n,max_leaf", [(1, 8), (2, 1), (7, 8), (9, 8),
                                        (1000, 1), (1001, 64), (4095, 33)])
def test_ragged_sizes(n, max_leaf):
    rng = np.random.default_rng(n)
    pos = rng.uniform(0, 20.0, (n, 3))
    m = rng.uniform(0.1, 1.0, n)
    L = host_lists(pos, m, 20.0, 0.6, 2.7, max_leaf, 3, 0.4)
    tree, lists = oracle_lists(pos, 20.0, 2.7, max_leaf, 3, 0.4)
    assert_same(L, tree, lists)
    assert np.all(L["leaf_count"] <= max_leaf)


def test_ties_and_duplicates():
    """Equal coordinates are split by caller index; coincident particles."""
    rng = np.random.default_rng(5)
    g = np.arange(8) * 2.5
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = np.concatenate([pos, pos[:40], rng.uniform(0, 20, (30, 3))])
    m = np.ones(len(pos))
    L = host_lists(pos, m, 20.0, 0.7, 3.15, 8, 4, 0.5)
    tree, lists = oracle_lists(pos, 20.0, 3.15, 8, 4, 0.5)
    assert_same(L, tree, lists)


def test_batch_matches_per_box():
    boxes = [inputs.clustered_small(n, 100 + n, max_leaf=32, order=-1)
             for n in (12, 16, 14)]
    ctx = B.Context()
    per_box = [B.make_params(box=w.box, r_s=w.r_s, r_cut=w.r_cut,
                             max_leaf=w.max_leaf, order=-1, theta=0.0)
               for w in boxes]
    counts = [len(w.mass) for w in boxes]
    pos = np.concatenate([w.pos for w in boxes])
    mass = np.concatenate([w.mass for w in boxes])
    ctx.plan_batch(per_box, counts, pos, mass)
    L = ctx.lists()
    p0 = 0
    for b, w in enumerate(boxes):
        tree, lists = oracle_lists(w.pos, w.box, w.r_cut, w.max_leaf, -1, 0.0)
        l0, l1 = L["box_first_leaf"][b], L["box_first_leaf"][b + 1]
        c0 = L["box_first_cell"][b]
        assert l1 - l0 == tree.n_leaves
        assert np.array_equal(L["perm"][p0:p0 + len(w.mass)] - p0, tree.perm)
        rows = L["p2p_row"][l0:l1 + 1]
        assert np.array_equal(rows - rows[0], lists.p2p_row)
        assert np.array_equal(L["p2p_j"][rows[0]:rows[-1]] - l0, lists.p2p[:, 1])
        assert np.array_equal(L["cell_child"][c0:c0 + len(tree.lo)],
                              np.where(tree.child >= 0, tree.child + c0, -1))
        p0 += len(w.mass)


def test_clustered_2m_headline_lists():
    """The headline workload itself (128^3 clustered, leaf <= 64, p = 4,
    theta = 0.25): 32,768 leaves, ~2.7 million P2P and some hundred M2L
    tasks, integer for integer and bit for bit against the oracle
    (about 15 s of CPU)."""
    w = inputs.clustered_2m()
    L = host_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64, 4, 0.25)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 64, 4, 0.25)
    assert L["n_leaves"] == 32768 and len(lists.m2l) > 0
    assert_same(L, tree, lists)

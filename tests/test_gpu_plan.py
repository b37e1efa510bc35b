"""The on-GPU planner (pmfmm_build with planner = 0) yields the same tree
and task lists as the oracle's independent builder, bit for bit, and the same
work items as the host planner."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs
from oracle import tree as T
from test_lists import assert_same, oracle_lists

pytestmark = pytest.mark.gpu


def gpu_lists(pos, mass, box, r_s, r_cut, max_leaf, order, theta, **kw):
    ctx = B.Context(box=box, r_s=r_s, r_cut=r_cut, max_leaf=max_leaf,
                    order=order, theta=theta, planner=0, **kw)
    ctx.build(torch.tensor(pos, device="cuda"), torch.tensor(mass, device="cuda"))
    return ctx.lists(), ctx


def test_uniform_32k():
    w = inputs.uniform_32k()
    print("case: gpu plan uniform 32^3", flush=True)
    L, _ = gpu_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, w.max_leaf, -1, 0.0)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, w.max_leaf, -1, 0.0)
    assert_same(L, tree, lists)


@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_clustered_centre_cut(theta):
    w = inputs.clustered_small(20, 41, halo_frac=0.4, n_halos=5, max_leaf=24)
    print(f"case: gpu plan centre cut theta {theta}", flush=True)
    L, _ = gpu_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 24, 4, theta,
                     m2l_cut=B.M2L_CENTRE)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 24, 4, theta, True)
    assert len(lists.m2l) > 0
    assert_same(L, tree, lists)


@pytest.mark.parametrize("theta", [0.25, 0.5])
def test_clustered_with_far_field(theta):
    w = inputs.clustered_small(20, 41, halo_frac=0.4, n_halos=5, max_leaf=24)
    print(f"case: gpu plan clustered 20^3 theta {theta}", flush=True)
    L, _ = gpu_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 24, 4, theta)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 24, 4, theta)
    assert len(lists.m2l) > 0
    assert_same(L, tree, lists)


def test_second_build_of_a_shape_gives_the_same_lists():
    """The second build of a tree shape walks without host round trips."""
    w = inputs.clustered_small(20, 41, halo_frac=0.4, n_halos=5, max_leaf=24)
    ctx = B.Context(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=24, order=4,
                    theta=0.4)
    tree, lists = oracle_lists(w.pos, w.box, w.r_cut, 24, 4, 0.4)
    p = torch.tensor(w.pos, device="cuda")
    m = torch.tensor(w.mass, device="cuda")
    for _ in range(3):
        ctx.build(p, m)
        assert_same(ctx.lists(), tree, lists)
    moved = inputs.wrap(w.pos + 0.37, w.box)
    ctx.build(torch.tensor(moved, device="cuda"), m)
    tree2, lists2 = oracle_lists(moved, w.box, w.r_cut, 24, 4, 0.4)
    assert_same(ctx.lists(), tree2, lists2)


# (1000, 1): subtrees are cut by their cell count (512), not their particle
# count; (4097, 8): one level in the level loop above the fused subtrees.
@pytest.mark.parametrize("n,max_leaf", [(1, 8), (2, 1), (7, 8), (9, 8),
                                        (1000, 1), (1001, 64), (4095, 33),
                                        (4097, 8)])
def test_ragged_sizes(n, max_leaf):
    rng = np.random.default_rng(n)
    pos = rng.uniform(0, 20.0, (n, 3))
    m = rng.uniform(0.1, 1.0, n)
    print(f"case: gpu plan ragged n={n} leaf={max_leaf}", flush=True)
    L, _ = gpu_lists(pos, m, 20.0, 0.6, 2.7, max_leaf, 3, 0.4)
    tree, lists = oracle_lists(pos, 20.0, 2.7, max_leaf, 3, 0.4)
    assert_same(L, tree, lists)


def test_ties_duplicates_and_unwrapped():
    rng = np.random.default_rng(5)
    g = np.arange(8) * 2.5
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos = np.concatenate([pos, pos[:40], rng.uniform(0, 20, (30, 3))])
    m = np.ones(len(pos))
    shifted = pos + rng.integers(-1, 2, pos.shape) * 20.0
    print("case: gpu plan ties/duplicates", flush=True)
    L, _ = gpu_lists(shifted, m, 20.0, 0.7, 3.15, 8, 4, 0.5)
    # the oracle sees the same wrapped coordinates (x + 20 - 20 can differ
    # from x in the last bit)
    tree, lists = oracle_lists(inputs.wrap(shifted, 20.0), 20.0, 3.15, 8, 4, 0.5)
    assert_same(L, tree, lists)


# Coordinates closer together than the sort key resolves (2^-24 of the box
# here), in scrambled caller order: a run of up to 64 equal keys is put in
# coordinate order in place; a longer one out of order makes the build sort
# by the full 64-bit keys.  With `ties`, the coordinates of a run come in
# equal pairs, which keep caller order.
@pytest.mark.parametrize("group,ties", [(4, False), (4, True), (5, False), (5, True), (8, False),
                                        (64, False), (64, True), (65, False), (300, False)])
def test_coordinates_below_sort_key_resolution(group, ties):
    rng = np.random.default_rng(100 + group + 1000 * ties)
    parts = [rng.uniform(0, 20.0, (3000, 3))]
    for axis in range(3):
        for _ in range(4):
            x0 = rng.uniform(1.0, 19.0)
            close = rng.uniform(0, 20.0, (group, 3))
            step = np.arange(group) // 2 if ties else np.arange(group)
            close[:, axis] = x0 + step * 1e-12
            parts.append(close)
    pos = np.concatenate(parts)
    pos = pos[rng.permutation(len(pos))]
    m = rng.uniform(0.5, 1.0, len(pos))
    print(f"case: gpu plan sub-key-resolution runs of {group} (ties {ties})", flush=True)
    L, _ = gpu_lists(pos, m, 20.0, 0.6, 2.7, 16, 3, 0.4)
    tree, lists = oracle_lists(pos, 20.0, 2.7, 16, 3, 0.4)
    assert_same(L, tree, lists)


# One dense clump inside the cutoff: every leaf row lists every leaf, so
# the rows are longer than one wavefront sorts; with PMFMM_ROW_LDS=64 they
# are sorted in global scratch instead of LDS.
@pytest.mark.parametrize("row_lds", [None, "64"])
def test_long_task_rows(row_lds, monkeypatch):
    if row_lds is not None:
        monkeypatch.setenv("PMFMM_ROW_LDS", row_lds)
    rng = np.random.default_rng(77)
    clump = 10.0 + rng.normal(0, 0.3, (3000, 3))
    pos = np.concatenate([clump, rng.uniform(0, 20.0, (500, 3))])
    pos = pos[rng.permutation(len(pos))]
    m = np.ones(len(pos))
    print(f"case: gpu plan long rows (row lds {row_lds})", flush=True)
    L, _ = gpu_lists(pos, m, 20.0, 0.6, 2.7, 8, -1, 0.0)
    host = B.Context(box=20.0, r_s=0.6, r_cut=2.7, max_leaf=8, order=-1, theta=0.0)
    host.plan(pos, m)
    H = host.lists()
    assert int(np.diff(H["p2p_row"]).max()) > 256
    for k in ("perm", "p2p_row", "p2p_j", "p2p_shift"):
        assert np.array_equal(L[k], H[k]), k


def test_matches_oracle_and_host_planner_clustered_2m():
    """The headline workload (128^3 clustered, leaf <= 64, p = 4, theta =
    0.25): the GPU planner's tree and lists against the oracle's own
    builder, integer for integer and bit for bit, and its work items
    against the host planner's."""
    w = inputs.clustered_2m()
    print("case: gpu plan vs oracle and host plan 128^3", flush=True)
    L, ctx = gpu_lists(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64, 4, 0.25)
    tree = T.build_orb(w.pos, 64)
    lists = T.dual_walk(tree, w.box, w.r_cut, 0.25, True)
    assert len(lists.m2l) > 0
    assert np.array_equal(L["perm"], tree.perm)
    assert np.array_equal(L["cell_lo"], tree.lo)
    assert np.array_equal(L["cell_hi"], tree.hi)
    assert np.array_equal(L["leaf_first"], tree.leaf_first)
    assert np.array_equal(L["leaf_count"], tree.leaf_count)
    assert np.array_equal(L["p2p_row"], lists.p2p_row)
    assert np.array_equal(L["p2p_j"], lists.p2p[:, 1])
    assert np.array_equal(L["p2p_shift"], lists.p2p[:, 2])
    assert np.array_equal(L["m2l_row"], lists.m2l_row)
    assert np.array_equal(L["m2l_src"], lists.m2l[:, 1])
    assert np.array_equal(L["m2l_shift"], lists.m2l[:, 2])
    assert L["candidate_pairs"] == T.candidate_pairs(tree, lists)
    host = B.Context(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=64,
                     order=4, theta=0.25)
    host.plan(w.pos, w.mass)
    H = host.lists()
    for k in ("n_p2p", "n_m2l", "n_items", "candidate_pairs"):
        assert L[k] == H[k], k


def test_batch_matches_per_box():
    boxes = [inputs.clustered_small(n, 100 + n, max_leaf=32, order=-1)
             for n in (12, 16, 14)]
    ctx = B.Context(planner=0)
    per_box = [B.make_params(box=w.box, r_s=w.r_s, r_cut=w.r_cut,
                             max_leaf=w.max_leaf, order=-1, theta=0.0)
               for w in boxes]
    counts = [len(w.mass) for w in boxes]
    pos = torch.tensor(np.concatenate([w.pos for w in boxes]), device="cuda")
    mass = torch.tensor(np.concatenate([w.mass for w in boxes]), device="cuda")
    print("case: gpu plan batch of 3", flush=True)
    ctx.build_batch(per_box, counts, pos, mass)
    L = ctx.lists()
    host = B.Context()
    host.plan_batch(per_box, counts, pos.cpu().numpy(), mass.cpu().numpy())
    H = host.lists()
    for k in ("perm", "cell_lo", "cell_hi", "p2p_row", "p2p_j", "p2p_shift",
              "cell_child", "leaf_first"):
        assert np.array_equal(L[k], H[k]), k


def test_rebuild_reuses_shape_and_rejects_bad_input():
    rng = np.random.default_rng(8)
    pos = rng.uniform(0, 20.0, (3000, 3))
    m = np.ones(3000)
    ctx = B.Context(box=20.0, r_s=0.6, r_cut=2.7, max_leaf=16, order=-1)
    for k in range(3):
        p = pos + 0.01 * k
        ctx.build(torch.tensor(p, device="cuda"), torch.tensor(m, device="cuda"))
        L = ctx.lists()
        tree, lists = oracle_lists(inputs.wrap(p, 20.0), 20.0, 2.7, 16, -1, 0.0)
        assert np.array_equal(L["p2p_j"], lists.p2p[:, 1])
    bad = pos.copy()
    bad[17, 2] = np.inf
    with pytest.raises(B.PmfmmError, match="particle 17"):
        ctx.build(torch.tensor(bad, device="cuda"), torch.tensor(m, device="cuda"))
    mm = m.copy()
    mm[5] = -1.0
    with pytest.raises(B.PmfmmError, match="mass"):
        ctx.build(torch.tensor(pos, device="cuda"), torch.tensor(mm, device="cuda"))

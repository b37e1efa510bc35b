"""Pins of the oracle's error statistic and of its candidate-pair count.

Every parity verdict of the GPU tests goes through ``metrics.error_summary``
(the per-particle relative force error of the configurations' "99.9 %
relative force error" metric, the statistic of the paper's Sec. 4 precision
runs), and the headline unit is ``tree.candidate_pairs`` (the n_i n_j pairs
of every P2P task, Sec. 3.2).  Both are pinned here on hand-built inputs
whose answers are fixed by arithmetic done by hand, chosen so that a
plausible slip fails a test: a component-wise or L1/L-inf norm instead of
the row-wise Euclidean norm, an absolute instead of a relative error, the
median or a linear quantile instead of numpy's "higher" quantile, a `tiny`
cut that drops large-force particles or keeps the near-zero ones, a count
of n_i + n_j or of one side of a task only.
"""

import numpy as np
import pytest

from oracle import metrics
from oracle import tree as T
from paper_2107_14008_amd import inputs


def test_row_wise_euclidean_relative_error():
    # |ref| = 5, 10, 1; the differences have Euclidean norms 0.05, 0.3 and
    # 1e-3 (L1 would give 0.07, 0.42, 1e-3; L-inf 0.04, 0.24, 1e-3)
    ref = np.array([[3.0, 4.0, 0.0], [0.0, 6.0, 8.0], [0.0, 0.0, 1.0]])
    acc = ref + np.array([[0.03, 0.04, 0.0], [0.18, 0.0, 0.24], [1e-3, 0.0, 0.0]])
    e, tiny = metrics.relative_errors(acc, ref)
    assert not tiny.any()
    np.testing.assert_allclose(e, [0.01, 0.03, 1e-3], rtol=1e-12)


def test_error_is_relative_not_absolute():
    # the same relative error 1e-4 at force magnitudes 1e-3 .. 1e3
    mags = 10.0 ** np.arange(-3, 4)
    ref = np.stack([mags, 0 * mags, 0 * mags], 1)
    acc = ref * (1 + 1e-4)
    s = metrics.error_summary(acc, ref)
    assert s["n"] == 7 and s["tiny"] == 0
    for k in ("median", "p99", "p999", "max"):
        assert s[k] == pytest.approx(1e-4, rel=1e-9)


def test_higher_quantiles():
    # 1501 particles with errors k * 1e-6, k = 1..1501 (|ref| = 1): the
    # "higher" quantile picks an observed error at index ceil(q (n - 1)):
    # median index 750 -> 751e-6; p99 index ceil(1485) = 1485 -> 1486e-6;
    # p99.9 index ceil(1498.5) = 1499 -> 1500e-6 (linear: 1499.5e-6)
    n = 1501
    k = np.arange(1, n + 1, dtype=np.float64)
    rng = np.random.default_rng(5)
    perm = rng.permutation(n)               # order must not matter
    ref = np.zeros((n, 3))
    ref[:, 1] = 1.0
    acc = ref.copy()
    acc[:, 0] = k[perm] * 1e-6
    s = metrics.error_summary(acc, ref)
    assert s["n"] == n
    assert s["median"] == pytest.approx(751e-6, rel=1e-12)
    assert s["p99"] == pytest.approx(1486e-6, rel=1e-12)
    assert s["p999"] == pytest.approx(1500e-6, rel=1e-12)
    assert s["max"] == pytest.approx(1501e-6, rel=1e-12)


def test_even_count_median_is_the_upper_middle():
    # errors 1, 2, 3, 4 (x 1e-6): the "higher" median is 3e-6 (not 2.5e-6)
    ref = np.tile([[0.0, 0.0, 2.0]], (4, 1))
    acc = ref.copy()
    acc[:, 2] += np.array([4.0, 2.0, 8.0, 6.0]) * 1e-6
    assert metrics.error_summary(acc, ref)["median"] == pytest.approx(3e-6, rel=1e-12)


@pytest.mark.parametrize("scale", [1.0, 1e-3, 1e4])
def test_tiny_reference_forces_are_counted_apart(scale):
    # median |ref| = 1 (the middle of 1001 unit forces); two particles far
    # below 1e-6 of it carry huge relative errors and must be set apart, one
    # at 2e-6 of it is kept (its relative error 0.5 is the maximum).  The
    # whole case is scaled: the cut is relative to the median force.
    n = 1001
    ref = np.zeros((n, 3))
    ref[:, 0] = 1.0
    ref[0, 0] = 1e-9
    ref[1, 0] = 5e-7
    ref[2, 0] = 2e-6
    acc = ref.copy()
    acc[0, 0] += 1.0
    acc[1, 0] += 1.0
    acc[2, 0] += 1e-6
    acc[3:, 1] = 1e-8                        # 1e-8 relative for the rest
    ref, acc = ref * scale, acc * scale
    e, tiny = metrics.relative_errors(acc, ref)
    assert tiny.tolist()[:4] == [True, True, False, False]
    assert int(tiny.sum()) == 2
    assert e[0] == 0.0 and e[1] == 0.0
    s = metrics.error_summary(acc, ref)
    assert s["tiny"] == 2 and s["n"] == n - 2
    assert s["max"] == pytest.approx(0.5, rel=1e-12)
    assert s["median"] == pytest.approx(1e-8, rel=1e-9)


def test_all_tiny_gives_an_empty_summary():
    ref = np.zeros((3, 3))
    s = metrics.error_summary(ref + 1.0, ref)
    assert s["n"] == 0 and s["tiny"] == 3


def _isolated_cluster(n, seed):
    # n particles inside a ball of radius 1 at the centre of a box of 100,
    # cutoff 20: every particle pair is inside the cutoff, no periodic image
    # is, so with the far field off every leaf pair is one P2P task
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return 50.0 + v * rng.uniform(0, 1, (n, 1))


@pytest.mark.parametrize("n,max_leaf", [(3, 2), (37, 5), (200, 16), (64, 64)])
def test_candidate_pairs_of_an_isolated_cluster_is_n_squared(n, max_leaf):
    pos = _isolated_cluster(n, n)
    tr = T.build_orb(pos, max_leaf)
    lists = T.dual_walk(tr, 100.0, 20.0, theta=0.0, far_field=False)
    # every ordered leaf pair (self pairs included) once, unshifted
    assert len(lists.p2p) == tr.n_leaves ** 2
    assert np.all(lists.p2p[:, 2] == 13)
    assert T.candidate_pairs(tr, lists) == n * n


def test_candidate_pairs_two_leaves_by_hand():
    # three particles, MAXLEAF 2: leaves of 1 and 2 particles; the tasks
    # (0,0), (0,1), (1,0), (1,1) hold 1 + 2 + 2 + 4 = 9 pairs
    pos = np.array([[50.0, 50.0, 50.0], [50.5, 50.0, 50.0], [51.0, 50.0, 50.0]])
    tr = T.build_orb(pos, 2)
    assert sorted(tr.leaf_count.tolist()) == [1, 2]
    lists = T.dual_walk(tr, 100.0, 20.0, theta=0.0, far_field=False)
    assert len(lists.p2p) == 4
    assert T.candidate_pairs(tr, lists) == 9


def test_candidate_pairs_full_leaves_32k():
    # 32^3 uniform particles with MAXLEAF 32: 1024 leaves of exactly 32, so
    # every task holds 32 * 32 candidate pairs
    w = inputs.uniform_32k()
    tr = T.build_orb(w.pos, 32)
    assert tr.n_leaves == 1024 and np.all(tr.leaf_count == 32)
    lists = T.dual_walk(tr, w.box, w.r_cut, theta=0.0, far_field=False)
    assert T.candidate_pairs(tr, lists) == 32 * 32 * len(lists.p2p)

"""The schedule autotuner picks one of its candidates, applies it, and the
forces stay within tolerance of the oracle for every schedule."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct, metrics
from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs, tune

pytestmark = pytest.mark.gpu


def test_autotune_batch(tmp_path):
    boxes = inputs.batch_64(n_box=4, lo=16, hi=24)
    per_box = [B.make_params(box=w.box, r_s=w.r_s, r_cut=w.r_cut,
                             max_leaf=w.max_leaf, order=-1, theta=0.0)
               for w in boxes]
    counts = [len(w.mass) for w in boxes]
    pos = torch.tensor(np.concatenate([w.pos for w in boxes]), device="cuda")
    mass = torch.tensor(np.concatenate([w.mass for w in boxes]), device="cuda")
    ctx = B.Context(precision=B.PMFMM_FP32, trunc=B.TRUNC_TABLE, table_size=512,
                    table_level=2)
    ctx.build_batch(per_box, counts, pos, mass)
    out = torch.empty((sum(counts), 3), dtype=torch.float64, device="cuda")
    cands = [(0, 4, 0), (8, 2, 0), (1 << 20, 8, 0), (16, 16, 64)]
    cache = str(tmp_path / "tune.json")
    best, res = tune.autotune(ctx, out, cands=cands, repeats=2, cache_path=cache)
    assert (best["chunk"], best["wg_waves"], best["grid_wgs"]) in cands
    assert len(res) == len(cands)
    again, res2 = tune.autotune(ctx, out, cache_path=cache)   # from the cache
    assert res2 == {} and again["chunk"] == best["chunk"]
    ctx.forward(out)
    torch.cuda.synchronize()
    acc = out.cpu().numpy()
    p0 = 0
    for w, n in zip(boxes, counts):
        ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut)
        s = metrics.error_summary(acc[p0:p0 + n], ref)
        assert s["median"] <= 1e-5 and s["p999"] <= 1e-4
        p0 += n


def test_autotune_default_candidates_through_the_abi(tmp_path):
    """pmfmm_autotune with the library's 24 default schedules on a float64
    exact context: the schedules with more than 4 waves per workgroup are
    skipped (that form runs at most 4), the winner is among the timed ones,
    it is applied, and a second call takes it from the cache file."""
    w = inputs.clustered_small(16, 9)
    ctx = B.Context(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=64, order=-1,
                    precision=B.PMFMM_FP64)
    ctx.build(torch.tensor(w.pos, device="cuda"), torch.tensor(w.mass, device="cuda"))
    out = torch.empty((len(w.mass), 3), dtype=torch.float64, device="cuda")
    ref = torch.empty_like(out)
    ctx.forward(ref)
    cache = str(tmp_path / "tune.txt")
    best, timed = ctx.autotune(out, repeats=1, cache_path=cache)
    assert len(timed) == 24
    ran = [r for r in timed if r["p2p_ms"] >= 0]
    assert len(ran) == 12 and all(r["wg_waves"] <= 4 for r in ran)
    assert (best["chunk"], best["wg_waves"]) in [(r["chunk"], r["wg_waves"]) for r in ran]
    assert best["p2p_ms"] == min(r["p2p_ms"] for r in ran)
    assert (ctx.params.chunk, ctx.params.wg_waves) == (best["chunk"], best["wg_waves"])
    assert open(cache).read().count("\n") == 1
    again, timed2 = ctx.autotune(out, cache_path=cache)
    assert timed2 == []
    assert [again[k] for k in ("chunk", "wg_waves", "grid_wgs")] == \
        [best[k] for k in ("chunk", "wg_waves", "grid_wgs")]
    assert abs(again["p2p_ms"] - best["p2p_ms"]) <= 1e-6      # kept to 6 decimals
    ctx.forward(out)
    torch.cuda.synchronize()
    # workgroup size and grid leave the result bitwise alone; the work-item
    # size regroups the float64 sums (rounding only)
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    if best["chunk"] == 0:
        assert np.array_equal(a, b)
    assert np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)) <= 1e-12

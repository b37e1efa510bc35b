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

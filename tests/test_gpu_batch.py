"""Many independent boxes in one persistent launch, against the oracle per
box."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct, metrics
from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def boxes():
    return inputs.batch_64(n_box=6, lo=16, hi=28)


def run_batch(boxes, **ev):
    ctx = B.Context(**ev)
    per_box = [B.make_params(box=w.box, r_s=w.r_s, r_cut=w.r_cut,
                             max_leaf=w.max_leaf, order=-1, theta=0.0)
               for w in boxes]
    counts = [len(w.mass) for w in boxes]
    pos = torch.tensor(np.concatenate([w.pos for w in boxes]), device="cuda")
    mass = torch.tensor(np.concatenate([w.mass for w in boxes]),
                        device="cuda")
    ctx.build_batch(per_box, counts, pos, mass)
    out = torch.empty((sum(counts), 3), dtype=torch.float64, device="cuda")
    ctx.forward(out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), counts


@pytest.mark.parametrize("prec,trunc", [(B.PMFMM_FP64, B.TRUNC_EXACT),
                                        (B.PMFMM_FP32, B.TRUNC_TABLE),
                                        (B.PMFMM_FP32, B.TRUNC_EXACT),
                                        (B.PMFMM_FP32, B.TRUNC_R2)])
def test_batch_against_oracle(boxes, prec, trunc):
    print(f"case: batch of {len(boxes)} boxes prec {prec} trunc {trunc}",
          flush=True)
    acc, counts = run_batch(boxes, precision=prec, trunc=trunc,
                            table_size=64 if trunc == B.TRUNC_R2 else 2048,
                            table_level=2)
    p0 = 0
    for w, n in zip(boxes, counts):
        ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut)
        s = metrics.error_summary(acc[p0:p0 + n], ref)
        if prec == B.PMFMM_FP64:
            assert s["max"] <= 1e-12, s
        else:
            assert s["median"] <= 1e-5 and s["p999"] <= 1e-4, s
        p0 += n

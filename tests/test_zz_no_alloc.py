"""pmfmm_forward_static (the forward that allocates nothing: its scratch is
a static device array of the library) against pmfmm_forward on the same
builds: bit for bit, on two calls in a row, the second with a smaller
input, and its refusals (plan too large for the array, table not current)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct, metrics
from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(ctx, n, stream):
    ref = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    out = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
    ctx.forward(ref, stream)
    ctx.forward_static(out, stream)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_forward_matches_forward_twice_larger_then_smaller():
    stream = torch.cuda.current_stream()
    cases = [
        # 64^3 clustered (262,144 particles), float32 r^2 table, P2P only
        (inputs.clustered_262k(), dict(order=-1, theta=0.0, precision=B.PMFMM_FP32,
                                       trunc=B.TRUNC_R2, table_size=64, table_level=2)),
        # 32^3 clustered with two halos close enough for M2L tasks, float64
        # exact with the far field on (p = 4, theta = 0.25)
        (inputs.clustered_small(32, 14017, halo_frac=0.5, n_halos=4),
         dict(order=4, theta=0.25, precision=B.PMFMM_FP64)),
    ]
    for w, ev in cases:
        n = len(w.mass)
        print(f"case: forward_static, {w.name} ({n} particles), {ev}", flush=True)
        ctx = B.Context(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=w.max_leaf, **ev)
        ctx.build(torch.tensor(w.pos, device="cuda"), torch.tensor(w.mass, device="cuda"), stream)
        L = ctx.lists()
        print(f"  {L['n_items']} work items, {L['n_m2l']} M2L tasks", flush=True)
        assert ev["order"] < 0 or L["n_m2l"] > 0
        ref, out = _pair(ctx, n, stream)
        assert np.array_equal(ref, out), np.abs(ref - out).max()
        # and a second static call on the same build (counters cleared again)
        out2 = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        ctx.forward_static(out2, stream)
        torch.cuda.synchronize()
        assert np.array_equal(ref, out2.cpu().numpy())
        # spot check against the oracle (the forward's own parity tests cover the rest)
        idx = np.arange(0, n, max(1, n // 300))
        a_ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut, targets=idx)
        s = metrics.error_summary(out[idx], a_ref)
        print(f"  vs oracle: {s}", flush=True)
        assert s["p999"] <= 1e-4
        ctx.close()


def test_static_forward_refusals():
    stream = torch.cuda.current_stream()
    w = inputs.clustered_small(16, 3, max_leaf=32)
    n = len(w.mass)
    ctx = B.Context(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=32, order=-1,
                    precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=64, table_level=2)
    out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PmfmmError):           # not built
        ctx.forward_static(out, stream)
    ctx.build(torch.tensor(w.pos, device="cuda"), torch.tensor(w.mass, device="cuda"), stream)
    ctx.set_eval(precision=B.PMFMM_FP32, trunc=B.TRUNC_TABLE, table_size=512, table_level=2)
    with pytest.raises(B.PmfmmError, match="ESTATE"):   # table not on the device yet
        ctx.forward_static(out, stream)
    ref, got = _pair(ctx, n, stream)             # pmfmm_forward uploads it
    assert np.array_equal(ref, got)
    ctx.close()
    # a plan with more work items than the array holds
    big = inputs.clustered_2m()
    ctx = B.Context(box=big.box, r_s=big.r_s, r_cut=big.r_cut, max_leaf=64, order=-1,
                    precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=64, table_level=2)
    ctx.build(torch.tensor(big.pos, device="cuda"), torch.tensor(big.mass, device="cuda"), stream)
    print(f"case: refusal, {ctx.lists()['n_items']} work items", flush=True)
    big_out = torch.empty((len(big.mass), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PmfmmError, match="EINVAL"):
        ctx.forward_static(big_out, stream)
    ctx.close()

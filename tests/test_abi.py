"""CPU checks of the C ABI: the library loads, exports every declared entry
point, validates its arguments and refuses calls made out of order.  None of
these calls touches a GPU."""

import math
import os
import re

import numpy as np
import pytest

from paper_2107_14008_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    return B.library()


def declared_functions(root):
    names = set()
    inc = os.path.join(root, "include")
    for h in sorted(os.listdir(inc)):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(inc, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(pmfmm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(lib, repo_root):
    names = declared_functions(repo_root)
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.SIGNATURES)


def test_version(lib):
    assert lib.pmfmm_version().decode().startswith("pmfmm")


@pytest.mark.parametrize("field,value", [
    ("box", 0.0), ("box", float("nan")), ("r_s", -1.0), ("r_cut", 60.0),
    ("r_cut", 0.0), ("theta", 1.0), ("theta", -0.1), ("max_leaf", 0),
    ("max_leaf", 65), ("order", 7), ("precision", 2), ("trunc", 5),
    ("table_size", 8), ("table_level", 5), ("table_round", 3),
    ("chunk", -1), ("wg_waves", 17), ("G", float("inf")), ("accum", 2),
])
def test_create_rejects_bad_params(field, value):
    with pytest.raises(B.PmfmmError) as e:
        B.Context(**{field: value})
    assert e.value.code == -1


def test_table_range_checked():
    # r_cut / (2 r_s) = 3.5 is beyond the x <= 3 table of Eq. (int)
    with pytest.raises(B.PmfmmError):
        B.Context(box=100.0, r_s=1.0, r_cut=7.0, trunc=B.TRUNC_TABLE)
    B.Context(box=100.0, r_s=1.0, r_cut=7.0, trunc=B.TRUNC_EXACT).close()


def test_fp64_table_size_limit():
    with pytest.raises(B.PmfmmError):
        B.Context(precision=B.PMFMM_FP64, trunc=B.TRUNC_TABLE, table_size=4096)
    B.Context(precision=B.PMFMM_FP32, trunc=B.TRUNC_TABLE, table_size=4096).close()


def test_r2_table_is_a_float32_form():
    for bad in (dict(precision=B.PMFMM_FP64, trunc=B.TRUNC_R2, table_size=64,
                     table_level=2),
                dict(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=64,
                     table_level=0),
                dict(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=64,
                     table_level=3),
                dict(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=48,
                     table_level=2),
                dict(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=32,
                     table_level=1),
                dict(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=256,
                     table_level=2),
                dict(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=1024,
                     table_level=1)):
        with pytest.raises(B.PmfmmError):
            B.Context(**bad)
    for size, level in ((16, 2), (64, 2), (128, 1), (256, 1), (512, 1)):
        B.Context(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=size,
                  table_level=level).close()


def test_r2_table_needs_one_cutoff_ratio():
    ctx = B.Context(precision=B.PMFMM_FP32, trunc=B.TRUNC_R2, table_size=64,
                    table_level=2)
    a = B.make_params(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=8)
    b = B.make_params(box=12.0, r_s=0.6, r_cut=2.7, max_leaf=8)     # same x_c
    c = B.make_params(box=12.0, r_s=0.6, r_cut=3.0, max_leaf=8)
    pos = np.random.default_rng(0).uniform(0, 10, (30, 3))
    with pytest.raises(B.PmfmmError, match="r_cut / r_s"):
        ctx.plan_batch([a, c], [10, 20], pos, np.ones(30))
    ctx.plan_batch([a, b], [10, 20], pos, np.ones(30))


def test_plan_rejects_bad_particles():
    ctx = B.Context(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=8)
    pos = np.random.default_rng(0).uniform(0, 10, (50, 3))
    m = np.ones(50)
    bad = pos.copy()
    bad[7, 1] = np.nan
    with pytest.raises(B.PmfmmError, match="non-finite"):
        ctx.plan(bad, m)
    mm = m.copy()
    mm[3] = -1.0
    with pytest.raises(B.PmfmmError, match="mass"):
        ctx.plan(pos, mm)
    with pytest.raises(B.PmfmmError):
        ctx.plan(pos[:0], m[:0])
    ctx.plan(pos, m)
    assert ctx.lists()["n"] == 50


def test_calls_out_of_order():
    lib = B.library()
    ctx = B.Context()
    lists = B.Lists()
    assert lib.pmfmm_get_lists(ctx._h, lists) == -4
    assert lib.pmfmm_forward(ctx._h, B.C.c_void_p(8), None) == -4
    assert lib.pmfmm_forward_static(ctx._h, B.C.c_void_p(8), None) == -4
    best = B.Schedule()
    assert lib.pmfmm_autotune(ctx._h, B.C.c_void_p(8), None, 0, 3, None, None,
                              B.C.byref(best), None) == -4
    assert lib.pmfmm_autotune(ctx._h, None, None, 0, 3, None, None,
                              B.C.byref(best), None) == -1
    assert lib.pmfmm_forward_static(ctx._h, None, None) == -1
    assert lib.pmfmm_adjoint(ctx._h, B.C.c_void_p(8), B.C.c_void_p(8),
                             B.C.c_void_p(8), None) == -4
    t = B.Timings()
    assert lib.pmfmm_get_timings(ctx._h, t) == -4
    assert "nothing timed" in lib.pmfmm_last_error().decode()
    assert lib.pmfmm_forward(None, None, None) == -1
    lib.pmfmm_destroy(None)


def test_wrap_into_box():
    ctx = B.Context(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=4)
    pos = np.array([[-0.5, 10.0, 3.0], [25.0, -13.0, 9.999], [1.0, 2.0, 3.0]])
    ctx.plan(pos, np.ones(3))
    L = ctx.lists()
    assert np.all(L["cell_lo"] >= 0) and np.all(L["cell_hi"] < 10.0)
    assert math.isclose(L["cell_lo"][0, 0], 1.0)    # -0.5 -> 9.5, 25 -> 5, 1
    assert math.isclose(L["cell_hi"][0, 0], 9.5)


def test_set_eval_validates():
    ctx = B.Context()
    with pytest.raises(B.PmfmmError):
        ctx.set_eval(table_level=9)
    ctx.set_eval(table_level=2, precision=B.PMFMM_FP32, trunc=B.TRUNC_TABLE,
                 table_size=512)


def test_batch_plan_names_bad_box():
    ctx = B.Context()
    good = B.make_params(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=8)
    bad = B.make_params(box=10.0, r_s=0.5, r_cut=6.0, max_leaf=8)
    pos = np.random.default_rng(0).uniform(0, 10, (30, 3))
    with pytest.raises(B.PmfmmError, match="box 1"):
        ctx.plan_batch([good, bad], [10, 20], pos, np.ones(30))
    ctx.plan_batch([good, good], [10, 20], pos, np.ones(30))
    L = ctx.lists()
    assert L["n_boxes"] == 2 and L["n"] == 30


def test_set_eval_keeps_params_after_a_rejected_call():
    ctx = B.Context(precision=B.PMFMM_FP32, trunc=B.TRUNC_TABLE, table_size=512,
                    table_level=2)
    with pytest.raises(B.PmfmmError):
        ctx.set_eval(table_level=9, chunk=7)
    assert ctx.params.table_level == 2 and ctx.params.chunk == 0
    ctx.set_eval(chunk=8)
    assert ctx.params.chunk == 8 and ctx.params.table_level == 2


def test_binding_rejects_bad_host_arrays_before_the_call():
    ctx = B.Context(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=8)
    pos = np.random.default_rng(0).uniform(0, 10, (50, 3))
    m = np.ones(50)
    with pytest.raises(ValueError, match="shape"):
        ctx.plan(pos[:, :2], m)
    with pytest.raises(ValueError, match="shape"):
        ctx.plan(pos, m[:49])
    with pytest.raises(ValueError, match="shape"):
        ctx.build(pos.reshape(-1), m)
    with pytest.raises(ValueError, match="both"):
        ctx.build(pos, object())
    with pytest.raises(ValueError, match="one count per box"):
        ctx.plan_batch([ctx.params], [25, 25], pos, m)
    with pytest.raises(ValueError, match="shape"):
        ctx.plan_batch([ctx.params, ctx.params], [25, 24], pos, m)


def test_binding_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    ctx = B.Context(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=8)
    pos = torch.zeros((50, 3), dtype=torch.float64)
    m = torch.ones(50, dtype=torch.float64)
    with pytest.raises(ValueError, match="CUDA"):
        ctx.build(pos, m)
    with pytest.raises(ValueError, match="CUDA"):
        B.kick(pos, pos, 0.1)
    ctx.plan(pos.numpy(), m.numpy())
    with pytest.raises(ValueError, match="CUDA"):
        ctx.forward(pos)
    with pytest.raises(ValueError, match="CUDA"):
        ctx.adjoint(pos, pos, m)
    with pytest.raises(ValueError, match="CUDA"):
        ctx.long_range(16, pos, m, pos)
    fresh = B.Context(box=10.0, r_s=0.5, r_cut=2.25, max_leaf=8)
    with pytest.raises(B.PmfmmError, match="before build"):
        fresh.forward(pos)


def test_accum_twosum_is_for_float32_forms():
    with pytest.raises(B.PmfmmError) as e:
        B.Context(precision=B.PMFMM_FP64, accum=B.ACCUM_FP32_TWOSUM)
    assert e.value.code == -1
    ctx = B.Context(precision=B.PMFMM_FP32, accum=B.ACCUM_FP32_TWOSUM)
    assert ctx.params.accum == B.ACCUM_FP32_TWOSUM
    with pytest.raises(B.PmfmmError):
        ctx.set_eval(precision=B.PMFMM_FP64)      # still TwoSum: refused, params kept
    assert ctx.params.precision == B.PMFMM_FP32

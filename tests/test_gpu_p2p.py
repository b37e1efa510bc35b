"""GPU parity of the P2P path against the CPU oracle (through the C ABI).

Tolerances (relative force error e_i = |a_i - a_ref| / |a_ref|):
  * float64, exact T:          max e_i <= 1e-12
  * float64, 2048-node T_[4]:  max e_i <= 1e-12 against the oracle's table
                               sum, and <= 1e-11 against the exact sum
  * float64, r^2 table:        99.9th percentile <= 1e-13 .. 1e-9 by degree
                               and segments (the table's error), max <= 100x
  * float32 (any T form):      median <= 1e-5, 99.9th percentile <= 1e-4
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import direct, metrics
from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs

pytestmark = pytest.mark.gpu


def gpu_forward(pos, mass, box, r_s, r_cut, max_leaf, order=-1, theta=0.0,
                **ev):
    ctx = B.Context(box=box, r_s=r_s, r_cut=r_cut, max_leaf=max_leaf,
                    order=order, theta=theta, **ev)
    p = torch.tensor(pos, dtype=torch.float64, device="cuda")
    m = torch.tensor(mass, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    ctx.build(p, m, s)
    out = torch.full((len(mass), 3), float("nan"), dtype=torch.float64,
                     device="cuda")
    ctx.forward(out, s)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ctx


def check_fp32(acc, ref):
    s = metrics.error_summary(acc, ref)
    assert s["median"] <= 1e-5, s
    assert s["p999"] <= 1e-4, s
    return s


@pytest.fixture(scope="module")
def c1():
    w = inputs.uniform_32k()
    ref, cnt = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut)
    return w, ref


@pytest.fixture(scope="module")
def clustered():
    w = inputs.clustered_small(24, 77, halo_frac=0.3, n_halos=6)
    ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut)
    return w, ref


def test_fp64_exact_uniform_32k(c1):
    w, ref = c1
    print("case: uniform 32^3, fp64 exact, leaf 32", flush=True)
    acc, ctx = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, w.max_leaf)
    s = metrics.error_summary(acc, ref)
    assert s["max"] <= 1e-12, s


def test_fp64_exact_clustered(clustered):
    w, ref = clustered
    print("case: clustered 24^3, fp64 exact, leaf 64", flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64)
    assert metrics.error_summary(acc, ref)["max"] <= 1e-12


@pytest.mark.parametrize("chunk", [1, 3, 1000])
def test_fp64_exact_any_chunking(clustered, chunk):
    w, ref = clustered
    print(f"case: clustered 24^3, fp64 exact, chunk {chunk}", flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64,
                         chunk=chunk)
    assert metrics.error_summary(acc, ref)["max"] <= 1e-12


def test_fp64_table_level4(clustered):
    w, ref = clustered
    print("case: clustered 24^3, fp64 table 2048 T_[4]", flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64,
                         precision=B.PMFMM_FP64, trunc=B.TRUNC_TABLE,
                         table_size=2048, table_level=4)
    ref_tab, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                    table=(2048, 4, "nearest"))
    assert metrics.error_summary(acc, ref_tab)["max"] <= 1e-12
    assert metrics.error_summary(acc, ref)["max"] <= 1e-11


# float64 r^2 table: degree 4..6 polynomials of T(r) / r^3 over 16..64
# segments per octave of r^2; pairs closer than 2^-8 r_cut exactly.  Against
# the exact sum with the error measured on the sum of pair-term magnitudes
# (the table's own error, ~1e-15 per pair at degree 6 and 64 segments per
# octave, is stated separately; a particle whose net force nearly cancels
# only resolves it to that error times the terms).
@pytest.mark.parametrize("degree,per_octave,tol", [(6, 64, 1e-13), (5, 64, 1e-12),
                                                   (6, 32, 1e-12), (4, 32, 1e-9)])
def test_fp64_r2_table(clustered, degree, per_octave, tol):
    w, ref = clustered
    print(f"case: clustered 24^3, fp64 r^2 table {per_octave}/octave degree {degree}",
          flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64,
                         precision=B.PMFMM_FP64, trunc=B.TRUNC_R2,
                         table_size=per_octave, table_level=degree)
    e = metrics.error_summary(acc, ref)
    print("   relative errors", e, flush=True)
    assert e["max"] <= 100 * tol, e
    assert e["p999"] <= tol, e


def test_fp64_r2_close_pairs_take_the_exact_path():
    """Pairs at 1e-4 .. 1e-2 r_cut (below the table's range) and coincident
    pairs, in float64 with the r^2 table, against the exact sum."""
    rng = np.random.default_rng(17)
    box = 20.0
    r_s, r_cut = 0.6, 2.7
    base = rng.uniform(0, box, (800, 3))
    close = base[:200] + rng.normal(0, 1, (200, 3)) * rng.uniform(1e-4, 1e-2, (200, 1)) * r_cut
    pos = inputs.wrap(np.concatenate([base, close, base[:5]]), box)
    m = rng.uniform(0.5, 1.5, len(pos))
    ref, _ = direct.brute_force(pos, m, box, r_s, r_cut)
    acc, _ = gpu_forward(pos, m, box, r_s, r_cut, 16, precision=B.PMFMM_FP64,
                         trunc=B.TRUNC_R2, table_size=64, table_level=6)
    e = metrics.error_summary(acc, ref)
    assert e["max"] <= 1e-11, e


@pytest.mark.parametrize("level,n_tab,rnd", [(2, 512, B.ROUND_NEAREST),
                                             (1, 2048, B.ROUND_NEAREST),
                                             (3, 2048, B.ROUND_NEAREST),
                                             (2, 512, B.ROUND_FLOOR)])
def test_fp32_table(c1, level, n_tab, rnd):
    w, ref = c1
    print(f"case: uniform 32^3 fp32 table {n_tab} level {level}", flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, w.max_leaf,
                         precision=B.PMFMM_FP32, trunc=B.TRUNC_TABLE,
                         table_size=n_tab, table_level=level, table_round=rnd)
    check_fp32(acc, ref)


@pytest.mark.parametrize("level,per_octave", [(2, 64), (1, 128), (2, 16),
                                              (2, 32), (1, 256), (1, 512)])
def test_fp32_r2_table(c1, level, per_octave):
    w, ref = c1
    print(f"case: uniform 32^3 fp32 r^2 table {per_octave}/octave degree "
          f"{level}", flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, w.max_leaf,
                         precision=B.PMFMM_FP32, trunc=B.TRUNC_R2,
                         table_size=per_octave, table_level=level)
    check_fp32(acc, ref)


def test_fp32_r2_table_clustered_and_coincident(clustered):
    w, ref = clustered
    print("case: clustered 24^3 fp32 r^2 table 64/octave degree 2",
          flush=True)
    acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64,
                         precision=B.PMFMM_FP32, trunc=B.TRUNC_R2,
                         table_size=64, table_level=2)
    check_fp32(acc, ref)
    rng = np.random.default_rng(19)
    pos = rng.uniform(0, 20.0, (2001, 3))
    pos[50:90] = pos[0]                         # coincident particles
    m = rng.uniform(0.2, 1.0, 2001) * 1e9       # large masses stay finite
    print("case: ragged 2001 coincident, fp32 r^2 table", flush=True)
    acc, _ = gpu_forward(pos, m, 20.0, 0.6, 2.7, 16, precision=B.PMFMM_FP32,
                         trunc=B.TRUNC_R2, table_size=64, table_level=2)
    ref2, _ = direct.all_pairs(pos, m, 20.0, 0.6, 2.7)
    assert np.all(np.isfinite(acc))
    check_fp32(acc, ref2)


@pytest.mark.parametrize("equal_mass", [False, True])
def test_fp32_r2_linear_close_pairs(equal_mass):
    """The linear r^2 table stops at r = 2^-9.5 r_cut and adds closer pairs
    exactly: pairs at 1e-4 .. 1e-2 r_cut (half of them below the floor) and
    coincident pairs, against the quadratic table, which covers them down to
    2^-17.5 r_cut with the same float32 displacements (so the two agree to
    the tables' error even where float32 cannot resolve the displacement),
    and against the exact float64 sum at the float32 tolerances away from
    the close pairs.  Equal masses take the one-mass-per-leaf path."""
    rng = np.random.default_rng(23)
    box, r_s, r_cut = 20.0, 0.6, 2.7
    base = rng.uniform(0, box, (1500, 3))
    u = rng.normal(0, 1, (300, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = r_cut * 10.0 ** rng.uniform(-4, -2, (300, 1))
    pos = inputs.wrap(np.concatenate([base, base[:300] + u * r, base[300:305]]), box)
    m = np.ones(len(pos)) if equal_mass else rng.uniform(0.5, 1.5, len(pos))
    print(f"case: fp32 r^2 linear 512/octave close pairs, equal mass {equal_mass}",
          flush=True)
    lin, _ = gpu_forward(pos, m, box, r_s, r_cut, 16, precision=B.PMFMM_FP32,
                         trunc=B.TRUNC_R2, table_size=512, table_level=1)
    quad, _ = gpu_forward(pos, m, box, r_s, r_cut, 16, precision=B.PMFMM_FP32,
                          trunc=B.TRUNC_R2, table_size=64, table_level=2)
    assert np.all(np.isfinite(lin))
    e = metrics.error_summary(lin, quad)
    assert e["max"] <= 1e-4, e
    ref, _ = direct.brute_force(pos, m, box, r_s, r_cut)
    far = np.ones(len(pos), bool)
    far[:300] = False
    far[1500:] = False
    far[300:305] = False
    check_fp32(lin[far], ref[far])


def test_fp32_exact_and_table_clustered(clustered):
    w, ref = clustered
    for trunc in (B.TRUNC_EXACT, B.TRUNC_TABLE):
        print(f"case: clustered 24^3 fp32 trunc {trunc}", flush=True)
        acc, _ = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64,
                             precision=B.PMFMM_FP32, trunc=trunc,
                             table_size=2048, table_level=2)
        check_fp32(acc, ref)


def test_bitwise_reproducible(clustered):
    w, _ = clustered
    for prec in (B.PMFMM_FP64, B.PMFMM_FP32):
        a1, ctx = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64,
                              precision=prec)
        out = torch.empty((len(w.mass), 3), dtype=torch.float64, device="cuda")
        for _ in range(3):
            ctx.forward(out, torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), a1)


def test_reused_context_switching_modes(clustered):
    w, ref = clustered
    acc, ctx = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64)
    out = torch.empty((len(w.mass), 3), dtype=torch.float64, device="cuda")
    # the r^2 table works on rescaled float32 offsets: switching into and out
    # of it rescales them
    for prec, trunc in [(B.PMFMM_FP32, B.TRUNC_TABLE), (B.PMFMM_FP64,
                                                        B.TRUNC_EXACT),
                        (B.PMFMM_FP32, B.TRUNC_R2), (B.PMFMM_FP32,
                                                     B.TRUNC_EXACT),
                        (B.PMFMM_FP32, B.TRUNC_R2), (B.PMFMM_FP64,
                                                     B.TRUNC_EXACT),
                        (B.PMFMM_FP32, B.TRUNC_TABLE)]:
        ctx.set_eval(precision=prec, trunc=trunc,
                     table_size=64 if trunc == B.TRUNC_R2 else 1024,
                     table_level=2, chunk=7)
        ctx.forward(out, torch.cuda.current_stream())
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        if prec == B.PMFMM_FP64:
            assert metrics.error_summary(a, ref)["max"] <= 1e-12
        else:
            check_fp32(a, ref)


# ------------------------------------------------------------- edge cases

def test_single_particle_and_pair():
    box, r_s, r_cut = 10.0, 0.5, 2.25
    acc, _ = gpu_forward(np.array([[1.0, 2.0, 3.0]]), np.array([2.0]), box,
                         r_s, r_cut, 8)
    assert np.all(acc == 0.0)
    pos = np.array([[9.8, 5.0, 5.0], [0.3, 5.0, 5.0]])   # across the boundary
    m = np.array([1.5, 0.5])
    acc, _ = gpu_forward(pos, m, box, r_s, r_cut, 8, G=3.0)
    ref, _ = direct.all_pairs(pos, m, box, r_s, r_cut, G=3.0)
    assert metrics.error_summary(acc, ref)["max"] <= 1e-14
    assert acc[0, 0] > 0 and acc[1, 0] < 0


def test_coincident_and_ragged():
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, 20.0, (3001, 3))
    pos[100:140] = pos[0]                       # 41 coincident particles
    m = rng.uniform(0.2, 1.0, 3001)
    for ml in (1, 7, 64):
        print(f"case: ragged 3001 coincident, leaf {ml}", flush=True)
        acc, _ = gpu_forward(pos, m, 20.0, 0.6, 2.7, ml)
        ref, _ = direct.all_pairs(pos, m, 20.0, 0.6, 2.7)
        assert np.all(np.isfinite(acc))
        assert metrics.error_summary(acc, ref)["max"] <= 1e-12


def test_pairs_just_inside_the_cutoff_are_kept():
    """Sources are culled per j leaf against the box of a wave's targets;
    sources placed at r_cut (1 - eps) from a target (eps down to 1e-14, along
    the axes, face diagonals and body diagonals, so also beyond box corners
    and across the periodic boundary) must still be counted: float64 exact
    against the oracle at 1e-12, and the float64 r^2 table, whose cutoff
    test is the same float64 one.  (The float32 forms decide pairs this
    close to r_cut in float32 and may place them on either side.)"""
    rng = np.random.default_rng(21)
    box, r_s, r_cut = 40.0, 1.0, 4.5
    targets = rng.uniform(0, box, (1500, 3))
    dirs = np.array([[1, 0, 0], [0, -1, 0], [1, 1, 0], [1, -1, 1], [-1, -1, -1],
                     [0, 1, 1]], float)
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    pick = rng.choice(len(targets), 600, replace=False)
    eps = 10.0 ** rng.uniform(-14, -6, 600)
    src = targets[pick] + (r_cut * (1 - eps))[:, None] * dirs[rng.integers(0, 6, 600)]
    pos = np.mod(np.concatenate([targets, src]), box)
    m = rng.uniform(0.5, 1.5, len(pos))
    ref, _ = direct.brute_force(pos, m, box, r_s, r_cut)
    for ml in (16, 64):
        print(f"case: near-cutoff shell, leaf {ml}", flush=True)
        acc, _ = gpu_forward(pos, m, box, r_s, r_cut, ml)
        assert metrics.error_summary(acc, ref)["max"] <= 1e-12
        acc, _ = gpu_forward(pos, m, box, r_s, r_cut, ml, precision=B.PMFMM_FP64,
                             trunc=B.TRUNC_R2, table_size=64, table_level=6)
        e = metrics.error_summary(acc, ref)
        assert e["p999"] <= 1e-12 and e["max"] <= 1e-10, e


def test_unwrapped_device_input_is_wrapped():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 20.0, (500, 3))
    shifted = pos + rng.integers(-2, 3, (500, 3)) * 20.0
    m = np.ones(500)
    a0, _ = gpu_forward(pos, m, 20.0, 0.6, 2.7, 16)
    a1, _ = gpu_forward(shifted, m, 20.0, 0.6, 2.7, 16)
    ref, _ = direct.all_pairs(pos, m, 20.0, 0.6, 2.7)
    assert metrics.error_summary(a1, ref)["max"] <= 1e-12
    assert metrics.error_summary(a0, ref)["max"] <= 1e-12


def test_host_input_build():
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 20.0, (700, 3))
    m = np.ones(700)
    ctx = B.Context(box=20.0, r_s=0.6, r_cut=2.7, max_leaf=16, order=-1)
    ctx.build(pos, m)                        # host pointers
    out = torch.empty((700, 3), dtype=torch.float64, device="cuda")
    ctx.forward(out)
    torch.cuda.synchronize()
    ref, _ = direct.all_pairs(pos, m, 20.0, 0.6, 2.7)
    assert metrics.error_summary(out.cpu().numpy(), ref)["max"] <= 1e-12


# ------------------------------------------------------------- full size

@pytest.fixture(scope="module")
def c2():
    return inputs.clustered_2m()


def test_full_size_clustered_2m_sampled(c2):
    """128^3 clustered at full size: sampled particles against the oracle."""
    w = c2
    rng = np.random.default_rng(2024)
    sample = rng.choice(len(w.mass), 1500, replace=False)
    ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut,
                                targets=sample)
    print("case: clustered 128^3 fp64 exact (sampled)", flush=True)
    acc, ctx = gpu_forward(w.pos, w.mass, w.box, w.r_s, w.r_cut, 64)
    assert metrics.error_summary(acc[sample], ref)["max"] <= 1e-12
    print("case: clustered 128^3 fp64 r^2 table (sampled)", flush=True)
    ctx.set_eval(precision=B.PMFMM_FP64, trunc=B.TRUNC_R2, table_size=64, table_level=6)
    out64 = torch.empty((len(w.mass), 3), dtype=torch.float64, device="cuda")
    ctx.forward(out64, torch.cuda.current_stream())
    torch.cuda.synchronize()
    e64 = metrics.error_summary(out64.cpu().numpy()[sample], ref)
    assert e64["p999"] <= 1e-13 and e64["max"] <= 1e-11, e64
    out = torch.empty((len(w.mass), 3), dtype=torch.float64, device="cuda")
    for trunc, level, n_tab in [(B.TRUNC_TABLE, 2, 512),
                                (B.TRUNC_TABLE, 1, 2048),
                                (B.TRUNC_EXACT, 0, 2048),
                                (B.TRUNC_R2, 2, 64)]:
        print(f"case: clustered 128^3 fp32 trunc {trunc} {n_tab} {level}",
              flush=True)
        ctx.set_eval(precision=B.PMFMM_FP32, trunc=trunc, table_size=n_tab,
                     table_level=level)
        ctx.forward(out, torch.cuda.current_stream())
        torch.cuda.synchronize()
        check_fp32(out.cpu().numpy()[sample], ref)


@pytest.mark.parametrize("trunc,size,level", [(B.TRUNC_R2, 64, 2), (B.TRUNC_TABLE, 512, 2),
                                              (B.TRUNC_EXACT, 512, 2)])
def test_fp32_twosum_accumulation(trunc, size, level):
    """accum = FP32_TWOSUM: each work item's j-leaf sums added in float32
    with a TwoSum compensation term.  Against the oracle at the float32
    tolerances, and within float32 rounding of the float64-accumulated
    result (the same pair sums, added differently)."""
    w = inputs.clustered_small(24, 21, halo_frac=0.3, n_halos=6)
    ref, _ = direct.brute_force(w.pos, w.mass, w.box, w.r_s, w.r_cut)
    print(f"case: float32 TwoSum accumulation, trunc {trunc}", flush=True)
    res = {}
    for acc in (B.ACCUM_FP64, B.ACCUM_FP32_TWOSUM):
        ctx = B.Context(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=64, order=-1,
                        precision=B.PMFMM_FP32, trunc=trunc, table_size=size,
                        table_level=level, accum=acc)
        ctx.build(torch.tensor(w.pos, device="cuda"), torch.tensor(w.mass, device="cuda"))
        out = torch.empty((len(w.mass), 3), dtype=torch.float64, device="cuda")
        ctx.forward(out)
        torch.cuda.synchronize()
        res[acc] = out.cpu().numpy()
    s = metrics.error_summary(res[B.ACCUM_FP32_TWOSUM], ref)
    print("  vs oracle:", s, flush=True)
    assert s["median"] <= 1e-5 and s["p999"] <= 1e-4
    d = metrics.error_summary(res[B.ACCUM_FP32_TWOSUM], res[B.ACCUM_FP64])
    print("  vs float64 accumulation:", d, flush=True)
    assert d["max"] <= 1e-6

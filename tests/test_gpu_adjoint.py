"""GPU adjoint (gradient of sum_i w_i . a_i) against the oracle's gradient
and against central finite differences of the GPU forward.

The mass gradient -sum_l g (w_l . d) sums terms of random sign (w is
Gaussian), so for some particles it nearly cancels; its rounding error is
then set by the size of the terms, not of the sum.  Besides the plain
relative error (used where the sum is well conditioned), every gradient is
checked with the error measured against the oracle's sum of term magnitudes
S_k: e_k = |g_k - g_ref,k| / S_k, with the force tolerances (float64
<= 1e-12; float32 median <= 1e-5, 99.9th percentile <= 1e-4).
"""

import numpy as np
import pytest
from scipy.special import erfc

torch = pytest.importorskip("torch")

from oracle import direct, fmm, metrics
from paper_2107_14008_amd import api
from paper_2107_14008_amd import binding as B
from paper_2107_14008_amd import inputs

pytestmark = pytest.mark.gpu


def rel_vec(a, ref):
    return metrics.error_summary(a, ref)


@pytest.fixture(scope="module")
def case():
    w = inputs.clustered_small(20, 55, halo_frac=0.3, n_halos=4)
    m = w.mass * np.random.default_rng(1).uniform(0.5, 1.5, len(w.mass))
    wv = inputs.cotangent(len(m), seed=15013)
    gx, gm, sx, sm = direct.gradient(w.pos, m, wv, w.box, w.r_s, w.r_cut,
                                     with_scale=True)
    return w, m, wv, gx, gm, sx, sm


def scaled(a, ref, scale):
    a = np.asarray(a).reshape(len(scale), -1)
    ref = np.asarray(ref).reshape(len(scale), -1)
    e = np.linalg.norm(a - ref, axis=1) / scale
    return dict(median=float(np.quantile(e, 0.5, method="higher")),
                p999=float(np.quantile(e, 0.999, method="higher")),
                max=float(e.max()))


def gpu_adjoint(w, m, wv, **ev):
    sr = api.ShortRange(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=64,
                        order=-1, theta=0.0, **ev)
    sr.build(torch.tensor(w.pos, device="cuda"), torch.tensor(m, device="cuda"))
    gp, gmass = sr.adjoint(torch.tensor(wv, device="cuda"))
    torch.cuda.synchronize()
    return gp.cpu().numpy(), gmass.cpu().numpy(), sr


def test_adjoint_fp64_matches_oracle(case):
    w, m, wv, gx, gm, sx, sm = case
    print("case: adjoint fp64, clustered 20^3", flush=True)
    gp, gmass, _ = gpu_adjoint(w, m, wv, precision=B.PMFMM_FP64)
    assert scaled(gp, gx, sx)["max"] <= 1e-12
    assert scaled(gmass, gm, sm)["max"] <= 1e-12
    assert rel_vec(gp, gx)["max"] <= 1e-11


def test_adjoint_fp32_matches_oracle(case):
    w, m, wv, gx, gm, sx, sm = case
    print("case: adjoint fp32, clustered 20^3", flush=True)
    gp, gmass, _ = gpu_adjoint(w, m, wv, precision=B.PMFMM_FP32)
    errs = (scaled(gp, gx, sx), scaled(gmass, gm, sm), rel_vec(gp, gx))
    print("errors (pos scaled, mass scaled, pos relative):", errs, flush=True)
    for s in errs:
        assert s["median"] <= 1e-5 and s["p999"] <= 1e-4, s


def test_adjoint_fp32_after_r2_table_forward(case):
    """The r^2 table form rescales the float32 offsets and its adjoint reads
    g and h from tables of their own (32 segments per octave); the scale is
    taken back out of the gradient."""
    w, m, wv, gx, gm, sx, sm = case
    print("case: adjoint fp32 with the r^2 table form set, clustered 20^3",
          flush=True)
    gp, gmass, _ = gpu_adjoint(w, m, wv, precision=B.PMFMM_FP32,
                               trunc=B.TRUNC_R2, table_size=64,
                               table_level=2)
    errs = (scaled(gp, gx, sx), scaled(gmass, gm, sm), rel_vec(gp, gx))
    print("errors (pos scaled, mass scaled, pos relative):", errs, flush=True)
    for s in errs:
        assert s["median"] <= 1e-5 and s["p999"] <= 1e-4, s


def test_adjoint_r2_tables_reproducible_across_launch_shapes(case):
    """Each work item sums its own pairs in a fixed order and the partials
    are reduced in slot order, so the gradients are bitwise the same for
    any workgroup size and grid, and on a repeated call."""
    w, m, wv, gx, gm, sx, sm = case
    print("case: adjoint fp32 r^2 tables, launch shapes", flush=True)
    runs = []
    for wg, grid in ((4, 0), (8, 0), (16, 0), (8, 37)):
        gp, gmass, sr = gpu_adjoint(w, m, wv, precision=B.PMFMM_FP32,
                                    trunc=B.TRUNC_R2, table_size=64,
                                    table_level=2, wg_waves=wg, grid_wgs=grid)
        runs.append((gp, gmass))
        gp2, gm2 = sr.adjoint(torch.tensor(wv, device="cuda"))
        torch.cuda.synchronize()
        runs.append((gp2.cpu().numpy(), gm2.cpu().numpy()))
    for gp, gmass in runs[1:]:
        assert np.array_equal(gp, runs[0][0]) and np.array_equal(gmass, runs[0][1])


@pytest.mark.parametrize("trunc", [B.TRUNC_EXACT, B.TRUNC_R2])
def test_adjoint_fp32_coincident_close_and_ragged(trunc):
    """Coincident particles (left out of each other's sums), pairs at 3e-2 ..
    1e-1 r_cut and a ragged particle count, float32 exact and r^2 tables."""
    rng = np.random.default_rng(23)
    box, r_s, r_cut = 20.0, 0.6, 2.7
    # ~20 neighbours per particle on average: none is left without any
    base = rng.uniform(0, box, (2000, 3))
    close = base[:300] + rng.normal(0, 1, (300, 3)) * rng.uniform(3e-2, 1e-1, (300, 1)) * r_cut
    pos = inputs.wrap(np.concatenate([base, close, base[:5]]), box)
    m = rng.uniform(0.5, 1.5, len(pos))
    wv = inputs.cotangent(len(m), seed=29)
    gx, gm, sx, sm = direct.gradient(pos, m, wv, box, r_s, r_cut, with_scale=True)
    print(f"case: adjoint fp32 trunc {trunc}, 2305 with coincident pairs", flush=True)
    sr = api.ShortRange(box=box, r_s=r_s, r_cut=r_cut, max_leaf=16, order=-1,
                        theta=0.0, precision=B.PMFMM_FP32, trunc=trunc,
                        table_size=64, table_level=2)
    sr.build(torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda"))
    gp, gmass = sr.adjoint(torch.tensor(wv, device="cuda"))
    torch.cuda.synchronize()
    gp, gmass = gp.cpu().numpy(), gmass.cpu().numpy()
    assert np.all(np.isfinite(gp)) and np.all(np.isfinite(gmass))
    for e in (scaled(gp, gx, sx), scaled(gmass, gm, sm)):
        print("errors:", e, flush=True)
        assert e["median"] <= 1e-5 and e["p999"] <= 1e-4, e


def clumps_with_close_pairs(seed=31):
    """128 clumps of 16 particles (radius 1e-4 r_cut) at jittered lattice
    points of a box of 20; every other clump holds a pair at 1e-6 .. 2.5e-6
    r_cut.  With max_leaf 16 each ORB leaf is exactly one clump (checked by
    the caller), so float32 offsets from the leaf centre resolve the close
    pairs to about 1e-5."""
    rng = np.random.default_rng(seed)
    box, r_s, r_cut = 20.0, 0.6, 2.7
    g = np.stack(np.meshgrid(np.arange(8), np.arange(4), np.arange(4), indexing="ij"),
                 -1).reshape(-1, 3)
    cen = (g + 0.5) * np.array([box / 8, box / 4, box / 4]) + rng.uniform(-0.6, 0.6, (128, 3))
    pts, close = [], []
    for c in range(128):
        u = rng.normal(0, 1, (16, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        p = cen[c] + u * (1e-4 * r_cut * rng.uniform(0, 1, (16, 1)) ** (1 / 3))
        if c % 2 == 0:
            v = rng.normal(0, 1, 3)
            v /= np.linalg.norm(v)
            p[1] = p[0] + v * rng.uniform(1e-6, 2.5e-6) * r_cut
            close += [16 * c, 16 * c + 1]
        pts.append(p)
    return inputs.wrap(np.concatenate(pts), box), np.array(close), box, r_s, r_cut


@pytest.mark.parametrize("trunc", [B.TRUNC_EXACT, B.TRUNC_R2])
def test_adjoint_fp32_pairs_below_table_floor(trunc):
    """Pairs at 1e-6 .. 2.5e-6 r_cut, below the float32 adjoint tables'
    floor (2^-18.5 r_cut = 2.7e-6 r_cut): the r^2 form takes them through
    the exact expression.  The gradients of the close-pair particles
    (dominated by the close pair) match the float64 oracle to 1e-4 of their
    term sums, the others to the float32 tolerances."""
    pos, close, box, r_s, r_cut = clumps_with_close_pairs()
    m = np.random.default_rng(5).uniform(0.5, 1.5, len(pos))
    wv = inputs.cotangent(len(m), seed=37)
    gx, gm, sx, sm = direct.gradient(pos, m, wv, box, r_s, r_cut, with_scale=True)
    print(f"case: adjoint fp32 trunc {trunc}, pairs at 1e-6 .. 2.5e-6 r_cut", flush=True)
    sr = api.ShortRange(box=box, r_s=r_s, r_cut=r_cut, max_leaf=16, order=-1,
                        theta=0.0, precision=B.PMFMM_FP32, trunc=trunc,
                        table_size=64, table_level=2)
    sr.build(torch.tensor(pos, device="cuda"), torch.tensor(m, device="cuda"))
    L = sr.ctx.lists()
    for l in range(L["n_leaves"]):           # each leaf is one clump
        mem = L["perm"][L["leaf_first"][l]:L["leaf_first"][l] + L["leaf_count"][l]]
        assert len(mem) == 16 and len(set(mem // 16)) == 1
    gp, gmass = sr.adjoint(torch.tensor(wv, device="cuda"))
    torch.cuda.synchronize()
    gp, gmass = gp.cpu().numpy(), gmass.cpu().numpy()
    assert np.all(np.isfinite(gp)) and np.all(np.isfinite(gmass))
    for e in (scaled(gp, gx, sx), scaled(gmass, gm, sm)):
        print("  all particles:", e, flush=True)
        assert e["median"] <= 1e-5 and e["p999"] <= 1e-4, e
    e = scaled(gp[close], gx[close], sx[close])
    print("  close-pair particles, position gradient:", e, flush=True)
    assert e["max"] <= 1e-4, e
    # The mass gradient sums g (w_l . d): for the close pair, d . w_l can
    # cancel, and float32 offsets resolve d to ~1e-5 of |d| only, so its
    # error scale is g |w_l| |d| rather than |g (w_l . d)|.
    k, l = close[0::2], close[1::2]
    d = pos[l] - pos[k]
    r = np.linalg.norm(d, axis=1)
    x = r / (2 * r_s)
    g = (erfc(x) + 2 * x / np.sqrt(np.pi) * np.exp(-x * x)) / r ** 3
    fac = np.empty(len(close))
    fac[0::2] = g * np.linalg.norm(wv[l], axis=1) * r
    fac[1::2] = g * np.linalg.norm(wv[k], axis=1) * r
    em = np.abs(gmass[close] - gm[close]) / (sm[close] + fac)
    print(f"  close-pair particles, mass gradient: max {em.max():.3g}", flush=True)
    assert em.max() <= 1e-4, em.max()


def test_autograd_function(case):
    w, m, wv, gx, gm, sx, sm = case
    pos = torch.tensor(w.pos, device="cuda", requires_grad=True)
    mass = torch.tensor(m, device="cuda", requires_grad=True)
    params = dict(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=64, order=-1,
                  precision="fp64")
    acc = api.ShortRangeForce.apply(pos, mass, params)
    loss = (acc * torch.tensor(wv, device="cuda")).sum()
    loss.backward()
    assert scaled(pos.grad.cpu().numpy(), gx, sx)["max"] <= 1e-12
    assert scaled(mass.grad.cpu().numpy(), gm, sm)["max"] <= 1e-12


def test_adjoint_vs_finite_differences_of_gpu_forward():
    """Central differences (h = 1e-4 grid spacings) of the float64 GPU loss."""
    w = inputs.clustered_small(16, 61)
    m = w.mass.copy()
    wv = inputs.cotangent(len(m), seed=7)
    gp, gmass, sr = gpu_adjoint(w, m, wv, precision=B.PMFMM_FP64)
    dg = w.box / w.n_pm
    h = 1e-4 * dg
    wt = torch.tensor(wv, device="cuda")

    def loss(pos, mass):
        s = api.ShortRange(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=64,
                           order=-1).build(torch.tensor(pos, device="cuda"),
                                           torch.tensor(mass, device="cuda"))
        return float((s.forward() * wt).sum())
    rng = np.random.default_rng(3)
    checked = 0
    for k in rng.choice(len(m), 12, replace=False):
        d = direct.image_displacement(w.pos[k][None, :], w.pos, w.box)
        r = np.linalg.norm(d, axis=1)
        if np.any(np.abs(r - w.r_cut) < 2 * h):
            continue
        for a in range(3):
            pp, pm = w.pos.copy(), w.pos.copy()
            pp[k, a] += h
            pm[k, a] -= h
            fd = (loss(pp, m) - loss(pm, m)) / (2 * h)
            assert gp[k, a] == pytest.approx(fd, rel=1e-3,
                                             abs=1e-6 * np.abs(gp).max())
            checked += 1
        mp_, mm_ = m.copy(), m.copy()
        mp_[k] *= 1.001
        mm_[k] *= 0.999
        fd = (loss(w.pos, mp_) - loss(w.pos, mm_)) / (0.002 * m[k])
        assert gmass[k] == pytest.approx(fd, rel=1e-6,
                                         abs=1e-9 * np.abs(gmass).max())
    assert checked >= 15


@pytest.fixture(scope="module")
def far_case():
    w = inputs.clustered_small(16, 3, halo_frac=0.6, n_halos=2, max_leaf=16)
    m = w.mass * np.random.default_rng(2).uniform(0.5, 1.5, len(w.mass))
    wv = inputs.cotangent(len(m), seed=15014)
    gx, gm, fx, fm, tree, lists = fmm.fmm_gradient(
        w.pos, m, wv, w.box, w.r_s, w.r_cut, 16, 4, 0.6, return_parts=True)
    assert len(lists.m2l) > 0
    _, _, sx, sm = direct.gradient(w.pos, m, wv, w.box, w.r_s, w.r_cut,
                                   with_scale=True)
    return w, m, wv, gx, gm, fx, fm, sx, sm


def far_adjoint(w, m, wv, **ev):
    sr = api.ShortRange(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=16,
                        order=4, theta=0.6, **ev)
    sr.build(torch.tensor(w.pos, device="cuda"), torch.tensor(m, device="cuda"))
    assert sr.ctx.lists()["n_m2l"] > 0
    gp, gmass = sr.adjoint(torch.tensor(wv, device="cuda"))
    torch.cuda.synchronize()
    return gp.cpu().numpy(), gmass.cpu().numpy()


def test_adjoint_with_far_field_fp64_matches_oracle(far_case):
    """The FMM adjoint (far field transposed on sign-flipped coefficients on
    the GPU, plain transposes in the oracle) on the same lists.  Error scale:
    the pair-term magnitudes plus the largest far-field term."""
    w, m, wv, gx, gm, fx, fm, sx, sm = far_case
    print("case: adjoint fp64 with far field, clustered 16^3 theta 0.6", flush=True)
    gp, gmass = far_adjoint(w, m, wv, precision=B.PMFMM_FP64)
    ex = scaled(gp, gx, sx + np.abs(fx).max())
    em = scaled(gmass, gm, sm + np.abs(fm).max())
    assert ex["max"] <= 1e-12, ex
    assert em["max"] <= 1e-12, em
    # the far field is a real part of the gradient here
    assert np.abs(fx).max() > 1e-4 * np.abs(gx).max()


def test_adjoint_with_far_field_fp32(far_case):
    w, m, wv, gx, gm, fx, fm, sx, sm = far_case
    print("case: adjoint fp32 with far field, clustered 16^3 theta 0.6", flush=True)
    gp, gmass = far_adjoint(w, m, wv, precision=B.PMFMM_FP32,
                            trunc=B.TRUNC_EXACT)
    for a, ref, sc in ((gp, gx, sx), (gmass, gm, sm)):
        e = scaled(a, ref, sc)
        assert e["median"] <= 1e-5 and e["p999"] <= 1e-4, e


def test_adjoint_with_far_field_fp32_r2_table(far_case):
    w, m, wv, gx, gm, fx, fm, sx, sm = far_case
    print("case: adjoint fp32 r^2 tables with far field, clustered 16^3 theta 0.6",
          flush=True)
    gp, gmass = far_adjoint(w, m, wv, precision=B.PMFMM_FP32,
                            trunc=B.TRUNC_R2, table_size=64, table_level=2)
    for a, ref, sc in ((gp, gx, sx), (gmass, gm, sm)):
        e = scaled(a, ref, sc)
        print("errors:", e, flush=True)
        assert e["median"] <= 1e-5 and e["p999"] <= 1e-4, e


def test_autograd_with_far_field(far_case):
    w, m, wv, gx, gm, fx, fm, sx, sm = far_case
    pos = torch.tensor(w.pos, device="cuda", requires_grad=True)
    mass = torch.tensor(m, device="cuda", requires_grad=True)
    params = dict(box=w.box, r_s=w.r_s, r_cut=w.r_cut, max_leaf=16, order=4,
                  theta=0.6, precision=B.PMFMM_FP64)
    acc = api.ShortRangeForce.apply(pos, mass, params)
    (acc * torch.tensor(wv, device="cuda")).sum().backward()
    ex = scaled(pos.grad.cpu().numpy(), gx, sx + np.abs(fx).max())
    em = scaled(mass.grad.cpu().numpy(), gm, sm + np.abs(fm).max())
    assert ex["max"] <= 1e-12 and em["max"] <= 1e-12, (ex, em)

"""The float64 exact truncation factor's polynomials (csrc/truncation_poly.h,
written by csrc/gen_truncation_poly.py): the header is what the generator
writes, and the kernels' evaluation steps, taken in float64 with the
header's coefficients, give T(x) = erfc(x) + (2x / sqrt(pi)) exp(-x^2)
(Eq. (tr)) within a few ulp of 40-digit mpmath values on [0, 3]."""

import importlib.util
import math
import os
import re

import mpmath as mp
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2107_14008_amd", "csrc")


def header_constants():
    text = open(os.path.join(CSRC, "truncation_poly.h")).read()
    scal = {m.group(1): float.fromhex(m.group(2)) if "0x" in m.group(2) else float(m.group(2))
            for m in re.finditer(r"constexpr (?:double|int) (\w+) = ([^;]+);", text)}
    arrs = {}
    for m in re.finditer(r"constexpr double (\w+)\[\d+\] = \{([^}]*)\};", text, re.S):
        arrs[m.group(1)] = [float.fromhex(v.strip()) for v in m.group(2).split(",") if v.strip()]
    return scal, arrs


def kernel_T(x, scal, arrs):
    """The steps of truncation_T_f64 for x <= 3, in float64 (math.fma where
    the kernel fuses)."""
    fma = getattr(math, "fma", None)
    if fma is None:                      # Python < 3.13: exact product, one rounding
        def fma(a, b, c):
            return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))
    s = x * x
    ds = fma(x, x, -s)
    n = float(np.rint(s * scal["kInvLn2"]))
    r = fma(n, scal["kLn2Hi"], -s)
    r = fma(n, scal["kLn2Lo"], r) - ds
    ep = arrs["kExpPoly"]
    p = ep[-1]
    for c in ep[-2::-1]:
        p = fma(p, r, c)
    e = math.ldexp(p, -int(n))
    tp = arrs["kTPoly"]
    deg = len(tp) - 1
    t = fma(x, scal["kTPolyInvHalfWidth"], -1.0)
    t2 = t * t
    ke = deg - (deg & 1)
    ko = deg - 1 + (deg & 1)
    ev, od = tp[ke], tp[ko]
    for k in range(ke - 2, -1, -2):
        ev = fma(ev, t2, tp[k])
    for k in range(ko - 2, 0, -2):
        od = fma(od, t2, tp[k])
    return e * fma(od, t, ev)


def test_header_is_generated():
    spec = importlib.util.spec_from_file_location("gen", os.path.join(CSRC, "gen_truncation_poly.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    coef, c = gen.coefficients()
    ecoef = gen.exp_coefficients()
    hi, lo = gen.ln2_split()
    scal, arrs = header_constants()
    assert arrs["kTPoly"] == coef
    assert arrs["kExpPoly"] == ecoef
    assert (scal["kLn2Hi"], scal["kLn2Lo"]) == (hi, lo)
    assert scal["kTPolyCentre"] == c == 1.5
    # the high part of ln 2 leaves room for n ln2_hi to be exact (n <= 13)
    assert float.hex(hi).endswith("800p-1") or (int(float.hex(hi)[4:17], 16) & 0x7FF) == 0


def test_kernel_steps_match_truncation_factor():
    mp.mp.dps = 40
    scal, arrs = header_constants()
    rng = np.random.default_rng(3)
    xs = np.concatenate([np.linspace(0.0, 3.0, 1201), rng.uniform(0.0, 3.0, 800),
                         [1e-300, 1e-8, 2.25, 2.9999999999999996]])
    worst = 0.0
    for x in xs:
        x = float(x)
        ref = mp.erfc(x) + 2 * mp.mpf(x) / mp.sqrt(mp.pi) * mp.exp(-mp.mpf(x) ** 2)
        got = kernel_T(x, scal, arrs)
        worst = max(worst, float(abs((mp.mpf(got) - ref) / ref)))
    # a few ulp of float64 (2^-52 = 2.2e-16)
    assert worst <= 4 * 2.0 ** -52, worst
    print("max relative error", worst)


@pytest.mark.parametrize("x", [0.0, 0.5, 1.0, 2.25, 3.0])
def test_special_values(x):
    scal, arrs = header_constants()
    got = kernel_T(x, scal, arrs)
    ref = math.erfc(x) + 2 * x / math.sqrt(math.pi) * math.exp(-x * x)
    assert abs(got - ref) <= 8e-16 * ref

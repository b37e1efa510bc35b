"""Pins of the oracle's truncation factor, table and derivative tensors.

Every check here compares the oracle against a route it does not share:
high-precision quadrature or differentiation (mpmath / sympy), Newton's law,
a convergence order, or the paper's stated adequacy of the table levels.
"""

import math

import mpmath as mp
import numpy as np
import pytest
import sympy as sp

from oracle import truncation as tr

mp.mp.dps = 40


def T_integral(x):
    """(4 / sqrt(pi)) int_x^inf u^2 exp(-u^2) du by quadrature (Sec. 3.3)."""
    x = mp.mpf(x)
    return 4 / mp.sqrt(mp.pi) * mp.quad(lambda u: u * u * mp.exp(-u * u),
                                        [x, x + 4, mp.inf])


@pytest.mark.parametrize("x", [0.0, 0.05, 0.3, 0.9, 1.5, 2.25, 2.9])
def test_T_equals_integral_form(x):
    assert abs(float(tr.T_exact(x)) - float(T_integral(x))) <= \
        2e-15 * float(T_integral(x))


@pytest.mark.parametrize("r", [0.1, 1.0, 3.3, 7.0, 15.0])
def test_short_plus_long_is_newton(r):
    """-d/dr psi_s from T, plus -d/dr of the erf part by differentiation, = 1/r^2."""
    r_s = 3.75
    rr = mp.mpf(r)
    long_force = -mp.diff(lambda q: mp.erf(q / (2 * r_s)) / q, rr)
    short = float(tr.T_of_r(r, r_s)) / r ** 2
    total = short + float(long_force)
    assert total == pytest.approx(1.0 / r ** 2, rel=2e-14)


@pytest.mark.parametrize("r", [0.2, 2.0, 9.0])
def test_T_is_minus_derivative_of_truncated_potential(r):
    r_s = 3.75
    force = -mp.diff(lambda q: mp.erfc(q / (2 * r_s)) / q, mp.mpf(r))
    assert float(tr.T_of_r(r, r_s)) / r ** 2 == pytest.approx(float(force),
                                                             rel=2e-14)


def test_T_at_zero_and_series():
    assert float(tr.T_exact(0.0)) == 1.0
    x = 1e-2
    series = 1 - 4 * x ** 3 / (3 * math.sqrt(math.pi)) \
        + 4 * x ** 5 / (5 * math.sqrt(math.pi))
    assert float(tr.T_exact(x)) == pytest.approx(series, rel=1e-13)


def test_T_of_r_matches_T_of_x():
    r = np.linspace(0.01, 20.0, 257)
    r_s = 2.5
    assert np.allclose(tr.T_of_r(r, r_s), tr.T_exact(r / (2 * r_s)),
                       rtol=1e-14, atol=0)


# ------------------------------------------------------------- table

def T_mp(x):
    return mp.erfc(x) + 2 * x / mp.sqrt(mp.pi) * mp.exp(-x * x)


@pytest.mark.parametrize("i", [1, 37, 200, 384, 511])
def test_taylor_terms_are_derivatives(i):
    """Term k of Eq. (int) equals T^(k)(x_i) / k! eps^k (high precision)."""
    xi_all, T_all, E_all, h = tr.table_nodes(512)
    xi = xi_all[i]
    eps = 0.37 * h
    terms = tr.table_terms(xi, E_all[i], eps)
    xm = mp.mpf(xi)
    for k, t in enumerate(terms, start=1):
        ref = mp.diff(T_mp, xm, k) / mp.factorial(k) * mp.mpf(eps) ** k
        assert float(t) == pytest.approx(float(ref), rel=1e-12, abs=1e-300)
    assert float(T_all[i]) == pytest.approx(float(T_mp(xm)), rel=2e-15)


@pytest.mark.parametrize("level", [0, 1, 2, 3])
@pytest.mark.parametrize("rounding", ["nearest", "floor"])
def test_table_convergence_order(level, rounding):
    """Max error over (0, 2.25] falls as h^(level+1) (catches a wrong term)."""
    x = np.linspace(1e-3, 2.25, 20001)
    ref = tr.T_exact(x)
    errs = []
    sizes = [64, 128, 256] if level >= 3 else [256, 512, 1024]
    for n in sizes:
        errs.append(np.max(np.abs(tr.T_table(x, n, level, rounding) - ref)))
    for a, b in zip(errs, errs[1:]):
        ratio = a / b
        assert 0.6 * 2 ** (level + 1) < ratio < 1.5 * 2 ** (level + 1)


def test_table_exact_at_nodes():
    xi, T, E, h = tr.table_nodes(2048)
    for level in range(5):
        assert np.allclose(tr.T_table(xi[:1536], 2048, level), tr.T_exact(xi[:1536]),
                           rtol=2e-15, atol=0)


def test_paper_table_adequacy():
    """Sec. 3.3: with 512 nodes on [0, 3], T_[2] suits single and T_[4] double."""
    claims = {}
    with open(__file__.replace("test_oracle_truncation.py",
                               "golden/paper_table_claims.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split("=")
                claims[k.strip()] = float(v)
    n = int(claims["table_size"])
    assert claims["x_max"] == tr.X_TABLE_MAX
    x = np.linspace(1e-4, 2.25, 40001)
    ref = tr.T_exact(x)
    e_sp = np.max(np.abs(tr.T_table(x, n, int(claims["sp_level"])) - ref) / ref)
    e_dp = np.max(np.abs(tr.T_table(x, n, int(claims["dp_level"])) - ref) / ref)
    e_sp_low = np.max(np.abs(tr.T_table(x, n, int(claims["sp_level"]) - 1)
                             - ref) / ref)
    # level 2 sits at a few float32 ulps, level 1 well above them
    assert e_sp < 4 * np.finfo(np.float32).eps
    assert e_sp_low > 10 * np.finfo(np.float32).eps
    # level 4 reaches the 1e-12 range needed by float64 work
    assert e_dp < 1e-12


# ------------------------------------------------------------- f_(n) and D

def _radial_derivatives(nmax):
    r, rs = sp.symbols("r r_s", positive=True)
    psi = sp.erfc(r / (2 * rs)) / r
    out = [psi]
    for _ in range(nmax):
        out.append(sp.simplify(sp.diff(out[-1], r) / r))
    return r, rs, out


@pytest.fixture(scope="module")
def radial():
    return _radial_derivatives(5)


@pytest.mark.parametrize("n", range(6))
@pytest.mark.parametrize("r", [0.9, 2.5, 6.0, 11.0])
def test_prefactor_is_radial_derivative(radial, n, r):
    rsym, rssym, fs = radial
    r_s = 1.875
    ref = float(fs[n].subs({rsym: r, rssym: r_s}).evalf(30))
    assert float(tr.f_prefactor(n, r, r_s)) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("n", range(5))
def test_prefactor_inverse_square_limit(n):
    """r_s -> infinity gives the inverse-square prefactor (the potential
    itself deviates by O(x), its derivatives by O(x^3))."""
    r = 1.3
    big = 1e6
    assert float(tr.f_prefactor(n, r, big)) == pytest.approx(
        float(tr.f_inverse_square(n, r)), rel=1e-5)


@pytest.fixture(scope="module")
def cart():
    X, Y, Z, rs = sp.symbols("X Y Z r_s", real=True)
    rr = sp.sqrt(X * X + Y * Y + Z * Z)
    return X, Y, Z, rs, sp.erfc(rr / (2 * rs)) / rr


def test_derivative_tensor_against_symbolic(cart):
    X, Y, Z, rs, psi = cart
    R = np.array([0.7, -1.1, 0.45])
    r_s = 0.9
    D = tr.derivative_tensor(R, 4, r_s)
    subs = {X: R[0], Y: R[1], Z: R[2], rs: r_s}
    for k in [(0, 0, 0), (1, 0, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (0, 1, 1),
              (3, 0, 0), (2, 1, 0), (1, 1, 1), (0, 0, 3), (4, 0, 0), (3, 1, 0),
              (2, 2, 0), (2, 1, 1), (0, 1, 3), (1, 2, 1)]:
        expr = sp.diff(psi, X, k[0], Y, k[1], Z, k[2])
        ref = float(expr.subs(subs).evalf(30))
        assert D[k] == pytest.approx(ref, rel=1e-11, abs=1e-14), k


def test_truncated_tensor_is_not_traceless():
    """Laplacian of psi_s is exp(-x^2) / (2 sqrt(pi) r_s^3), not zero."""
    R = np.array([0.6, 0.2, -0.3])
    r_s = 0.5
    D = tr.derivative_tensor(R, 2, r_s)
    lap = D[(2, 0, 0)] + D[(0, 2, 0)] + D[(0, 0, 2)]
    x = np.linalg.norm(R) / (2 * r_s)
    assert lap == pytest.approx(math.exp(-x * x) / (2 * math.sqrt(math.pi)
                                                    * r_s ** 3), rel=1e-10)
    Dn = tr.derivative_tensor(R, 2, r_s,
                              prefactor=lambda j, r: tr.f_inverse_square(j, r))
    lapn = Dn[(2, 0, 0)] + Dn[(0, 2, 0)] + Dn[(0, 0, 2)]
    assert abs(lapn) < 1e-12 * abs(Dn[(2, 0, 0)])


def test_multi_index_count():
    for p in range(7):
        assert len(tr.multi_indices(p)) == (p + 1) * (p + 2) * (p + 3) // 6

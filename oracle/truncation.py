"""Truncation factor, its interpolation table and the M2L derivative tensors.

Test infrastructure (see the package docstring).  Float64 numpy/scipy.

Paper passages followed:
  * Sec. 2, Eq. (tr): short-range pair force F_s = -(r / r^3) T(r; r_s) with
    T = erfc(r / 2 r_s) + r / (r_s sqrt(pi)) exp(-r^2 / 4 r_s^2).  With
    x = r / (2 r_s) this is T(x) = erfc(x) + (2 x / sqrt(pi)) exp(-x^2).
  * Sec. 3.3: the integral form T(x) = (4 / sqrt(pi)) int_x^inf u^2 e^-u^2 du
    and the Taylor table of Eq. (int): nodes x_i on [0, 3], stored values
    E_i = -4 exp(-x_i^2) / sqrt(pi) and T_i = erfc(x_i) - x_i E_i / 2, and
    the five terms T_[0] .. T_[4] in eps = x - x_i.
  * Sec. 2, M2L prefactor equation: (-1)^n r_s^(2n+1) f_(n)(x) as a sum of an
    erfc term and n Gaussian terms; and the inverse-square special case
    f_inv_(n) = (-1)^n (2n-1)!! / r^(2n+1).
  * Sec. 2, M2L equation: D_n = grad^n psi for the truncated potential
    psi = erfc(r / 2 r_s) / r.

Readings (the paper does not fix these):
  * table spacing h = 3 / N_tab, nodes x_i = i h for i = 0 .. N_tab - 1;
    index either nearest, d = floor(x / h + 1/2), or floor, d = floor(x / h),
    clamped to [0, N_tab - 1];
  * the paper calls D_n "traceless"; that holds for 1/r only.  For the
    truncated psi the Laplacian is exp(-x^2) / (2 sqrt(pi) r_s^3), so D is
    built here as the full symmetric Cartesian tensor from the radial
    derivatives f_(k) = ((1/r) d/dr)^k psi.

Parity: pinned by tests/test_oracle_truncation.py (integral form by
quadrature, split identity against Newton's law, Taylor terms against
high-precision derivatives, table convergence order, f_(n) against
high-precision radial derivatives, D against multivariate high-precision
derivatives, inverse-square limit).
"""

from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import erfc

SQRT_PI = math.sqrt(math.pi)
X_TABLE_MAX = 3.0


# --------------------------------------------------------------------------
# T(x): Eq. (tr)
# --------------------------------------------------------------------------

def T_exact(x):
    """T(x) = erfc(x) + (2x / sqrt(pi)) exp(-x^2), x = r / (2 r_s)."""
    x = np.asarray(x, dtype=np.float64)
    return erfc(x) + (2.0 / SQRT_PI) * x * np.exp(-x * x)


def T_of_r(r, r_s):
    """Eq. (tr) written in r: erfc(r/2r_s) + r/(r_s sqrt(pi)) exp(-r^2/4r_s^2)."""
    r = np.asarray(r, dtype=np.float64)
    return erfc(r / (2.0 * r_s)) + r / (r_s * SQRT_PI) * np.exp(
        -r * r / (4.0 * r_s * r_s))


def dT_dx(x):
    """Derivative of the integral form: dT/dx = -(4 / sqrt(pi)) x^2 e^-x^2."""
    x = np.asarray(x, dtype=np.float64)
    return -(4.0 / SQRT_PI) * x * x * np.exp(-x * x)


def psi_short(r, r_s):
    """Truncated potential kernel psi_s(r) = erfc(r / 2 r_s) / r."""
    r = np.asarray(r, dtype=np.float64)
    return erfc(r / (2.0 * r_s)) / r


# --------------------------------------------------------------------------
# Interpolation table: Sec. 3.3, Eq. (int)
# --------------------------------------------------------------------------

def table_nodes(n_tab: int):
    """Nodes x_i = i h, h = 3 / n_tab, with E_i and T_i as stored by the paper."""
    h = X_TABLE_MAX / n_tab
    xi = np.arange(n_tab, dtype=np.float64) * h
    E = -4.0 * np.exp(-xi * xi) / SQRT_PI
    T = erfc(xi) - xi * E / 2.0
    return xi, T, E, h


def table_index(x, n_tab: int, rounding: str = "nearest"):
    """Table node index d and offset eps = x - x_d for each x."""
    x = np.asarray(x, dtype=np.float64)
    h = X_TABLE_MAX / n_tab
    if rounding == "nearest":
        d = np.floor(x / h + 0.5)
    elif rounding == "floor":
        d = np.floor(x / h)
    else:
        raise ValueError(rounding)
    d = np.clip(d, 0, n_tab - 1).astype(np.int64)
    eps = x - d * h
    return d, eps


def table_terms(xi, E, eps):
    """The five Taylor terms T_[1] .. T_[4] of Eq. (int) (T_[0] is T_i)."""
    x2 = xi * xi
    t1 = x2 * E * eps
    t2 = -xi * (x2 - 1.0) * E * eps ** 2
    t3 = ((2.0 / 3.0) * x2 * x2 - (5.0 / 3.0) * x2 + 1.0 / 3.0) * E * eps ** 3
    t4 = -xi * ((1.0 / 3.0) * x2 * x2 - 1.5 * x2 + 1.0) * E * eps ** 4
    return t1, t2, t3, t4


def T_table(x, n_tab: int, level: int, rounding: str = "nearest"):
    """Table-interpolated T at interpolation level 0..4 (Eq. (int))."""
    if not 0 <= level <= 4:
        raise ValueError("level must be 0..4")
    xi_all, T_all, E_all, _ = table_nodes(n_tab)
    d, eps = table_index(x, n_tab, rounding)
    xi, E = xi_all[d], E_all[d]
    out = T_all[d].copy()
    for k, term in enumerate(table_terms(xi, E, eps), start=1):
        if k <= level:
            out = out + term
    return out


# --------------------------------------------------------------------------
# M2L prefactors f_(n) and Cartesian derivative tensors: Sec. 2
# --------------------------------------------------------------------------

def double_factorial(k: int) -> int:
    """k!! with (-1)!! = 0!! = 1."""
    if k <= 0:
        return 1
    out = 1
    while k > 1:
        out *= k
        k -= 2
    return out


def f_prefactor(n: int, r, r_s):
    """f_(n)(r) for the truncated kernel, from the paper's closed form.

    (-1)^n r_s^(2n+1) f_(n)(x) = (2n-1)!! / 2^(2n+1) * erfc(x) / x^(2n+1)
        + sum_{q=1..n} 2^(-q-n) (2n-1)!! / (2n-2q+1)!! * e^(-x^2) / (sqrt(pi) x^(2q))
    with x = r / (2 r_s).  f_(n) = ((1/r) d/dr)^n psi_s.
    """
    r = np.asarray(r, dtype=np.float64)
    x = r / (2.0 * r_s)
    df = double_factorial(2 * n - 1)
    acc = df / 2.0 ** (2 * n + 1) * erfc(x) / x ** (2 * n + 1)
    g = np.exp(-x * x) / SQRT_PI
    for q in range(1, n + 1):
        c = 2.0 ** (-q - n) * df / double_factorial(2 * n - 2 * q + 1)
        acc = acc + c * g / x ** (2 * q)
    return (-1.0) ** n * acc / r_s ** (2 * n + 1)


def f_inverse_square(n: int, r):
    """Prefactor of the plain 1/r kernel: (-1)^n (2n-1)!! / r^(2n+1)."""
    r = np.asarray(r, dtype=np.float64)
    return (-1.0) ** n * double_factorial(2 * n - 1) / r ** (2 * n + 1)


def multi_indices(p: int):
    """All (a, b, c) with a + b + c <= p, ordered by total degree then lex."""
    out = []
    for deg in range(p + 1):
        for a in range(deg, -1, -1):
            for b in range(deg - a, -1, -1):
                out.append((a, b, deg - a - b))
    return out


def factorial_mi(k) -> float:
    return float(math.factorial(k[0]) * math.factorial(k[1])
                 * math.factorial(k[2]))


def derivative_tensor(R, p: int, r_s, prefactor=None):
    """D_k(R) = d^k psi(R) for every multi-index |k| <= p.

    Full Cartesian form for a radial kernel psi(r):
        d^k psi(R) = sum_{m : 2 m_a <= k_a} prod_a [k_a! / (2^m_a m_a! (k_a - 2 m_a)!)]
                     R_a^(k_a - 2 m_a) f_(|k| - |m|)(|R|),
    where f_(j) = ((1/r) d/dr)^j psi.  ``prefactor(j, r)`` defaults to the
    truncated kernel's f_(j); pass ``lambda j, r: f_inverse_square(j, r)``
    for the plain 1/r kernel.  R has shape (3,) or (K, 3); returns a dict
    multi-index -> value (scalar or (K,) array).
    """
    R = np.asarray(R, dtype=np.float64)
    single = R.ndim == 1
    R = np.atleast_2d(R)
    r = np.sqrt((R[:, 0] * R[:, 0] + R[:, 1] * R[:, 1]) + R[:, 2] * R[:, 2])
    if prefactor is None:
        f = [f_prefactor(j, r, r_s) for j in range(p + 1)]
    else:
        f = [prefactor(j, r) for j in range(p + 1)]
    out = {}
    for k in multi_indices(p):
        total = np.zeros(len(R))
        for m in itertools.product(*(range(ka // 2 + 1) for ka in k)):
            coef = 1.0
            mono = np.ones(len(R))
            for a in range(3):
                ka, ma = k[a], m[a]
                coef *= math.factorial(ka) / (2 ** ma * math.factorial(ma)
                                              * math.factorial(ka - 2 * ma))
                mono = mono * R[:, a] ** (ka - 2 * ma)
            total = total + coef * mono * f[sum(k) - sum(m)]
        out[k] = float(total[0]) if single else total
    return out

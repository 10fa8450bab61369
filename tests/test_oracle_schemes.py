"""Pins for the oracle's coefficient tables and Gauss-Legendre weights.

Each check compares the typed tables with a *different* fact from the paper or
from mathematics: the order conditions (Sec. 4.1 eqs. Order1/Order2 and the
sixth-order conditions of Appendix C), the closed-form relations of Sec. 4.2
and Appendix C, the printed CF4:2 quadrature form (Sec. 7, eq. UCF4Gauss), and
numpy's Gauss-Legendre rule.
"""
import math
import os
from math import sqrt

import numpy as np
import pytest

from oracle import schemes as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ALL = list(S.SCHEMES)


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


@pytest.mark.parametrize("name", ALL)
def test_order1_conditions(name):
    # Sec. 4.1, eq. Order1: sum_i f_{i,n} = delta_{n,1}
    f = S.scheme(name).f
    sums = f.sum(axis=0)
    assert abs(sums[0] - 1.0) < 1e-14
    assert np.all(np.abs(sums[1:]) < 1e-14)


@pytest.mark.parametrize("name", [n for n in ALL if S.scheme(n).order >= 4])
def test_order2_condition(name):
    # Sec. 4.1, eq. Order2: sum_{i<j} f_{i1} f_{j2} - f_{j1} f_{i2} = -1/3
    f = S.scheme(name).f
    s = f.shape[0]
    acc = 0.0
    for i in range(s):
        for j in range(i + 1, s):
            acc += f[i, 0] * f[j, 1] - f[j, 0] * f[i, 1]
    assert abs(acc + 1.0 / 3.0) < 1e-14


@pytest.mark.parametrize("name", ALL)
def test_time_symmetry_rule(name):
    # Sec. 4.1, eq. FSymm: f_{s-i+1,n} = (-1)^(n+1) f_{i,n}
    f = S.scheme(name).f
    s, nmax = f.shape
    for i in range(s):
        for n in range(1, nmax + 1):
            assert f[s - 1 - i, n - 1] == pytest.approx((-1) ** (n + 1) * f[i, n - 1], abs=1e-15)


def _appc_conditions(f):
    """The seven sixth-order conditions for s = 5 as printed in Appendix C,
    eq. app:6thOrderConds (rows 1, 2 and the central row 3)."""
    f11, f12, f13 = f[0, 0], f[0, 1], f[0, 2]
    f21, f22, f23 = f[1, 0], f[1, 1], f[1, 2]
    f31, f33 = f[2, 0], f[2, 2]
    r = {}
    r["A1"] = 2 * f11 + 2 * f21 + f31 - 1
    r["A3"] = 2 * f13 + 2 * f23 + f33
    r["A1A2"] = (-f11 * f12 - 2 * f21 * f12 - f21 * f22 - f31 * f12 - f31 * f22) + 1 / 6
    r["A2A3"] = (f12 * f13 + 2 * f12 * f23 + f12 * f33 + f22 * f23 + f22 * f33) + 1 / 30
    r["A1A1A3"] = (f11 * f21 * f13 / 3 - 2 * f11 * f21 * f23 / 3 - f11 * f21 * f33 / 3
                   + f11 * f31 * f13 / 6 - f11 * f31 * f23 / 3 - f11 * f31 * f33 / 6
                   - f11 ** 2 * f23 / 3 - f11 ** 2 * f33 / 6 + 2 * f21 * f31 * f13 / 3
                   + f21 * f31 * f23 / 6 - f21 * f31 * f33 / 6 + 2 * f21 ** 2 * f13 / 3
                   - f21 ** 2 * f33 / 6 + f31 ** 2 * f13 / 6 + f31 ** 2 * f23 / 6) - 1 / 60
    r["A2A1A2"] = (-f11 * f12 ** 2 / 3 - f21 * f12 * f22 - f21 * f12 ** 2 - f21 * f22 ** 2 / 3
                   - f31 * f12 * f22 - f31 * f12 ** 2 / 2 - f31 * f22 ** 2 / 2) + 1 / 60
    r["A1A1A1A2"] = (f11 * f21 * f31 * f12 / 3 + f11 * f21 * f31 * f22 / 2
                     + f11 * f21 ** 2 * f12 / 3 + f11 * f21 ** 2 * f22 / 3
                     + f11 * f31 ** 2 * f12 / 12 + f11 * f31 ** 2 * f22 / 6
                     + f11 ** 2 * f21 * f12 / 3 + f11 ** 2 * f21 * f22 / 6
                     + f11 ** 2 * f31 * f12 / 6 + f11 ** 2 * f31 * f22 / 6
                     + f11 ** 3 * f12 / 12 + f21 * f31 ** 2 * f22 / 12
                     + f21 ** 2 * f31 * f22 / 6 + f21 ** 3 * f22 / 12) - 1 / 360
    return r


@pytest.mark.parametrize("name", ["CF6:5", "CF6:5b", "CF6:5Imp", "CF6:5Opt"])
def test_appendix_c_sixth_order_conditions(name):
    res = _appc_conditions(S.scheme(name).f)
    for key, v in res.items():
        assert abs(v) < 1e-14, (name, key, v)


def test_appendix_c_conditions_detect_a_typo():
    # the conditions are sensitive enough to catch a changed 8th digit
    f = S.scheme("CF6:5").f.copy()
    f[0, 1] += 1e-8
    f[4, 1] -= 1e-8
    res = _appc_conditions(f)
    assert max(abs(v) for v in res.values()) > 1e-10


def _pxy():
    coeffs = [[float(c) for c in line.split()] for line in _read_rows("app_c_pxy.txt")]

    def p(x, y):
        return sum(sum(c * x ** k for k, c in enumerate(row)) * y ** j
                   for j, row in enumerate(coeffs))
    return p


@pytest.mark.parametrize("name", ["CF6:5", "CF6:5b", "CF6:5Imp", "CF6:5Opt"])
def test_appendix_c_polynomial_root(name):
    f = S.scheme(name).f
    p = _pxy()
    x, y = f[0, 0], f[1, 0]
    # scale: derivative wrt y, so the check is relative to how fast p changes
    dp = (p(x, y + 1e-6) - p(x, y - 1e-6)) / 2e-6
    assert abs(p(x, y) / dp) < 1e-13


def test_appendix_c_remaining_coefficients_reproduce_cf65():
    # Appendix C, eq. app:RemCoeff, evaluated at the CF6:5 (f11, f21)
    f = S.scheme("CF6:5").f
    f11, f21 = f[0, 0], f[1, 0]
    f22 = (1 + 5 * f11 * (f11 - 1)) / (30 * (f11 + f21 - 1) * (f11 + f21) * (2 * f11 + f21 - 1))
    f12 = (1 - 6 * f22 + 12 * f11 * f22 + 6 * f21 * f22) / (6 * (1 - f11))
    D = 30 * (f12 * (2 * f11 - 1) * (2 * f11 + f21 - 1)
              + f22 * (1 + 8 * f11 ** 2 + 2 * (f21 - 2) * f21 + (8 * f21 - 7) * f11))
    f13 = ((2 * f11 - 1) * (2 * f11 + f21 - 1) - 3 * f22) / D
    f23 = (f11 + 3 * f12 + 4 * f11 * f21 + 2 * (f21 - 1) * f21 + 6 * f22 - 1) / D
    assert f22 == pytest.approx(f[1, 1], rel=1e-13)
    assert f12 == pytest.approx(f[0, 1], rel=1e-13)
    assert f13 == pytest.approx(f[0, 2], rel=1e-12)
    assert f23 == pytest.approx(f[1, 2], rel=1e-12)


def test_cf65_quintic_root():
    c = [float(v) for v in _read_rows("cf65_quintic.txt")]
    roots = np.roots(c[::-1])
    real = [r.real for r in roots if abs(r.imag) < 1e-9]
    assert len(real) == 1
    assert real[0] == pytest.approx(S.scheme("CF6:5").f[1, 0], rel=1e-13)


def test_fourth_order_family_relations():
    # Sec. 4.2, eq. Coeff4th: f11 = (1 - f21)/2, f12 = 1/(3 (1 + f21))
    for name in ("CF4:3", "CF4:3Opt"):
        f = S.scheme(name).f
        f21 = f[1, 0]
        assert f[0, 0] == pytest.approx((1 - f21) / 2, rel=1e-15)
        assert f[0, 1] == pytest.approx(1 / (3 * (1 + f21)), rel=1e-15)
    # Sec. 5.2: the A_3 order condition 2 f13 + f23 = 0
    f = S.scheme("CF4:3Opt").f
    assert 2 * f[0, 2] + f[1, 2] == pytest.approx(0.0, abs=1e-16)


def test_cf64_closed_form_is_sixth_order_member():
    f = S.scheme("CF6:4").f
    assert f.shape == (4, 3)
    # first-half row sums: f11 + f21 = 1/2
    assert f[0, 0] + f[1, 0] == pytest.approx(0.5, abs=1e-15)


def test_scheme_shapes_and_quadrature_points():
    expect = {"CF2:1": (1, 1), "CF4:2": (2, 2), "CF4:3": (3, 2), "CF4:3Opt": (3, 3),
              "CF6:4": (4, 3), "CF6:5": (5, 3), "CF6:5b": (5, 3), "CF6:6": (6, 3),
              "CF6:5Imp": (5, 4), "CF6:5Opt": (5, 4), "CF6:6Opt": (6, 4),
              "CF8:11": (11, 4)}
    for name, (s, M) in expect.items():
        sc = S.scheme(name)
        assert (sc.s, sc.M) == (s, M), name


def test_legendre_explicit_forms_and_orthogonality():
    xs = np.linspace(0, 1, 13)
    for line in _read_rows("legendre_explicit.txt"):
        parts = [float(v) for v in line.split()]
        n, coef = int(parts[0]), parts[1:]
        ref = sum(c * xs ** k for k, c in enumerate(coef))
        assert np.allclose(S.legendre_shifted(n, xs), ref, atol=1e-13)
    # orthogonality on [0,1] with numpy's Gauss-Legendre rule (library routine)
    t, w = np.polynomial.legendre.leggauss(12)
    x = 0.5 * (t + 1)
    w = 0.5 * w
    for a in range(6):
        for b in range(6):
            val = np.sum(w * S.legendre_shifted(a, x) * S.legendre_shifted(b, x))
            assert val == pytest.approx((a == b) / (2 * a + 1), abs=1e-14)
    # parity P_n(1-x) = (-1)^n P_n(x)  (Sec. 3.1, eq. PSymm)
    for n in range(6):
        assert np.allclose(S.legendre_shifted(n, 1 - xs), (-1) ** n * S.legendre_shifted(n, xs))


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_gauss_legendre_matches_numpy(M):
    x, w = S.gauss_legendre(M)
    t, wn = np.polynomial.legendre.leggauss(M)
    assert np.allclose(x, 0.5 * (t + 1), atol=1e-15)
    assert np.allclose(w, 0.5 * wn, atol=1e-15)
    # exact for polynomials up to degree 2M-1
    for k in range(2 * M):
        assert np.sum(w * x ** k) == pytest.approx(1.0 / (k + 1), abs=1e-15)


def test_cf42_printed_gauss_form():
    x, g = S.gl_weights(S.scheme("CF4:2"))
    assert x[0] == pytest.approx(0.5 - sqrt(3) / 6)
    for line in _read_rows("cf42_gauss_form.txt"):
        i, m, a, b, d = (int(v) for v in line.split())
        assert g[i - 1, m - 1] == pytest.approx((a + b * sqrt(3)) / d, abs=1e-15)


@pytest.mark.parametrize("name", ALL)
def test_gl_weights_sum_to_first_coefficient(name):
    # sum_m w_m P_{n-1}(x_m) = delta_{n,1} exactly for n <= 2M, so
    # sum_m g[i,m] = f[i,1]
    sc = S.scheme(name)
    x, g = S.gl_weights(sc)
    assert np.allclose(g.sum(axis=1), sc.f[:, 0], atol=5e-16)


@pytest.mark.parametrize("name", ALL)
def test_gl_weights_reproduce_legendre_moments(name):
    # With A(t) = sum_l c_l P_{l-1}(t/dt) (degree < M), the quadrature of
    # Sec. 7 eq. AnGauss gives back A_n = dt c_n for n <= nmax, so
    # dt sum_m g[i,m] A(x_m dt) = dt sum_n f[i,n] c_n.
    sc = S.scheme(name)
    x, g = S.gl_weights(sc)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(sc.M)
    A = sum(c[l] * S.legendre_shifted(l, x) for l in range(sc.M))
    lhs = g @ A
    rhs = sc.f[:, :sc.M] @ c[:sc.nmax]
    assert np.allclose(lhs, rhs, atol=1e-14)

"""Pins for oracle.rational: the approximants of eq. 1 and the partial
fractions of Table 1 (Section 2), checked against facts that do not come
from the oracle's own arithmetic."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import rational

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
XS = np.array([0.01, 0.3, 2.0, 50.0])


def _frac(s):
    return Fraction(s) if "/" in s else Fraction(s)


def load_table1():
    out = {}
    for line in open(os.path.join(GOLDEN, "table1_partial_fractions.txt")):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        k = int(parts[0])
        ent = out.setdefault(k, {"b": None, "poles": []})
        if parts[1] == "b":
            ent["b"] = float(Fraction(parts[2]))
        else:
            ent["poles"].append((float(Fraction(parts[2])), float(Fraction(parts[3]))))
    return out


@pytest.mark.parametrize("k", range(1, 7))
def test_r_of_one_is_zero_and_antisymmetry(k):
    # Section 1: r(1) = 0 and r_n(z) = -r_n(1/z)
    assert abs(rational.r_eval(k, 1.0)) < 1e-15
    z = np.array([0.05, 0.5, 3.0, 40.0])
    np.testing.assert_allclose(rational.r_eval(k, z), -rational.r_eval(k, 1.0 / z), rtol=1e-13)


@pytest.mark.parametrize("k", range(1, 7))
def test_slope_one_at_one(k):
    # r_k matches log to first order at 1 (z r'(z) - 1 vanishes at z = 1), computed exactly
    pref, num, den = rational.EQ1[k]
    deg = len(num) - 1
    dnum1 = sum(Fraction(c) * (deg - i) for i, c in enumerate(num[:-1]))
    den1 = sum(Fraction(c) for c in den)
    assert pref * dnum1 / den1 == 1


@pytest.mark.parametrize("k", rational.ORDERS_ON_PATH)
def test_partial_fraction_reconstructs_eq1(k):
    np.testing.assert_allclose(rational.r_partial(k, XS), rational.r_eval(k, XS), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("k", rational.ORDERS_ON_PATH)
def test_partial_fraction_matches_table1(k):
    tab = load_table1()[k]
    b, a, c = rational.partial_fraction(k)
    assert b == pytest.approx(tab["b"], rel=1e-15)
    printed = sorted(tab["poles"], key=lambda p: p[1])
    assert len(printed) == len(a)
    for (C, A), aj, cj in zip(printed, a, c):
        assert aj == pytest.approx(A, rel=1e-14)
        assert -cj == pytest.approx(C, rel=1e-14)


@pytest.mark.parametrize("k", rational.ORDERS_ON_PATH)
def test_poles_closed_form(k):
    # The denominator of eq. 1 is sum_i C(2k,2i) z^i = ((1+sqrt z)^2k + (1-sqrt z)^2k)/2,
    # whose roots are z = -tan^2(pi (2m+1) / (4k)).
    _, a, _ = rational.partial_fraction(k)
    closed = np.sort([np.tan(np.pi * (2 * m + 1) / (4 * k)) ** 2 for m in range(k)])
    np.testing.assert_allclose(a, closed, rtol=1e-13)
    from math import comb
    assert rational.EQ1[k][2] == [comb(2 * k, 2 * i) for i in range(k, -1, -1)]


@pytest.mark.parametrize("k,total", [(1, -4), (3, -52), (5, -148)])
def test_residue_sum_from_asymptotics(k, total):
    # r(x) - b ~ (sum_j c_j) / x as x -> inf; from eq. 1 that sum is
    # pref * (n_{k-1} - n_k d_{k-1} / d_k).
    pref, num, den = rational.EQ1[k]
    exact = pref * (Fraction(num[1]) - Fraction(num[0]) * den[1] / den[0])
    assert exact == total
    _, _, c = rational.partial_fraction(k)
    assert np.sum(c) == pytest.approx(total, rel=1e-14)


@pytest.mark.parametrize("k", rational.ORDERS_ON_PATH)
def test_shift_pairing(k):
    # r(z) = -r(1/z) pairs each pole a with 1/a and c_{1/a} = c_a / a^2;
    # r(1) = 0 <=> sum c/(1+a) = -b.
    b, a, c = rational.partial_fraction(k)
    np.testing.assert_allclose(np.sort(a), np.sort(1.0 / a), rtol=1e-13)
    for aj, cj in zip(a, c):
        i = np.argmin(np.abs(a - 1.0 / aj))
        assert c[i] == pytest.approx(cj / aj ** 2, rel=1e-13)
    assert np.sum(c / (1.0 + a)) == pytest.approx(-b, rel=1e-14)


def test_fig1_error_values_exact_rational():
    # Figure 1 plots log z - r_k(z); at z = 2 the approximants are exact rationals.
    z = Fraction(2)
    exact = {}
    for k in (1, 3, 5):
        pref, num, den = rational.EQ1[k]
        nv = sum(Fraction(cf) * z ** (len(num) - 1 - i) for i, cf in enumerate(num))
        dv = sum(Fraction(cf) * z ** (len(den) - 1 - i) for i, cf in enumerate(den))
        exact[k] = pref * nv / dv
    assert exact[1] == Fraction(2, 3)
    assert exact[3] == Fraction(206, 297)
    for k in (1, 3, 5):
        assert rational.r_partial(k, 2.0) == pytest.approx(float(exact[k]), rel=1e-15)
    err = {k: np.log(2.0) - float(exact[k]) for k in (1, 3, 5)}
    assert err[1] == pytest.approx(0.026480514, rel=1e-6)
    assert err[3] == pytest.approx(-4.5543e-4, rel=1e-3)
    assert abs(err[5]) < abs(err[3]) < abs(err[1])

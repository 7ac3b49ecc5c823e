"""Rational approximations r_k to log (Section 1, eq. 1) and their partial
fraction form (Section 2, Table 1; Algorithm 1 inputs).

Oracle module (test infrastructure).  Parity pins: see tests/test_oracle_rational.py.

r_k(z) = pref_k * N_k(z) / D_k(z) with the integer coefficients printed in
eq. 1.  The partial-fraction form used by Algorithm 1 is

    r_k(x) = b + sum_j c_j / (x - alpha_j),

whose poles alpha_j are the roots of D_k (all real and negative, Section 2).
This module writes the shift a_j = -alpha_j > 0, so each term reads
c_j / (x + a_j) with c_j < 0, the sign convention of Table 1.

The poles are found from the printed polynomials (numpy companion-matrix
roots, then Newton refinement in 50-digit decimal arithmetic), and the
residues are c_j = pref * N(alpha_j) / D'(alpha_j); b is the ratio of the
leading coefficients.  Nothing here uses the closed form of the poles; the
tests check the closed form separately.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

# eq. 1: prefactor, numerator and denominator coefficients, highest power first.
EQ1 = {
    1: (Fraction(2), [1, -1], [1, 1]),
    2: (Fraction(4), [1, 0, -1], [1, 6, 1]),
    3: (Fraction(2, 3), [7, 27, -27, -7], [1, 15, 15, 1]),
    4: (Fraction(16, 3), [1, 10, 0, -10, -1], [1, 28, 70, 28, 1]),
    5: (Fraction(2, 15), [43, 825, 1150, -1150, -825, -43], [1, 45, 210, 210, 45, 1]),
    6: (Fraction(4, 15), [23, 708, 2355, 0, -2355, -708, -23], [1, 66, 495, 924, 495, 66, 1]),
}

ORDERS_ON_PATH = (1, 3, 5)  # the odd orders the paper keeps (Section 1)


def r_eval(k: int, z):
    """r_k(z) evaluated directly from the eq. 1 polynomials (FP64)."""
    pref, num, den = EQ1[k]
    z = np.asarray(z, dtype=np.float64)
    return float(pref) * np.polyval(num, z) / np.polyval(den, z)


def _poly_dec(coeffs, x: Decimal) -> Decimal:
    acc = Decimal(0)
    for c in coeffs:
        acc = acc * x + Decimal(c)
    return acc


def _deriv(coeffs):
    deg = len(coeffs) - 1
    return [c * (deg - i) for i, c in enumerate(coeffs[:-1])]


def partial_fraction_decimal(k: int, digits: int = 50):
    """(b, a_j, c_j) for r_k as Decimals, a_j ascending.

    r_k(x) = b + sum_j c_j / (x + a_j)."""
    getcontext().prec = digits
    pref, num, den = EQ1[k]
    dden = _deriv(den)
    approx = np.roots(np.array(den, dtype=np.float64))
    poles = []
    for z0 in approx:
        x = Decimal(float(np.real(z0)))
        for _ in range(100):
            step = _poly_dec(den, x) / _poly_dec(dden, x)
            x -= step
            if step == 0 or abs(step) <= abs(x) * Decimal(10) ** (-(digits - 5)):
                break
        poles.append(x)
    poles.sort(reverse=True)  # alpha closest to 0 first -> a_j ascending
    pref_d = Decimal(pref.numerator) / Decimal(pref.denominator)
    b = pref_d * Decimal(num[0]) / Decimal(den[0])
    a = [-p for p in poles]
    c = [pref_d * _poly_dec(num, p) / _poly_dec(dden, p) for p in poles]
    return b, a, c


def partial_fraction(k: int):
    """(b, a, c) as float64: b scalar, a and c arrays of length deg D_k."""
    b, a, c = partial_fraction_decimal(k)
    return float(b), np.array([float(v) for v in a]), np.array([float(v) for v in c])


def r_partial(k: int, x):
    """r_k evaluated from the partial-fraction form."""
    b, a, c = partial_fraction(k)
    x = np.asarray(x, dtype=np.float64)
    out = np.full_like(x, b)
    for aj, cj in zip(a, c):
        out = out + cj / (x + aj)
    return out

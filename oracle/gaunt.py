"""Wigner 3j symbols and Gaunt integrals, exact up to the final rounding.

The 3j symbol uses Racah's closed formula with Python integers and fractions,
so the only rounding is the final conversion to FP64.  The Gaunt integral is
the integral over the unit sphere of three spherical harmonics in the
convention of `oracle.special` (no Condon-Shortley phase, Y^{-m} = conj Y^m).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache


@lru_cache(maxsize=None)
def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    if m1 + m2 + m3 != 0:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    f = math.factorial
    delta = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3),
                     f(j1 + j2 + j3 + 1))
    pref = (f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2)
            * f(j3 + m3) * f(j3 - m3))
    tmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    tmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for t in range(tmin, tmax + 1):
        den = (f(t) * f(j3 - j2 + t + m1) * f(j3 - j1 + t - m2)
               * f(j1 + j2 - j3 - t) * f(j1 - t - m1) * f(j2 - t + m2))
        s += Fraction((-1) ** t, den)
    sq = delta * pref                      # exact rational under the root
    sign = -1 if (j1 - j2 - m3) % 2 else 1
    # sqrt(sq) * s; do it as sqrt(sq * s^2) with the sign of s to keep one rounding
    val2 = sq * s * s
    mag = math.sqrt(val2.numerator) / math.sqrt(val2.denominator)
    return sign * (1 if s >= 0 else -1) * mag


def _eps(m: int) -> int:
    """Y_n^m (this convention) = eps(m) * Y_n^m (Condon-Shortley)."""
    return -1 if (m > 0 and m % 2 == 1) else 1


@lru_cache(maxsize=None)
def gaunt(n: int, m: int, n2: int, m2: int, l: int) -> float:
    """G(n,m; n2,m2; l) = integral of Y_n^m conj(Y_n2^m2) conj(Y_l^{m-m2}) dOmega."""
    mu = m - m2
    if abs(mu) > l or abs(m) > n or abs(m2) > n2:
        return 0.0
    if (n + n2 + l) % 2:
        return 0.0
    # conj(Y_a^b) = Y_a^{-b} in this convention, then convert to Condon-Shortley
    e = _eps(m) * _eps(-m2) * _eps(-mu)
    pre = math.sqrt((2 * n + 1) * (2 * n2 + 1) * (2 * l + 1) / (4.0 * math.pi))
    return e * pre * wigner3j(n, n2, l, 0, 0, 0) * wigner3j(n, n2, l, m, -m2, -mu)

"""Wigner 3j symbols by the Racah formula in exact rational arithmetic.

Test infrastructure (part of the oracle).  The 3j symbol enters the isotropic
4PCF basis through C^Lambda_M = (-1)^(l1+l2+l3) (l1 l2 l3; m1 m2 m3)
(Sec. 2.3, the equation defining C^Lambda_M).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache


def _f(n: int) -> int:
    return math.factorial(n)


@lru_cache(maxsize=None)
def threej_squared_signed(l1: int, l2: int, l3: int, m1: int, m2: int, m3: int):
    """Return (sign, value**2) of the 3j symbol as (int, Fraction), exactly."""
    if m1 + m2 + m3 != 0:
        return 0, Fraction(0)
    if l3 < abs(l1 - l2) or l3 > l1 + l2:
        return 0, Fraction(0)
    if abs(m1) > l1 or abs(m2) > l2 or abs(m3) > l3:
        return 0, Fraction(0)
    tri = Fraction(_f(l1 + l2 - l3) * _f(l1 - l2 + l3) * _f(-l1 + l2 + l3), _f(l1 + l2 + l3 + 1))
    pf = (_f(l1 + m1) * _f(l1 - m1) * _f(l2 + m2) * _f(l2 - m2) * _f(l3 + m3) * _f(l3 - m3))
    kmin = max(0, l2 - l3 - m1, l1 - l3 + m2)
    kmax = min(l1 + l2 - l3, l1 - m1, l2 + m2)
    s = Fraction(0)
    for k in range(kmin, kmax + 1):
        den = (_f(k) * _f(l3 - l2 + k + m1) * _f(l3 - l1 + k - m2) * _f(l1 + l2 - l3 - k)
               * _f(l1 - k - m1) * _f(l2 - k + m2))
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0, Fraction(0)
    phase = -1 if (l1 - l2 - m3) % 2 else 1
    sign = phase * (1 if s > 0 else -1)
    return sign, s * s * tri * pf


def threej(l1: int, l2: int, l3: int, m1: int, m2: int, m3: int) -> float:
    """(l1 l2 l3; m1 m2 m3) as a float64 (the square root is the only rounding)."""
    sign, sq = threej_squared_signed(l1, l2, l3, m1, m2, m3)
    if sign == 0:
        return 0.0
    return sign * math.sqrt(float(sq))

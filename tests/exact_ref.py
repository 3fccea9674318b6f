"""Exact-rational brute force used to pin the oracle (tests only).

These routines re-derive results from the mathematics with Python's
``fractions.Fraction`` and CPython's correctly rounded int/int division and
``math.fsum``; they share no code with the oracle (C) or the GPU path.
"""

from __future__ import annotations

import math
from fractions import Fraction

DBL_MAX = float.fromhex("0x1.fffffffffffffp+1023")
OVERFLOW_EDGE = Fraction(2) ** 1024 - Fraction(2) ** 970  # RN(v) = inf for |v| >= this


def rn(v: Fraction) -> float:
    """Nearest double to v, ties to even (CPython's int/int division rounds correctly)."""
    if abs(v) >= OVERFLOW_EDGE:
        return math.inf if v > 0 else -math.inf
    if v == 0:
        return 0.0
    return v.numerator / v.denominator


def dot_fraction(x, y) -> Fraction:
    return sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))


def dot_rn(x, y) -> float:
    return rn(dot_fraction(x, y))


def dot_fsum(x, y) -> float:
    """Correctly rounded dot via math.fsum of the exact product halves.

    Each product a*b is split into hi = RN(a*b) and lo = a*b - hi (exact,
    representable when no underflow occurs); fsum rounds the exact sum of its
    inputs correctly (Shewchuk's algorithm as implemented by CPython)."""
    terms = []
    for a, b in zip(x, y):
        a, b = float(a), float(b)
        hi = a * b
        lo = float(Fraction(a) * Fraction(b) - Fraction(hi))
        terms.append(hi)
        terms.append(lo)
    return math.fsum(terms)


def fma_exact(a: float, b: float, c: float) -> float:
    return rn(Fraction(a) * Fraction(b) + Fraction(c))


def rn_fmt(v: Fraction, prec: int, qmin: int, emax_inf: int) -> float:
    """Nearest value with `prec` significant bits, last-bit weight >= 2^qmin,
    ties to even, overflow to infinity at 2^emax_inf (binary32: 24, -149, 128)."""
    if v == 0:
        return 0.0
    neg = v < 0
    a = -v if neg else v
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    q = max(e - (prec - 1), qmin)
    scaled = a / (Fraction(2) ** q)
    I = scaled.numerator // scaled.denominator
    rem = scaled - I
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and I % 2 == 1):
        I += 1
    val = Fraction(I) * Fraction(2) ** q
    if val >= Fraction(2) ** emax_inf:
        return -math.inf if neg else math.inf
    f = val.numerator / val.denominator
    return -f if neg else f


def rn32(v: Fraction) -> float:
    return rn_fmt(v, 24, -149, 128)

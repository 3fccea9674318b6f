"""Host check of the digit split the exact dot's direct path uses for a
product x y (Section 4.1: the product enters the long accumulator exactly).
The device forms the 106-bit product of the significands (four 32 x 32-bit
products of their halves), negates it once as
a 128-bit two's complement value when the signs differ, shifts it onto the
accumulator's 32-bit word grid and adds four unsigned 32-bit digits and the
signed rest. This test replays that integer arithmetic with 64-bit
wraparound and checks, against exact rationals, that the five adds sum to
x y exactly, that each is below 2^32 in magnitude (the accumulator's
headroom argument) and that the top word stays inside the 68 words."""

import math
import random
import struct
from fractions import Fraction

M64 = (1 << 64) - 1
ACC_EXP0 = -1088
ACC_WORDS = 68


def _bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def _sar64(v, n):
    v = v - (1 << 64) if v >> 63 else v
    return (v >> n) & M64


def _digits(x, y):
    bx, by = _bits(x), _bits(y)
    ex, ey = (bx >> 52) & 0x7FF, (by >> 52) & 0x7FF
    mx, my = bx & ((1 << 52) - 1), by & ((1 << 52) - 1)
    if ex:
        mx |= 1 << 52
    else:
        ex = 1
    if ey:
        my |= 1 << 52
    else:
        ey = 1
    off = ex + ey - 2150 - ACC_EXP0
    k, s = off >> 5, off & 31
    # the device's schoolbook on 32-bit halves, each step checked for 64-bit overflow
    xl, xh, yl, yh = mx & 0xFFFFFFFF, mx >> 32, my & 0xFFFFFFFF, my >> 32
    p0 = xl * yl
    mid = xl * yh + (p0 >> 32)
    assert mid <= M64
    mid += xh * yl
    assert mid <= M64
    lo = (p0 & 0xFFFFFFFF) | ((mid << 32) & M64)
    hi = xh * yh + (mid >> 32)
    assert hi < 1 << 42 and (hi << 64) | lo == mx * my
    if (bx ^ by) >> 63:
        nlo = (0 - lo) & M64
        hi = (~hi + (1 if lo == 0 else 0)) & M64
        lo = nlo
    w0 = (lo << s) & M64
    w1 = ((hi << s) | ((lo >> (64 - s)) if s else 0)) & M64
    w2 = _sar64(hi, 64 - s) if s else _sar64(hi, 63)
    c = [w0 & 0xFFFFFFFF, w0 >> 32, w1 & 0xFFFFFFFF, w1 >> 32, w2]
    return k, [v - (1 << 64) if v >> 63 else v for v in c]


def _check(x, y):
    k, c = _digits(x, y)
    assert 0 <= k and k + 4 < ACC_WORDS, (x, y, k)
    assert all(abs(v) < (1 << 32) for v in c), (x, y, c)
    got = sum(Fraction(v) * Fraction(2) ** (32 * (k + i) + ACC_EXP0) for i, v in enumerate(c))
    assert got == Fraction(x) * Fraction(y), (x, y)


def _in_range(x, y):
    r = x * y
    return x != 0 and y != 0 and math.isfinite(r) and abs(r) >= 2.0 ** -969


def test_random_products_all_exponents():
    rng = random.Random(20)
    n = 0
    while n < 20000:
        x = rng.choice((-1, 1)) * rng.random() * 2.0 ** rng.randint(-1074, 1023)
        y = rng.choice((-1, 1)) * rng.random() * 2.0 ** rng.randint(-1074, 1023)
        if _in_range(x, y):
            _check(x, y)
            n += 1


def test_edge_products():
    tiny = 5e-324
    big = 1.7976931348623157e308
    cases = [(tiny, 2.0 ** 1000), (-3 * tiny, 2.0 ** 1023), (big, 0.9999999999999999), (-big, 0.5),
             (2.0 ** -500, -2.0 ** -469), (-1.0, -1.0), (1.0, -1.0), (-(2.0 ** 53 - 1), 2.0 ** 53 - 1)]
    for x, y in cases:
        assert _in_range(x, y)
        _check(x, y)


def test_every_shift_both_signs():
    for s in range(64):
        for sign in (1, -1):
            _check(sign * (1 + 2.0 ** -52) * 2.0 ** (s - 10), 3.0 * 2.0 ** 7)
            _check(sign * 2.0 ** (s - 40), -(2.0 - 2.0 ** -52))


def _exponents_in_range(x, y):
    """The device's exponent-only test for the direct add (normal operands,
    1077 <= ex + ey <= 3067 on the biased exponents)."""
    ex, ey = (_bits(x) >> 52) & 0x7FF, (_bits(y) >> 52) & 0x7FF
    return 0 < ex < 0x7FF and 0 < ey < 0x7FF and 1077 <= ex + ey <= 3067


def test_exponent_test_implies_range():
    """Where the exponent-only test admits a product, the rounded-product
    condition holds too (so the direct add's preconditions are met), checked
    at the bounds of the test with the smallest and largest significands and
    on random pairs."""
    lo_sig, hi_sig = 1.0, 2.0 - 2.0 ** -52
    cases = []
    for e in (1077, 1078, 2046, 3066, 3067):
        for ex in (max(1, e - 2046), e // 2, min(2046, e - 1)):
            ey = e - ex
            if not (0 < ex < 2047 and 0 < ey < 2047):
                continue
            for sx in (lo_sig, hi_sig):
                for sy in (lo_sig, hi_sig):
                    cases.append((sx * 2.0 ** (ex - 1023), -sy * 2.0 ** (ey - 1023)))
    rng = random.Random(21)
    while len(cases) < 20000:
        x = rng.choice((-1, 1)) * (1 + rng.random()) * 2.0 ** rng.randint(-1022, 1023)
        y = rng.choice((-1, 1)) * (1 + rng.random()) * 2.0 ** rng.randint(-1022, 1023)
        if _exponents_in_range(x, y):
            cases.append((x, y))
    for x, y in cases:
        assert _exponents_in_range(x, y), (x, y)
        assert _in_range(x, y), (x, y)
        _check(x, y)
    # the bounds are tight: one binade lower may fall below 2^-969
    assert not _in_range(2.0 ** -485, 2.0 ** -485)

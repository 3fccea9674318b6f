"""Pins for the oracle's exact dot product (Sections 2, 2.1 and 4.3: the
result of the reproducible dot is the exact sum of products rounded once to
nearest, ties to even). Checked against exact rational brute force, math.fsum,
hand-derived rounding cases, invariances and closed-form constructions."""

import math
import random
import struct
from fractions import Fraction

import numpy as np
import pytest

from exact_ref import DBL_MAX, dot_fraction, dot_fsum, dot_rn, rn
from rpcg_workloads import exdot_conditioned, exdot_narrow, exdot_wide


def bits(v: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def same(a: float, b: float) -> bool:
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return bits(a) == bits(b)


def _rand_double(rng, emin, emax):
    m = 1.0 + rng.getrandbits(52) * 2.0 ** -52
    return math.copysign(math.ldexp(m, rng.randint(emin, emax)), rng.choice((-1.0, 1.0)))


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_small(orc, seed):
    rng = random.Random(seed)
    n = rng.randint(0, 64)
    lo, hi = [(-2, 2), (-60, 60), (-300, 300), (-1074, -1000), (900, 1000)][seed % 5]
    x = [_rand_double(rng, lo, hi) for _ in range(n)]
    y = [_rand_double(rng, lo, hi) for _ in range(n)]
    if seed % 7 == 3 and n > 1:  # insert exact cancellations
        x[1], y[1] = x[0], -y[0]
    want = dot_rn(x, y)
    got = orc.exdot(np.array(x), np.array(y))
    assert same(got, want), (seed, got, want)


def test_subnormal_products(orc):
    tiny = 5e-324  # 2^-1074
    cases = [
        ([3 * tiny], [0.5], 2 * tiny),   # 1.5 ulp -> tie -> even (2 ulp)
        ([tiny], [0.5], 0.0),            # 0.5 ulp -> tie -> even (0)
        ([tiny], [0.75], tiny),          # 0.75 ulp -> 1 ulp
        ([5 * tiny], [0.5], 2 * tiny),   # 2.5 ulp -> tie -> 2 ulp
        ([7 * tiny], [0.5], 4 * tiny),   # 3.5 ulp -> tie -> 4 ulp
        ([2.0 ** -1022], [-0.5], -(2.0 ** -1023)),
        ([tiny, tiny], [tiny, tiny], 0.0),  # 2^-2147 rounds to +0
        ([3 * tiny, tiny], [0.5, -(2.0 ** -60)], tiny),  # just below a tie: one rounding only
        ([5 * tiny, tiny], [0.5, 2.0 ** -70], 3 * tiny),  # just above a tie
    ]
    for x, y, want in cases:
        got = orc.exdot(np.array(x), np.array(y))
        assert same(got, want), (x, y, got, want)
        assert same(got, dot_rn(x, y))


def test_hand_ties(orc):
    e = 2.0 ** -53
    cases = [
        ([1.0, e], 1.0),                      # exact half-ulp tie, 1.0 has even mantissa
        ([1.0, 3 * e], 1.0 + 2.0 ** -51),     # 1 + 1.5 ulp -> tie to even -> 1 + 2 ulp
        ([1.0, e, 2.0 ** -200], 1.0 + 2.0 ** -52),  # sticky bit breaks the tie upward
        ([1.0 + 2.0 ** -52, e], 1.0 + 2.0 ** -51),  # odd mantissa + half ulp -> up
        ([-1.0, -e], -1.0),
        ([2.0 ** 600, 1.0, -(2.0 ** 600)], 1.0),    # large cancellation leaves 1
    ]
    for x, want in cases:
        got = orc.exdot(np.array(x), np.ones(len(x)))
        assert same(got, want), (x, got, want)


def test_overflow_boundary(orc):
    # Midpoint between DBL_MAX and 2^1024 rounds to even, i.e. up to infinity.
    x = np.array([DBL_MAX, 2.0 ** 970])
    assert orc.exdot(x, np.ones(2)) == math.inf
    assert orc.exdot(-x, np.ones(2)) == -math.inf
    x = np.array([DBL_MAX, 2.0 ** 970, -(2.0 ** -1074)])
    assert orc.exdot(x, np.ones(3)) == DBL_MAX
    # Sum beyond the double range that cancels back into range stays exact.
    x = np.array([DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX, 3.0])
    assert orc.exdot(x, np.ones(5)) == 3.0


def test_zero_and_signs(orc):
    assert same(orc.exdot(np.array([]), np.array([])), 0.0)
    assert same(orc.exdot(np.array([-0.0]), np.array([1.0])), 0.0)
    assert same(orc.exdot(np.array([-0.0, -0.0]), np.array([0.0, 0.0])), 0.0)
    x = np.array([1.5, -1.5, 2.0 ** -30, -(2.0 ** -30)])
    assert same(orc.exdot(x, np.ones(4)), 0.0)  # exact zero is +0


def test_nonfinite_gives_nan(orc):
    assert math.isnan(orc.exdot(np.array([1.0, math.inf]), np.array([1.0, 1.0])))
    assert math.isnan(orc.exdot(np.array([1.0, math.nan]), np.array([1.0, 1.0])))


@pytest.mark.parametrize("kind", ["narrow", "wide"])
def test_fsum_medium(orc, kind):
    n = 20000
    x, y = (exdot_narrow if kind == "narrow" else exdot_wide)(5, n)
    assert same(orc.exdot(x, y), dot_fsum(x, y))


@pytest.mark.parametrize("cond", [1e0, 1e8, 1e16, 1e24, 1e32])
def test_conditioned_closed_form(orc, cond):
    n = 5000
    x, y, exact = exdot_conditioned(11, n, cond)
    got = orc.exdot(x, y)
    if exact is not None:
        assert got == exact
    assert same(got, dot_fsum(x, y))
    # measured condition number lands within a decade of the request
    E_abs = orc.exdot_exact(np.abs(x), np.abs(y))
    E = orc.exdot_exact(x, y)
    meas = abs(E_abs) / abs(E)
    assert cond / 10 <= meas <= cond * 10


def test_conditioned_large_n_closed_form(orc):
    x, y, exact = exdot_conditioned(3, 1 << 20, 1e24)
    assert orc.exdot(x, y) == exact


def test_exact_integer_matches_fraction(orc):
    rng = random.Random(7)
    for _ in range(10):
        n = rng.randint(1, 40)
        x = [_rand_double(rng, -1074, 1000) for _ in range(n)]
        y = [_rand_double(rng, -1074, 1000) for _ in range(n)]
        F = dot_fraction(x, y) * Fraction(2) ** 2148
        assert F.denominator == 1
        assert orc.exdot_exact(np.array(x), np.array(y)) == F.numerator
        assert same(orc.round_exact(F.numerator), rn(F / Fraction(2) ** 2148))


def test_permutation_and_split_invariance(orc):
    x, y = exdot_wide(21, 4097)
    ref = orc.exdot(x, y)
    rng = np.random.default_rng(0)
    for _ in range(5):
        p = rng.permutation(x.size)
        assert same(orc.exdot(x[p], y[p]), ref)
    E = orc.exdot_exact(x, y)
    for cut in (0, 1, 100, 2048, 4096, 4097):
        assert orc.exdot_exact(x[:cut], y[:cut]) + orc.exdot_exact(x[cut:], y[cut:]) == E


def test_plain_sum_degrades_with_condition(orc):
    """Contrast: a naive left-to-right fp64 sum loses all digits at cond 1e32,
    while the oracle keeps relative error <= 2^-53."""
    x, y, exact = exdot_conditioned(4, 4000, 1e32)
    naive = float(np.sum(x * y))
    assert abs(naive - exact) / abs(exact) > 1e-3
    assert abs(orc.exdot(x, y) - exact) <= abs(exact) * 2.0 ** -53

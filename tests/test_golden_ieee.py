"""The oracle's rounding and long accumulator against the floating-point
parameters the paper prints (Table 1 and the dynamic-range sentence of
Section 2), read from tests/golden/ieee754_parameters.txt."""

import math
import os
from decimal import Decimal, getcontext

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ieee754_parameters.txt")


def golden():
    rows = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, *vals = line.split()
        rows[name] = vals
    return rows


def test_unit_roundoff_is_the_tie_point(orc):
    """u = 2^-53 (binary64) and 2^-24 (binary32) are where rounding to
    nearest-even flips: 1 + u is a tie that rounds down to 1, anything above
    it rounds up to the next number, 1 + 2u."""
    g = golden()
    p64, _, e64 = (int(v) for v in g["double"])
    p32, _, e32 = (int(v) for v in g["single"])
    assert e64 == -p64 and e32 == -p32
    u = 2.0 ** e64
    assert orc.exdot(np.array([1.0, u]), np.ones(2)) == 1.0
    assert orc.exdot(np.array([1.0, u, 2.0 ** -200]), np.ones(3)) == 1.0 + 2 * u
    u32 = 2.0 ** e32
    one32 = np.float32(1.0)
    assert orc.exdot_f32(np.array([1.0, u32], np.float32), np.ones(2, np.float32)) == one32
    above = orc.exdot_f32(np.array([1.0, u32, 2.0 ** -100], np.float32), np.ones(3, np.float32))
    assert above == np.nextafter(one32, np.float32(2.0))


def test_binary64_range_and_dynamic_range(orc):
    """The printed extremes and their ratio are those of binary64 (to two
    digits), and the oracle's exact accumulation holds both ends at once."""
    g = golden()
    tiny, huge = 2.0 ** -1074, float(np.finfo(np.float64).max)
    getcontext().prec = 50
    pmin, pmax, prange = (Decimal(g[k][0]) for k in ("double_min", "double_max", "double_range"))
    # two printed digits: within half a unit of the second digit
    assert abs(Decimal(tiny) - pmin) <= Decimal("0.05e-324")
    assert abs(Decimal(huge) - pmax) <= Decimal("0.05e308")
    # the printed range is the ratio of the printed extremes, rounded to two digits
    assert f"{pmax / pmin:.1e}" == f"{prange:.1e}"
    true_ratio = Decimal(huge) / Decimal(tiny)
    assert abs(true_ratio / prange - 1) < Decimal("0.03")
    E = orc.exdot_exact(np.array([huge, tiny]), np.ones(2))
    Eh = orc.exdot_exact(np.array([huge]), np.ones(1))
    assert E - Eh == 1 << (2148 - 1074)  # the smallest subnormal, exactly
    assert orc.round_exact(E) == huge and math.isfinite(orc.round_exact(E))

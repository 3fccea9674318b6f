"""The oracle's threaded loops give the same bits at any thread count: the
exact dot adds per-thread integer accumulators exactly, and every other loop
computes each element by the same operations whatever thread runs it."""

import numpy as np
import pytest

from rpcg_workloads import (exdot_conditioned, exdot_wide, stencil27_csr, stencil27_rhs_from_int52,
                            stencil7_varcoef_csr, uniform_pm1, uniform_pm1_int52)


@pytest.fixture
def threads(orc):
    before = orc.get_threads()
    yield orc
    orc.set_threads(before)


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("counts", [(1, 2), (1, 3), (1, 8), (1, 16)])
def test_exdot_thread_invariant(threads, counts):
    orc = threads
    for x, y in (exdot_wide(5, 100_003), exdot_conditioned(6, 50_001, 1e24)[:2]):
        got = []
        for t in counts:
            orc.set_threads(t)
            got.append((orc.exdot(x, y), orc.exdot_exact(x, y)))
        assert _bits([got[0][0]])[0] == _bits([got[1][0]])[0]
        assert got[0][1] == got[1][1]


def test_pcg_and_residual_thread_invariant(threads):
    orc = threads
    N = 20
    A = stencil27_csr(N)
    b = stencil27_rhs_from_int52(N, uniform_pm1_int52(4, A.n))
    V = stencil7_varcoef_csr(12, 3)
    bv = uniform_pm1(5, V.n)
    res = {}
    for t in (1, 7):
        orc.set_threads(t)
        assert orc.get_threads() == t
        r1 = orc.pcg(A, b, tol=1e-10)
        r2 = orc.pcg(V, bv, tol=1e-10)
        res[t] = (r1, r2, orc.true_residual(V, bv, r2["x"]))
    for a, c in zip(res[1][:2], res[7][:2]):
        assert a["iters"] == c["iters"]
        assert np.array_equal(_bits(a["x"]), _bits(c["x"]))
        assert np.array_equal(_bits(a["hist"]), _bits(c["hist"]))
    assert np.array_equal(_bits(res[1][2]), _bits(res[7][2]))


def test_cpu_plain_loop_converges(threads):
    """The host comparison loop (ordinary dots) reaches the tolerance in about
    the exact loop's iteration count."""
    orc = threads
    N = 16
    A = stencil27_csr(N)
    b = stencil27_rhs_from_int52(N, uniform_pm1_int52(2, A.n))
    ref = orc.pcg(A, b)
    p = orc.cpu_plain_pcg(A, b)
    assert p["status"] == 0 and abs(p["iters"] - ref["iters"]) <= 2
    assert orc.relres_true(A, b, p["x"]) < 1.01e-8

"""Pins for the oracle's binary32 routines and the mixed-precision refinement
(the precision form of the method: binary32 inner Jacobi-PCG with exact
dots rounded to binary32, binary64 outer residuals with exact accumulation)."""

import math
import random
from fractions import Fraction

import numpy as np
import pytest

from exact_ref import rn32
from rpcg_workloads import CSRHost, random_spd_csr, stencil27_csr, stencil27_rhs_from_int52, uniform_pm1_int52


def _f32(v):
    return float(np.float32(v))


@pytest.mark.parametrize("seed", range(20))
def test_exdot_f32_bruteforce(orc, seed):
    rng = random.Random(seed)
    n = rng.randint(0, 50)
    lo, hi = [(-3, 3), (-40, 40), (-149, -120), (100, 127)][seed % 4]
    x = np.array([math.ldexp(rng.random() + 1.0, rng.randint(lo, hi)) * rng.choice((-1, 1)) for _ in range(n)],
                 dtype=np.float32)
    y = np.array([math.ldexp(rng.random() + 1.0, rng.randint(lo, hi)) * rng.choice((-1, 1)) for _ in range(n)],
                 dtype=np.float32)
    exact = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    want = rn32(exact)
    got = float(orc.exdot_f32(x, y))
    assert got == want or (math.isnan(got) and math.isnan(want)), (seed, got, want)


def test_exdot_f32_ties_and_subnormals(orc):
    e = 2.0 ** -24
    assert float(orc.exdot_f32([1.0, e], [1.0, 1.0])) == 1.0                 # tie to even
    assert float(orc.exdot_f32([1.0, 3 * e], [1.0, 1.0])) == 1.0 + 2.0 ** -22
    assert float(orc.exdot_f32([1.0, e, 2.0 ** -100], [1.0, 1.0, 1.0])) == 1.0 + 2.0 ** -23
    t = 2.0 ** -149
    assert float(orc.exdot_f32([3 * t], [0.5])) == 2 * t                    # 1.5 ulp -> 2 ulp
    assert float(orc.exdot_f32([3 * t, t], [0.5, -(2.0 ** -30)])) == t      # just below a tie
    big = float(np.finfo(np.float32).max)
    assert float(orc.exdot_f32([big, 2.0 ** 103], [1.0, 1.0])) == math.inf   # midpoint -> even -> inf
    assert float(orc.exdot_f32([big, 2.0 ** 103, -t], [1.0, 1.0, 1.0])) == big


def test_exdot_f32_differs_from_double_rounding(orc):
    """Rounding the exact value straight to binary32 is not the same as rounding
    to binary64 first: a value just above a binary32 tie that rounds to the tie
    in binary64 must still round up."""
    x = [1.0, 2.0 ** -24, 2.0 ** -80]
    exact = Fraction(1) + Fraction(2) ** -24 + Fraction(2) ** -80
    assert rn32(exact) == 1.0 + 2.0 ** -23
    assert float(np.float32(float(exact))) == 1.0  # double rounding gets it wrong
    assert float(orc.exdot_f32(x, [1.0, 1.0, 1.0])) == 1.0 + 2.0 ** -23


def test_spmv_f32_fmaf_chain(orc):
    rng = np.random.default_rng(2)
    n = 40
    rows, cols = np.nonzero(rng.random((n, n)) < 0.3)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    A = CSRHost(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32),
                rng.standard_normal(rows.size).astype(np.float32).astype(np.float64))
    x = rng.standard_normal(n).astype(np.float32)
    y = orc.spmv_f32(A, x)
    for i in range(n):
        acc = 0.0
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc = rn32(Fraction(float(np.float32(A.val[k]))) * Fraction(float(x[A.col_idx[k]])) + Fraction(acc))
        assert float(y[i]) == acc


def test_pcg_f32_converges_and_stops_right(orc):
    N = 10
    A = stencil27_csr(N)
    b = orc.spmv_f32(A, np.ones(A.n, np.float32))
    res = orc.pcg_f32(A, b, tol=1e-4)
    assert res["status"] == 0
    L = res["iters"]
    bb = float(orc.exdot_f32(b, b))
    thr = _f32(_f32(_f32(1e-4) * _f32(1e-4)) * bb)
    assert res["hist"][L] <= thr < res["hist"][L - 1]
    assert np.max(np.abs(res["x"] - 1.0)) < 1e-2


def test_pcg_f32_diagonal_one_step(orc):
    n = 8
    d = (np.arange(1, n + 1) * 0.25).astype(np.float64)
    A = CSRHost(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    res = orc.pcg_f32(A, np.ones(n, np.float32), tol=1e-6)
    assert res["iters"] == 1
    assert np.array_equal(res["x"], (np.float32(1.0) / d.astype(np.float32)).astype(np.float32))


def test_pcg_f32_tracks_exact_cg(orc):
    A = random_spd_csr(6, 3)
    b = np.array([0.5, -1.0, 0.25, 2.0, -0.75, 1.5], np.float32)
    res = orc.pcg_f32(A, b, tol=1e-6)
    xs = np.linalg.solve(_dense(A), b.astype(float))
    assert np.allclose(res["x"], xs, rtol=1e-4, atol=1e-5)


def _dense(A):
    D = np.zeros((A.n, A.n))
    for i in range(A.n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col_idx[k]] = A.val[k]
    return D


def test_ir_scale(orc):
    for rr, want in ((1.0, 0), (2.0, 0), (4.0, 1), (0.25, -1), (0.5, -1), (2.0 ** -101, -51), (3 * 2.0 ** 40, 20)):
        assert orc.ir_scale(rr) == want, rr


def test_ir_reaches_fp64_accuracy(orc):
    """The refinement reaches 1e-10 relative residual with a binary32 inner solver;
    its solution agrees with the binary64 exact-dot PCG solution to ~1e-9."""
    N = 12
    A = stencil27_csr(N)
    K = uniform_pm1_int52(5, A.n)
    b = stencil27_rhs_from_int52(N, K)
    xs = K * 2.0 ** -52
    res = orc.ir(A, b, tol=1e-10, tol_in=1e-4)
    assert res["status"] == 0
    assert 2 <= res["outer"] <= 6
    h = res["hist"]
    assert all(h[k + 1] < h[k] * 1e-2 for k in range(len(h) - 1))
    assert orc.relres_true(A, b, res["x"]) <= 1e-10
    ref = orc.pcg(A, b, tol=1e-10)
    err = np.max(np.abs(res["x"] - ref["x"])) / np.max(np.abs(ref["x"]))
    assert err < 1e-8
    assert np.max(np.abs(res["x"] - xs)) < 1e-8


def test_ir_adaptive_inner_tolerance(orc):
    """The adaptive rule only loosens a step's inner tolerance when the outer
    residual needs less than tol_in of reduction: the earlier steps are the
    fixed-tolerance ones bit for bit, the last one stops nearer the target
    (still below it) with fewer inner iterations."""
    N = 16
    A = stencil27_csr(N)
    K = uniform_pm1_int52(8, A.n)
    b = stencil27_rhs_from_int52(N, K)
    fixed = orc.ir(A, b, tol=1e-10, tol_in=1e-4, adaptive=False)
    ad = orc.ir(A, b, tol=1e-10, tol_in=1e-4, adaptive=True)
    assert fixed["status"] == 0 and ad["status"] == 0
    k = ad["outer"]
    assert fixed["outer"] == k >= 2
    assert np.array_equal(ad["hist"][:k], fixed["hist"][:k])
    thr = 1e-20 * orc.exdot(b, b)
    assert fixed["hist"][k] < ad["hist"][k] <= thr
    assert ad["inner"] < fixed["inner"]
    assert orc.relres_true(A, b, ad["x"]) <= 1e-10


def test_ir_first_step_is_the_f32_solve(orc):
    """With one outer step the refinement's x is exactly (double)c 2^s of the
    binary32 solve of the scaled right-hand side (x0 = 0, r0 = b)."""
    N = 6
    A = stencil27_csr(N)
    b = orc.spmv(A, np.linspace(-1, 1, A.n))
    res = orc.ir(A, b, tol=1e-30, maxit_out=1, tol_in=1e-4)
    rr = orc.exdot(b, b)
    s = orc.ir_scale(rr)
    inner = orc.pcg_f32(A, np.ldexp(b, -s).astype(np.float32), tol=1e-4)
    assert np.array_equal(res["x"], np.ldexp(inner["x"].astype(np.float64), s))


def test_ir_outer_residual_uses_binary64_values(orc):
    """Values not representable in binary32 (a stencil scaled by 1/3 and an
    SPD shift): the inner solves see the binary32 rounding of A, but the outer
    residual is formed with A itself, so the refinement still drives the true
    binary64 residual below 1e-12; a solve of the rounded system alone would
    stall near binary32's relative precision (~1e-8)."""
    N = 8
    A0 = stencil27_csr(N)
    val = A0.val / 3.0 + np.where(A0.val > 0, 0.1, 0.0)
    A = CSRHost(A0.n, A0.row_ptr, A0.col_idx, val)
    assert np.any(val.astype(np.float32).astype(np.float64) != val)
    b = orc.spmv(A, np.linspace(-1, 1, A.n))
    res = orc.ir(A, b, tol=1e-12, tol_in=1e-4)
    assert res["status"] == 0
    assert orc.relres_true(A, b, res["x"]) <= 1e-12
    A32 = CSRHost(A.n, A.row_ptr, A.col_idx, val.astype(np.float32).astype(np.float64))
    x32 = orc.pcg(A32, b, tol=1e-14, maxit=5000)["x"]
    assert orc.relres_true(A, b, x32) > 1e-10

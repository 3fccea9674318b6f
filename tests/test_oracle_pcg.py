"""Pins for the oracle's Jacobi-PCG (Fig. 1 / Fig. 2, Section 3.1 Jacobi,
Section 4.3 fma updates): exact-rational CG on tiny systems, textbook CG
invariants, closed-form spectral bounds, and the degenerate cases."""

import math
from fractions import Fraction

import numpy as np
import pytest

from rpcg_workloads import (CSRHost, random_spd_csr, stencil27_csr, stencil27_rhs_from_int52,
                            uniform_pm1_int52)


def _dense(A):
    D = np.zeros((A.n, A.n))
    for i in range(A.n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col_idx[k]] = A.val[k]
    return D


def rational_pcg(A, b, iters):
    """Textbook Jacobi-PCG in exact rational arithmetic (no rounding)."""
    n = A.n
    D = [[Fraction(v) for v in row] for row in _dense(A)]
    M = [D[i][i] for i in range(n)]
    x = [Fraction(0)] * n
    r = [Fraction(v) for v in b]
    z = [r[i] / M[i] for i in range(n)]
    d = list(z)
    beta = sum(z[i] * r[i] for i in range(n))
    taus = [sum(v * v for v in r)]
    xs = [list(x)]
    for _ in range(iters):
        if taus[-1] == 0:
            break
        w = [sum(D[i][j] * d[j] for j in range(n)) for i in range(n)]
        rho = beta / sum(d[i] * w[i] for i in range(n))
        x = [x[i] + rho * d[i] for i in range(n)]
        r = [r[i] - rho * w[i] for i in range(n)]
        z = [r[i] / M[i] for i in range(n)]
        beta_new = sum(z[i] * r[i] for i in range(n))
        d = [z[i] + (beta_new / beta) * d[i] for i in range(n)]
        beta = beta_new
        taus.append(sum(v * v for v in r))
        xs.append(list(x))
    return xs, taus


@pytest.mark.parametrize("seed", range(6))
def test_tiny_spd_matches_exact_rational_cg(orc, seed):
    n = 3 + seed % 5
    A = random_spd_csr(n, seed)
    b = (np.arange(n) % 3 - 1.0) + 0.5
    res = orc.pcg(A, b, tol=1e-12, maxit=50)
    xs, taus = rational_pcg(A, b, n)
    # exact CG terminates in at most n steps
    assert taus[-1] == 0 or len(taus) <= n + 1
    xstar = np.linalg.solve(_dense(A), b)
    assert res["status"] == 0
    assert np.allclose(res["x"], xstar, rtol=1e-10, atol=1e-12)
    assert res["iters"] <= n + 2
    # the first steps track exact arithmetic closely
    for l in range(1, min(3, len(taus), res["iters"] + 1)):
        assert abs(res["hist"][l] - float(taus[l])) <= 1e-9 * float(taus[0])


def test_diagonal_matrix_one_step(orc):
    """Jacobi is exact for a diagonal matrix: one iteration reaches r = 0."""
    n = 16
    d = np.arange(1, n + 1, dtype=np.float64) * 0.5
    A = CSRHost(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = np.ones(n)
    res = orc.pcg(A, b, tol=1e-14, maxit=10)
    assert res["iters"] == 1
    assert np.array_equal(res["x"], 1.0 / d)


def _lam_stencil27(N):
    j = np.arange(1, N + 1)
    mu = 1 + 2 * np.cos(np.pi * j / (N + 1))
    lam = 27 - np.einsum("i,j,k->ijk", mu, mu, mu).reshape(-1)
    return lam.min(), lam.max()


def test_stencil27_convergence_and_invariants(orc):
    N = 8
    A = stencil27_csr(N)
    K = uniform_pm1_int52(1, A.n)
    b = stencil27_rhs_from_int52(N, K)
    xstar = K * 2.0 ** -52
    res = orc.pcg(A, b, tol=1e-8, maxit=500, trace=True)
    L = res["iters"]
    assert res["status"] == 0
    # closed-form spectrum: CG iteration bound 1/2 sqrt(kappa) ln(2/tol), kappa of the
    # Jacobi-preconditioned operator = kappa(A) since diag(A) = 26 I
    lmin, lmax = _lam_stencil27(N)
    kappa = lmax / lmin
    assert L <= math.ceil(0.5 * math.sqrt(kappa) * math.log(2 / 1e-8)) + 2
    # stopping rule: tau_L <= thr < tau_{L-1}
    thr = (1e-8 * 1e-8) * orc.exdot(b, b)
    assert res["hist"][L] <= thr < res["hist"][L - 1]
    assert res["hist"][0] == orc.exdot(b, b)
    # recursively updated residual tracks the true residual
    R, Dd, X = res["trace_r"], res["trace_d"], res["trace_x"]
    nb = math.sqrt(orc.exdot(b, b))
    for l in range(0, L + 1, max(1, L // 6)):
        rt = orc.true_residual(A, b, X[l])
        assert np.linalg.norm(R[l] - rt) <= 1e-12 * nb
    # M^-1 orthogonality of residuals and A-conjugacy of directions
    dinv = 1.0 / 26.0
    for i in range(0, L, 3):
        for j in range(i + 1, min(L, i + 4)):
            zi = dinv * R[i]
            c = orc.exdot(zi, R[j]) / math.sqrt(orc.exdot(zi, R[i]) * orc.exdot(dinv * R[j], R[j]))
            assert abs(c) < 1e-6, (i, j, c)
            Adi = orc.spmv(A, Dd[i])
            Adj = orc.spmv(A, Dd[j])
            c = orc.exdot(Dd[j], Adi) / math.sqrt(orc.exdot(Dd[i], Adi) * orc.exdot(Dd[j], Adj))
            assert abs(c) < 1e-6, (i, j, c)
    # A-norm of the error decreases monotonically
    errs = []
    for l in range(L + 1):
        e = X[l] - xstar
        errs.append(orc.exdot(e, orc.spmv(A, e)))
    assert all(errs[l + 1] < errs[l] for l in range(L))
    # and the answer is the known solution
    assert np.max(np.abs(res["x"] - xstar)) < 1e-6


def test_paper_rhs_ones(orc):
    """Section 5.1 setup: b = A * ones, x0 = 0, tolerance 1e-8."""
    N = 10
    A = stencil27_csr(N)
    b = orc.spmv(A, np.ones(A.n))
    res = orc.pcg(A, b, tol=1e-8, maxit=500)
    assert res["status"] == 0
    assert np.max(np.abs(res["x"] - 1.0)) < 1e-6
    assert orc.relres_true(A, b, res["x"]) < 1e-8


def test_zero_rhs_zero_iterations(orc):
    A = stencil27_csr(4)
    res = orc.pcg(A, np.zeros(A.n), tol=1e-8, maxit=10)
    assert res["iters"] == 0 and res["status"] == 0
    assert np.all(res["x"] == 0)


def test_maxit_warning(orc):
    A = stencil27_csr(6)
    b = orc.spmv(A, np.ones(A.n))
    res = orc.pcg(A, b, tol=1e-8, maxit=3)
    assert res["iters"] == 3 and res["status"] == 1
    assert len(res["hist"]) == 4


def test_not_spd_and_nonfinite(orc):
    A = stencil27_csr(3)
    bad = CSRHost(A.n, A.row_ptr, A.col_idx, np.where(A.val == 26.0, -26.0, A.val))
    assert orc.pcg(bad, np.ones(A.n))["status"] == -4
    b = np.ones(A.n)
    b[5] = np.nan
    assert orc.pcg(A, b)["status"] == -6


def test_missing_diagonal_is_not_spd(orc):
    A = CSRHost(2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    assert orc.pcg(A, np.ones(2))["status"] == -4


def test_breakdown_on_indefinite(orc):
    """Positive diagonal but indefinite matrix: <d, A d> <= 0 is reported."""
    A = CSRHost(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32),
                np.array([1.0, 3.0, 3.0, 1.0]))
    res = orc.pcg(A, np.array([1.0, -1.0]))
    assert res["status"] == -5


def test_jacobi_is_inverse_then_multiply(orc):
    """Section 4.3 (preconditioner paragraph): the inverse diagonal is formed once and
    z = RN(dinv * r); this differs from r / a_ii in the last bit for many entries."""
    n = 400
    d = 3.0 + (np.arange(n) % 7)
    A = CSRHost(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b = np.random.default_rng(2).uniform(-1, 1, n)
    res = orc.pcg(A, b, tol=0.0, maxit=0, trace=True)
    r0, d0 = res["trace_r"][0], res["trace_d"][0]
    assert np.array_equal(r0, b)
    assert np.array_equal(d0, (1.0 / d) * r0)
    assert not np.array_equal(d0, r0 / d)

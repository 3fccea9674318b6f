"""Pins of the stress-workload generators (the band transform of Section 5.1,
the first-row/column scaling of Section 5.3, the SuiteSparse-shaped stand-ins
of Section 5.4) and a scaling invariance of Jacobi-PCG with exact dots that
the oracle must show: for D = diag(2^e_i), PCG on (D B D, D b) runs the
iterates of PCG on (B, b) scaled exactly, r' = D r, p' = D^-1 p,
x' = D^-1 x, bit for bit, since every product, fma and correctly rounded dot
only meets power-of-two factors that cancel (no overflow or subnormals)."""

import numpy as np
import pytest
import scipy.sparse as sp

from rpcg_workloads import (SUITESPARSE_LIKE, band_csr, scale_first, scale_sym, suitesparse_like,
                            suitesparse_like_parts, uniform_pm1)


def _dense(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n)).toarray()


def _eq(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("n,w", [(1, 0), (5, 1), (9, 4), (60, 7), (40, 39), (30, 100)])
def test_band_structure(n, w):
    A = band_csr(n, w)
    wc = min(w, n - 1)
    assert A.row_ptr[-1] == (2 * wc + 1) * n - wc * (wc + 1)
    M = _dense(A)
    i, j = np.indices((n, n))
    inside = np.abs(i - j) <= w
    assert np.array_equal(M != 0, inside)
    assert np.all(M[inside & (i != j)] == -1.0)
    assert np.all(np.diag(M) == 2 * w + 1)
    for r in range(n):
        cols = A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


def test_band_spectrum():
    """The band matrix is a section of the Toeplitz operator whose symbol is
    f(t) = 2w + 2 - D_w(t), D_w the Dirichlet kernel sin((w + 1/2) t) / sin(t / 2):
    its eigenvalues lie strictly inside (min f, max f) = (1, max f) and
    approach both ends as n grows."""
    for n, w in [(60, 7), (400, 3)]:
        t = np.linspace(1e-9, np.pi, 200001)
        f = 2 * w + 2 - np.sin((w + 0.5) * t) / np.sin(t / 2)
        ev = np.linalg.eigvalsh(_dense(band_csr(n, w)))
        assert ev[0] > 1.0 and ev[-1] < f.max()
        assert ev[0] < 1.0 + 30.0 / n and ev[-1] > 0.97 * f.max()


def test_scale_first_exact():
    A = band_csr(20, 3)
    s = 2.0 ** 16
    S = scale_first(A, s)
    M, Ms = _dense(A), _dense(S)
    D = np.ones(20)
    D[0] = s
    assert _eq(Ms, D[:, None] * M * D[None, :])
    assert Ms[0, 0] == M[0, 0] * s * s and Ms[0, 1] == -s and Ms[1, 1] == M[1, 1]
    # the row and column scaling raises the condition number by about sigma^2
    c0, c1 = np.linalg.cond(M), np.linalg.cond(Ms)
    assert 0.1 * s * s < c1 / c0 < 10 * s * s


@pytest.mark.parametrize("nnz,cond", [p for p in SUITESPARSE_LIKE if p[0] < 40000])
def test_suitesparse_like_shape(nnz, cond):
    B, e = suitesparse_like_parts(3, nnz, cond)
    A = suitesparse_like(3, nnz, cond)
    assert nnz - 1 <= A.row_ptr[-1] <= nnz
    assert A.n == max(100, nnz // 32)
    Bd, Ad = _dense(B), _dense(A)
    assert np.array_equal(Bd, Bd.T) and np.array_equal(Ad, Ad.T)
    assert _eq(Ad, np.ldexp(Bd, e[:, None] + e[None, :]))
    np.linalg.cholesky(Bd)  # SPD
    evb = np.linalg.eigvalsh(Bd)
    kb = min(cond, 1e6)
    assert 0.1 * kb < evb[-1] / evb[0] < 10 * kb
    assert e.min() >= 0 and e.max() <= int(round(np.log2(cond / kb) / 2)) + 1


def _traces(orc, A, b, k):
    out = orc.pcg(A, b, tol=0.0, maxit=k, trace=True)
    assert out["iters"] == k
    return out


@pytest.mark.parametrize("case", ["suitesparse_1666", "suitesparse_27520", "band_scaled"])
def test_oracle_jacobi_scaling_invariance(orc, case):
    if case == "band_scaled":
        B = band_csr(300, 12)
        e = np.zeros(B.n, dtype=np.int64)
        e[0] = 16  # the first-row/column scaling with sigma = 2^16
        A = scale_sym(B, e)
        assert _eq(A.val, scale_first(B, 2.0 ** 16).val)
    else:
        nnz = int(case.split("_")[1])
        cond = dict(SUITESPARSE_LIKE)[nnz]
        B, e = suitesparse_like_parts(5, nnz, cond)
        A = scale_sym(B, e)
    b = uniform_pm1(11, B.n)
    bs = np.ldexp(b, e)
    k = 25
    t0 = _traces(orc, B, b, k)
    t1 = _traces(orc, A, bs, k)
    assert _eq(t1["trace_r"], np.ldexp(t0["trace_r"], e[None, :]))
    assert _eq(t1["trace_d"], np.ldexp(t0["trace_d"], -e[None, :]))
    assert _eq(t1["trace_x"], np.ldexp(t0["trace_x"], -e[None, :]))
    assert _eq(t1["x"], np.ldexp(t0["x"], -e))
    # tau = <r, r> does see the scaling, so it is the stopping test that differs
    assert not _eq(t1["hist"], t0["hist"]) or not e.any()


def test_oracle_scaled_band_converges(orc):
    """The ill-conditioned band system (sigma = 2^16, b = A 1, x0 = 0, tol
    1e-8, the setting of Section 5.3 at a small size) converges with the
    true residual at the requested level. The norm of b is dominated by its
    first entry (about sigma^2 times the others), so the test stops long
    before the other components of x are accurate."""
    A = scale_first(band_csr(2000, 20), 2.0 ** 16)
    b = orc.spmv(A, np.ones(A.n))
    out = orc.pcg(A, b, tol=1e-8, maxit=2000)
    assert out["status"] == 0
    assert orc.relres_true(A, b, out["x"]) < 2e-8
    assert abs(out["x"][0] - 1.0) < 1e-5
    assert np.max(np.abs(out["x"] - 1.0)) > 1e-3

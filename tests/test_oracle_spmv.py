"""Pins for the oracle's SpMV (Section 4.3, SpMV paragraph: each row is a
sequential chain of fma over its stored entries, starting from zero)."""

import numpy as np
import pytest

from exact_ref import fma_exact
from rpcg_workloads import CSRHost, stencil27_csr, uniform_pm1, uniform_pm1_int52, stencil27_rhs_from_int52


def _random_csr(n, m, seed, density=0.2, intvals=True):
    rng = np.random.default_rng(seed)
    mask = rng.random((n, m)) < density
    rows, cols = np.nonzero(mask)
    vals = rng.integers(-9, 10, rows.size).astype(np.float64) if intvals else rng.standard_normal(rows.size)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return CSRHost(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), vals), mask, rows, cols, vals


def test_fma_chain_rational_emulation(orc):
    """Each step equals the correctly rounded a*x + acc (an fma), in CSR order."""
    A, _, _, _, _ = _random_csr(30, 30, 1, density=0.5, intvals=False)
    x = uniform_pm1(3, 30) * 1e3
    y = orc.spmv(A, x)
    for i in range(A.n):
        acc = 0.0
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc = fma_exact(A.val[k], x[A.col_idx[k]], acc)
        assert y[i] == acc


def test_row_order_matters_and_is_csr_order(orc):
    """Reversing a row's storage order changes the chain; the oracle follows storage order."""
    A = CSRHost(1, np.array([0, 3], np.int32), np.array([0, 1, 2], np.int32),
                np.array([1.0, 2.0 ** -53, 2.0 ** -53]))
    x = np.ones(3)
    # forward: fma(1,1,0)=1; fma(u,1,1)=1 (tie to even); again 1
    assert orc.spmv(A, x)[0] == 1.0
    B = CSRHost(1, np.array([0, 3], np.int32), np.array([2, 1, 0], np.int32),
                np.array([2.0 ** -53, 2.0 ** -53, 1.0]))
    # reversed: 2^-53, 2^-52, then 1 + 2^-52 exactly
    assert orc.spmv(B, x)[0] == 1.0 + 2.0 ** -52


def test_exact_integer_product_nonsymmetric(orc):
    """With integer values and x on a coarse dyadic grid every partial sum is
    exact, so y equals the integer matrix-vector product (catches a transposed
    operand: the matrix is not symmetric)."""
    A, mask, rows, cols, vals = _random_csr(200, 200, 5)
    K = np.random.default_rng(9).integers(-2 ** 20, 2 ** 20, 200)
    dense = np.zeros((200, 200), dtype=np.int64)
    dense[rows, cols] = vals.astype(np.int64)
    want = (dense @ K).astype(np.float64) * 2.0 ** -20
    assert np.array_equal(orc.spmv(A, K.astype(np.float64) * 2.0 ** -20), want)
    assert not np.array_equal(dense, dense.T)


@pytest.mark.parametrize("N", [1, 2, 5, 12])
def test_stencil27_ones_closed_form(orc, N):
    """A = 27 I - T(x)T(x)T, T = tridiag(1,1,1): (A 1)_i = 27 - prod_k c_k, with
    c_k in {1,2,3} the number of in-grid cells among {i_k-1, i_k, i_k+1}."""
    A = stencil27_csr(N)
    y = orc.spmv(A, np.ones(A.n))
    c = np.array([min(j + 1, N - 1) - max(j - 1, 0) + 1 for j in range(N)])
    want = 27.0 - (c[:, None, None] * c[None, :, None] * c[None, None, :]).reshape(-1)
    assert np.array_equal(y, want)
    assert A.nnz == (3 * N - 2) ** 3


def test_stencil27_rhs_generator_consistency(orc):
    """For x* on the 2^-20 grid the fma chain is exact, and equals the generator's
    integer-built right-hand side."""
    N = 10
    K = uniform_pm1_int52(4, N ** 3) >> 32  # |K| < 2^20
    A = stencil27_csr(N)
    y = orc.spmv(A, K.astype(np.float64) * 2.0 ** -20)
    b = stencil27_rhs_from_int52(N, K << 32)
    assert np.array_equal(y, b)


def test_empty_rows_give_plus_zero(orc):
    A = CSRHost(3, np.array([0, 0, 1, 1], np.int32), np.array([0], np.int32), np.array([-0.0]))
    y = orc.spmv(A, np.array([5.0, 1.0, 1.0]))
    assert [np.signbit(v) for v in y] == [False, False, False]
    assert np.all(y == 0.0)

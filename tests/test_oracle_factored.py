"""Pins of the oracle's PCG with a factored preconditioner M^-1 = G G^T + eps I
(the solve of the learned preconditioner): exact rational PCG on tiny
systems, bit-identity with the Jacobi path when G G^T = D^-1 exactly, the
pure eps I case, and the statuses."""

from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from rpcg_workloads import CSRHost, random_spd_csr, stencil7_varcoef_csr, uniform_pm1


def _csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return CSRHost(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def _dense(C):
    return sp.csr_matrix((C.val, C.col_idx, C.row_ptr), shape=(C.n, C.n)).toarray()


def rational_pcg(A, Minv, b, iters):
    """Textbook PCG in exact rationals; returns the tau history."""
    n = len(b)
    A = [[Fraction(v) for v in row] for row in A]
    Minv = [[Fraction(v) for v in row] for row in Minv]
    mv = lambda M, v: [sum(M[i][j] * v[j] for j in range(n)) for i in range(n)]
    dot = lambda u, v: sum(a * c for a, c in zip(u, v))
    x = [Fraction(0)] * n
    r = [Fraction(v) for v in b]
    z = mv(Minv, r)
    d = list(z)
    beta, tau = dot(z, r), dot(r, r)
    hist = [tau]
    for _ in range(iters):
        if tau == 0:
            break
        w = mv(A, d)
        rho = beta / dot(d, w)
        x = [xi + rho * di for xi, di in zip(x, d)]
        r = [ri - rho * wi for ri, wi in zip(r, w)]
        z = mv(Minv, r)
        bnew, tau = dot(z, r), dot(r, r)
        d = [zi + (bnew / beta) * di for zi, di in zip(z, d)]
        beta = bnew
        hist.append(tau)
    return hist, x


def test_transpose_csr(orc):
    A = random_spd_csr(23, 2)
    L = _csr(np.tril(_dense(A)) * 0.5)
    T = orc.transpose_csr(L)
    assert np.array_equal(_dense(T), _dense(L).T)
    for i in range(T.n):
        c = T.col_idx[T.row_ptr[i]:T.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rational_pcg(orc, seed):
    """n = 9 SPD system, G lower triangular with dyadic entries, eps = 2^-6:
    the oracle's tau history follows exact PCG to rounding level and its
    solution solves the system."""
    rng = np.random.default_rng(seed)
    n = 9
    B = rng.integers(-3, 4, size=(n, n)).astype(float)
    A = B.T @ B + n * np.eye(n)
    G = np.tril(rng.integers(-2, 3, size=(n, n)).astype(float) / 8.0, -1) + np.diag(rng.integers(1, 5, n) / 4.0)
    eps = 2.0 ** -6
    Minv = G @ G.T + eps * np.eye(n)
    b = rng.integers(-5, 6, n).astype(float)
    Ac, Gc = _csr(A), _csr(G)
    res = orc.pcg_factored(Ac, Gc, orc.transpose_csr(Gc), eps, b, tol=1e-12, maxit=40)
    assert res["status"] == 0 and res["iters"] <= n + 2
    hist, _ = rational_pcg(A, Minv, b, 4)
    for k in range(4):
        assert abs(res["hist"][k] - float(hist[k])) <= 1e-11 * float(hist[0])
    xs = np.linalg.solve(A, b)
    assert np.max(np.abs(res["x"] - xs)) <= 1e-10 * np.max(np.abs(xs))


def test_equals_jacobi_when_exact(orc):
    """Diagonal 16 (a power of 4): G = diag(1/4) gives G G^T = D^-1 exactly and
    every step of t = G^T r, s = G t is exact, so with eps = 0 the factored
    path reproduces the Jacobi path bit for bit (two independent code paths)."""
    N = 7
    A0 = stencil7_varcoef_csr(N, 4)
    val = np.where(A0.col_idx == np.repeat(np.arange(A0.n), np.diff(A0.row_ptr)), 16.0, -1.0)
    A = CSRHost(A0.n, A0.row_ptr, A0.col_idx, val)
    G = _csr(sp.identity(A.n) * 0.25)
    b = uniform_pm1(5, A.n)
    f = orc.pcg_factored(A, G, orc.transpose_csr(G), 0.0, b, tol=1e-12)
    j = orc.pcg(A, b, tol=1e-12)
    assert f["status"] == j["status"] == 0
    assert f["iters"] == j["iters"]
    assert np.array_equal(f["hist"], j["hist"])
    assert np.array_equal(f["x"], j["x"])


def test_pure_eps_is_scaled_cg(orc):
    """G = 0, eps = 2^-3: M^-1 = eps I, a constant multiple of the identity,
    leaves the CG iterates unchanged: exact unpreconditioned CG."""
    rng = np.random.default_rng(7)
    n = 8
    B = rng.integers(-3, 4, size=(n, n)).astype(float)
    A = B.T @ B + np.eye(n)
    b = rng.integers(-4, 5, n).astype(float)
    Z = CSRHost(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    res = orc.pcg_factored(_csr(A), Z, Z, 0.125, b, tol=1e-13, maxit=40)
    hist, xr = rational_pcg(A, np.eye(n), b, 3)
    for k in range(3):
        assert abs(res["hist"][k] - float(hist[k])) <= 1e-11 * float(hist[0])
    assert np.max(np.abs(res["x"] - np.linalg.solve(A, b))) < 1e-9


def test_statuses(orc):
    A = random_spd_csr(10, 3)
    G = _csr(np.eye(10))
    Gt = orc.transpose_csr(G)
    b = np.ones(10)
    r = orc.pcg_factored(A, G, Gt, 0.0, b, tol=1e-12, maxit=2)
    assert r["status"] == 1 and r["iters"] == 2
    r = orc.pcg_factored(A, G, Gt, 0.0, np.zeros(10))
    assert r["status"] == 0 and r["iters"] == 0
    bn = b.copy()
    bn[3] = np.inf
    assert orc.pcg_factored(A, G, Gt, 0.0, bn)["status"] == -6
    ind = _csr(np.array([[1.0, 3.0], [3.0, 1.0]]))
    I2 = _csr(np.eye(2))
    assert orc.pcg_factored(ind, I2, I2, 0.0, np.array([1.0, -1.0]))["status"] == -5

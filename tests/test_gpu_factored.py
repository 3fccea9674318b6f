"""GPU parity of rpcg_pcg_solve_factored (M^-1 = G G^T + eps I) against the
oracle: bit-identical iteration counts, tau histories and solutions in the
exact modes for any launch configuration, given G."""

import numpy as np
import pytest
import scipy.sparse as sp

from rpcg_workloads import CSRHost, grf_diffusion_csr, stencil7_varcoef_csr, uniform_pm1

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.context(0)
    return rpcg


def _eq(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return CSRHost(M.shape[0], M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def lower_factor(A, w=0.3):
    """A G with the lower-triangle pattern of A: scaled incomplete-Cholesky-like
    entries (positive diagonal, so G is nonsingular)."""
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    d = M.diagonal()
    s = 1.0 / np.sqrt(d)
    L = sp.tril(M, -1).tocoo()
    vals = -w * L.data * s[L.row] * s[L.col] * s[L.row]
    G = sp.coo_matrix((np.concatenate([s, vals]), (np.concatenate([np.arange(A.n), L.row]),
                                                   np.concatenate([np.arange(A.n), L.col]))), shape=(A.n, A.n))
    return _csr(G.tocsr())


def _solve(R, A, G, Gt, eps, b, mode, **kw):
    x, info = R.pcg_solve_factored(R.CSR.from_host(A), R.CSR.from_host(G), R.CSR.from_host(Gt), eps,
                                   torch.from_numpy(b).cuda(), mode=mode, **kw)
    return x.cpu().numpy(), info


@pytest.fixture(scope="module")
def fp(orc):
    A, _ = grf_diffusion_csr(14, 5)
    G = lower_factor(A)
    Gt = orc.transpose_csr(G)
    b = uniform_pm1(6, A.n)
    ref = orc.pcg_factored(A, G, Gt, 1e-6, b, tol=1e-10, maxit=3000)
    jac = orc.pcg(A, b, tol=1e-10, maxit=3000)
    assert ref["status"] == 0 and ref["iters"] < jac["iters"]
    return A, G, Gt, b, ref


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_factored_bitexact(R, fp, mode):
    A, G, Gt, b, ref = fp
    x, info = _solve(R, A, G, Gt, 1e-6, b, mode, tol=1e-10, maxit=3000)
    assert info["status"] == 0 and info["iterations"] == ref["iters"]
    assert _eq(info["hist"].numpy(), ref["hist"])
    assert _eq(x, ref["x"])


def test_factored_launch_invariance(R, fp):
    A, G, Gt, b, ref = fp
    for block, grid, sb, sg in ((64, 1, 64, 3), (1024, 7, 512, 64), (256, 999, 1024, 1), (128, 37, 64, 4096)):
        print(f"factored block={block} grid={grid} spmv={sb}x{sg}", flush=True)
        x, info = _solve(R, A, G, Gt, 1e-6, b, "exblas", tol=1e-10, maxit=3000, block_size=block, grid_size=grid,
                         spmv_block_size=sb, spmv_grid_size=sg)
        assert info["iterations"] == ref["iters"]
        assert _eq(info["hist"].numpy(), ref["hist"]) and _eq(x, ref["x"])


def test_factored_equals_jacobi_when_exact(R, orc):
    """Diagonal 16, G = diag(1/4), eps = 0: G G^T = D^-1 exactly, so the
    factored solve and the Jacobi solve agree bit for bit (on the GPU too)."""
    A0 = stencil7_varcoef_csr(9, 4)
    val = np.where(A0.col_idx == np.repeat(np.arange(A0.n), np.diff(A0.row_ptr)), 16.0, -1.0)
    A = CSRHost(A0.n, A0.row_ptr, A0.col_idx, val)
    G = _csr(sp.identity(A.n) * 0.25)
    b = uniform_pm1(9, A.n)
    xf, inf = _solve(R, A, G, G, 0.0, b, "exblas", tol=1e-12)
    xj, inj = R.pcg_solve(R.CSR.from_host(A), torch.from_numpy(b).cuda(), mode="exblas", tol=1e-12)
    ref = orc.pcg(A, b, tol=1e-12)
    assert inf["iterations"] == inj["iterations"] == ref["iters"]
    assert _eq(xf, xj.cpu().numpy()) and _eq(xf, ref["x"])


def test_factored_statuses(R, orc, fp):
    A, G, Gt, b, ref = fp
    x, info = _solve(R, A, G, Gt, 1e-6, b, "exblas", tol=1e-10, maxit=4)
    r = orc.pcg_factored(A, G, Gt, 1e-6, b, tol=1e-10, maxit=4)
    assert info["status"] == R.WARN_MAXIT and _eq(x, r["x"])
    x, info = _solve(R, A, G, Gt, 1e-6, np.zeros(A.n), "exblas")
    assert info["status"] == 0 and info["iterations"] == 0
    bn = b.copy()
    bn[2] = np.nan
    with pytest.raises(R.RpcgError) as e:
        _solve(R, A, G, Gt, 1e-6, bn, "exblas")
    assert e.value.status == R.ERR_NONFINITE
    badG = CSRHost(G.n, G.row_ptr, np.where(np.arange(G.col_idx.size) == 5, G.n + 3, G.col_idx).astype(np.int32), G.val)
    with pytest.raises(R.RpcgError) as e:
        _solve(R, A, badG, Gt, 1e-6, b, "exblas")
    assert e.value.status == R.ERR_INVALID

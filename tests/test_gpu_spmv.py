"""GPU parity of rpcg_spmv against the oracle's fma chains (bit-exact)."""

import numpy as np
import pytest

from rpcg_workloads import CSRHost, band_csr, stencil27_csr, stencil7_varcoef_csr, uniform_pm1

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.context(0)
    return rpcg


def _random_csr(n, seed, maxrow=40):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, maxrow, n)
    lens[rng.random(n) < 0.05] = 0
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(lens)
    col = rng.integers(0, n, rp[-1]).astype(np.int32)
    val = rng.standard_normal(rp[-1]) * np.exp2(rng.integers(-30, 30, rp[-1]))
    return CSRHost(n, rp.astype(np.int32), col, val)


@pytest.mark.parametrize("case", ["random", "stencil27", "stencil7", "empty_rows", "tiny"])
def test_spmv_bitexact(R, orc, case):
    print(f"spmv {case}", flush=True)
    if case == "random":
        A = _random_csr(10007, 1)
    elif case == "stencil27":
        A = stencil27_csr(19)
    elif case == "stencil7":
        A = stencil7_varcoef_csr(17, 3)
    elif case == "empty_rows":
        A = CSRHost(5, np.array([0, 0, 2, 2, 3, 3], np.int32), np.array([4, 0, 1], np.int32),
                    np.array([2.0, -0.0, 3.0]))
    else:
        A = CSRHost(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    x = uniform_pm1(5, A.n) * 1e3
    want = orc.spmv(A, x)
    y = R.spmv(R.CSR.from_host(A), torch.from_numpy(x).cuda())
    got = y.cpu().numpy()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_spmv_zero_rows(R):
    A = CSRHost(0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0))
    y = R.spmv(R.CSR.from_host(A), torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert y.numel() == 0


def test_spmv_rejects_aliasing_and_bad_dtype(R):
    A = stencil27_csr(4)
    Ad = R.CSR.from_host(A)
    x = torch.ones(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RpcgError):
        R.spmv(Ad, x, x)
    with pytest.raises(TypeError):
        R.spmv(Ad, x.float())


def _long_rows_csr(n, seed):
    """Mostly short rows, with rows of 256..300 entries, rows longer than the
    kernel's 4096-entry staging chunk (one of 9000 entries) and empty rows
    scattered in; unsorted columns, values spread over 60 binades."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 12, n)
    lens[rng.choice(n, 40, replace=False)] = rng.integers(256, 301, 40)
    lens[rng.choice(n, 3, replace=False)] = [4097, 5000, 9000]
    lens[rng.random(n) < 0.05] = 0
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(lens)
    col = rng.integers(0, n, rp[-1]).astype(np.int32)
    val = rng.standard_normal(rp[-1]) * np.exp2(rng.integers(-30, 30, rp[-1]))
    return CSRHost(n, rp.astype(np.int32), col, val)


@pytest.mark.parametrize("case", ["band100", "long_rows", "ragged_blocks", "one_long_row"])
def test_spmv_bitexact_long_and_ragged(R, orc, case):
    """Rows longer than 255 entries and longer than the staging chunk, a band
    of 201 entries per row (the paper's band transform, bandL = bandU = 100),
    and row counts that end inside a 512-row block."""
    print(f"spmv {case}", flush=True)
    if case == "band100":
        A = band_csr(100_003, 100)
    elif case == "long_rows":
        A = _long_rows_csr(20_011, 4)
    elif case == "ragged_blocks":
        A = _random_csr(512 * 7 + 301, 6, maxrow=70)
    else:
        n = 3
        A = CSRHost(n, np.array([0, 0, 20_000, 20_001], np.int32),
                    np.concatenate([np.arange(20_000) % n, [2]]).astype(np.int32),
                    np.random.default_rng(2).standard_normal(20_001))
    x = uniform_pm1(7, A.n) * 3.3
    want = orc.spmv(A, x)
    y = R.spmv(R.CSR.from_host(A), torch.from_numpy(x).cuda())
    assert np.array_equal(y.cpu().numpy().view(np.uint64), want.view(np.uint64))


@pytest.mark.slow
def test_spmv_full_size_stencil(R, orc):
    """The 27-point operator on 160^3 (109 M entries), every row bit-exact."""
    A = stencil27_csr(160)
    x = uniform_pm1(8, A.n)
    print("spmv 160^3", flush=True)
    want = orc.spmv(A, x)
    y = R.spmv(R.CSR.from_host(A), torch.from_numpy(x).cuda())
    assert np.array_equal(y.cpu().numpy().view(np.uint64), want.view(np.uint64))


def _prepared_case(case):
    if case == "random":  # unsorted columns: 32-bit column indices in the copy
        return _random_csr(10007, 21)
    if case == "stencil27":  # 16-bit column codes, odd widths
        return stencil27_csr(19)
    if case == "stencil7":
        return stencil7_varcoef_csr(17, 3)
    if case == "empty_rows":
        return CSRHost(5, np.array([0, 0, 2, 2, 3, 3], np.int32), np.array([4, 0, 1], np.int32),
                       np.array([2.0, -0.0, 3.0]))
    if case == "tiny":
        return CSRHost(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]))
    if case == "band100":
        return band_csr(30_011, 100)
    if case == "long_rows":  # rows of 256 or more entries: lengths from the copied row pointers
        return _long_rows_csr(20_011, 24)
    if case == "one_long_row":
        return CSRHost(3, np.array([0, 0, 20_000, 20_001], np.int32),
                       np.concatenate([np.arange(20_000) % 3, [2]]).astype(np.int32),
                       np.random.default_rng(3).standard_normal(20_001))
    raise ValueError(case)


@pytest.mark.parametrize("case", ["random", "stencil27", "stencil7", "empty_rows", "tiny", "band100", "long_rows",
                                  "one_long_row"])
def test_prepared_matrix_bitexact(R, orc, case):
    """A prepared (sliced-ELL) copy gives the oracle's fma chains bit for bit
    and the same bits as rpcg_spmv, on two vectors in a row, and still gives
    them after the CSR arrays it was made from are overwritten."""
    print(f"prepared spmv {case}", flush=True)
    A = _prepared_case(case)
    Ad = R.CSR.from_host(A)
    M = R.PreparedMatrix(Ad)
    outs = []
    for seed in (11, 12):
        x = uniform_pm1(seed, A.n) * 7.7
        xd = torch.from_numpy(x).cuda()
        want = orc.spmv(A, x)
        got = M.spmv(xd).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), seed
        assert np.array_equal(R.spmv(Ad, xd).cpu().numpy().view(np.uint64), got.view(np.uint64))
        outs.append((xd, got))
    Ad.val.fill_(0.0)
    Ad.col_idx.fill_(0)
    Ad.row_ptr.fill_(0)
    for xd, got in outs:
        assert np.array_equal(M.spmv(xd).cpu().numpy().view(np.uint64), got.view(np.uint64))
    M.close()


def test_prepared_matrix_errors(R):
    """Zero rows, aliasing, a malformed CSR (column out of range) and closing twice."""
    Z = R.PreparedMatrix(R.CSR.from_host(CSRHost(0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0))))
    assert Z.spmv(torch.zeros(0, dtype=torch.float64, device="cuda")).numel() == 0
    Z.close()
    A = stencil27_csr(4)
    M = R.PreparedMatrix(R.CSR.from_host(A))
    x = torch.ones(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RpcgError):
        M.spmv(x, x)
    M.close()
    M.close()
    bad = CSRHost(2, np.array([0, 1, 2], np.int32), np.array([0, 5], np.int32), np.array([1.0, 1.0]))
    with pytest.raises(R.RpcgError) as e:
        R.PreparedMatrix(R.CSR.from_host(bad))
    assert e.value.status == R.ERR_INVALID


@pytest.mark.slow
def test_prepared_matrix_full_size_stencil(R, orc):
    """The prepared copy of the 27-point 160^3 operator (odd widths, 16-bit
    codes): every row bit-identical to the oracle and to rpcg_spmv."""
    A = stencil27_csr(160)
    x = uniform_pm1(9, A.n)
    print("prepared spmv 160^3", flush=True)
    want = orc.spmv(A, x)
    Ad = R.CSR.from_host(A)
    xd = torch.from_numpy(x).cuda()
    M = R.PreparedMatrix(Ad)
    got = M.spmv(xd).cpu().numpy()
    M.close()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert np.array_equal(R.spmv(Ad, xd).cpu().numpy().view(np.uint64), got.view(np.uint64))

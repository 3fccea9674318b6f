"""GPU parity of rpcg_pcg_solve against the oracle.

Exact modes (exblas, fpe): iteration count, the whole tau history and the
solution are bit-identical to the oracle for every launch configuration.
Plain mode: converges, and its true relative residual is within 1e-12 of
the oracle's at the same iteration count."""

import math

import numpy as np
import pytest

from rpcg_workloads import (CSRHost, band_csr, random_spd_csr, stencil27_csr, stencil27_rhs_from_int52,
                            stencil7_varcoef_csr, uniform_pm1, uniform_pm1_int52)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.context(0)
    return rpcg


def stencil_problem(N, seed):
    A = stencil27_csr(N)
    K = uniform_pm1_int52(seed, A.n)
    return A, stencil27_rhs_from_int52(N, K), K * 2.0 ** -52


@pytest.fixture(scope="module")
def w1(orc):
    """The 32^3 parity workload: 27-point operator, b = A x*, x* ~ U[-1,1) (seed 1)."""
    A, b, xs = stencil_problem(32, 1)
    ref = orc.pcg(A, b, tol=1e-8, maxit=2000)
    assert ref["status"] == 0
    return A, b, xs, ref


def _eq(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _solve(R, A, b, mode, **kw):
    Ad = R.CSR.from_host(A)
    x, info = R.pcg_solve(Ad, torch.from_numpy(b).cuda(), mode=mode, **kw)
    return x.cpu().numpy(), info


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_w1_bitexact(R, w1, mode):
    A, b, xs, ref = w1
    print(f"pcg 32^3 {mode}", flush=True)
    x, info = _solve(R, A, b, mode)
    assert info["status"] == 0
    assert info["iterations"] == ref["iters"]
    assert _eq(info["hist"].numpy(), ref["hist"])
    assert _eq(x, ref["x"])
    if mode == "fpe":
        assert info["fpe_escapes"] == 0 and info["fallbacks"] == 0


LAUNCH = [(64, 1), (64, 37), (128, 256), (256, 0), (512, 13), (1024, 64), (256, 2048)]
SPMV_LAUNCH = [(256, 0), (64, 3), (1024, 7), (128, 999), (512, 64), (256, 1), (64, 4096)]


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_w1_launch_config_invariance(R, w1, mode):
    A, b, xs, ref = w1
    for (block, grid), (sb, sg) in zip(LAUNCH, SPMV_LAUNCH):
        for p in ((3, 4, 8) if mode == "fpe" else (1, 4)):
            narrow = (block + grid + p) % 2
            print(f"pcg 32^3 {mode} block={block} grid={grid} spmv={sb}x{sg} p={p} no_col16={narrow}", flush=True)
            x, info = _solve(R, A, b, mode, block_size=block, grid_size=grid, fpe_size=p,
                             spmv_block_size=sb, spmv_grid_size=sg, no_col16=narrow)
            assert info["iterations"] == ref["iters"], (block, grid, p)
            assert _eq(info["hist"].numpy(), ref["hist"]), (block, grid, p)
            assert _eq(x, ref["x"]), (block, grid, p)


def test_w1_plain_within_tolerance(R, orc, w1):
    """Plain fp64 (the paper's Regular variant): converges; at the oracle's
    iteration count its true relative residual is within 1e-12 of the oracle's."""
    A, b, xs, ref = w1
    x, info = _solve(R, A, b, "plain")
    assert info["status"] == 0
    assert abs(info["iterations"] - ref["iters"]) <= 2
    x2, info2 = _solve(R, A, b, "plain", maxit=ref["iters"])
    rr_plain = orc.relres_true(A, b, x2)
    rr_orc = orc.relres_true(A, b, ref["x"])
    assert abs(rr_plain - rr_orc) <= 1e-12
    h = info["hist"].numpy()
    L = min(len(h), len(ref["hist"]))
    rel = np.abs(h[:L] / ref["hist"][:L] - 1)
    print("plain vs exact tau, max relative deviation", rel.max())
    assert rel.max() < 1e-6


def test_paper_rhs_ones(R, orc):
    """Section 5.1: b = A * ones, x0 = 0, tolerance 1e-8."""
    A = stencil27_csr(24)
    b = orc.spmv(A, np.ones(A.n))
    ref = orc.pcg(A, b, tol=1e-8)
    for mode in ("exblas", "fpe"):
        x, info = _solve(R, A, b, mode)
        assert info["iterations"] == ref["iters"]
        assert _eq(x, ref["x"])


@pytest.mark.parametrize("case", ["spd_small", "stencil7", "ragged_n", "nonzero_x0"])
def test_other_systems_bitexact(R, orc, case):
    x0 = None
    if case == "spd_small":
        A = random_spd_csr(37, 4)
        b = uniform_pm1(3, A.n)
    elif case == "stencil7":
        A = stencil7_varcoef_csr(13, 8)
        b = uniform_pm1(4, A.n)
    elif case == "ragged_n":
        A, b, _ = stencil_problem(11, 6)  # n = 1331, not a multiple of 64
    else:
        A, b, _ = stencil_problem(9, 2)
        x0 = uniform_pm1(9, A.n)
    ref = orc.pcg(A, b, x0=x0, tol=1e-10, maxit=3000)
    for mode in ("exblas", "fpe"):
        Ad = R.CSR.from_host(A)
        x, info = R.pcg_solve(Ad, torch.from_numpy(b).cuda(), None if x0 is None else torch.from_numpy(x0).cuda(),
                              mode=mode, tol=1e-10, maxit=3000)
        assert info["status"] == ref["status"]
        assert info["iterations"] == ref["iters"], (case, mode)
        assert _eq(info["hist"].numpy(), ref["hist"])
        assert _eq(x.cpu().numpy(), ref["x"])


def test_permuted_matrix_wide_columns(R, orc):
    """A symmetric permutation P A P^T of the 27-point operator (still SPD) moves
    entries far from the diagonal (|col - row| > 32767), so the solver keeps
    32-bit column indices; results still match the oracle bit for bit."""
    A0 = stencil27_csr(35)
    n = A0.n
    perm = np.random.default_rng(3).permutation(n)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(A0.row_ptr))
    nr, nc = inv[rows], inv[A0.col_idx]
    order = np.lexsort((nc, nr))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, nr + 1, 1)
    A = CSRHost(n, np.cumsum(rp).astype(np.int32), nc[order].astype(np.int32), A0.val[order])
    assert np.max(np.abs(A.col_idx.astype(np.int64) - np.repeat(np.arange(n), np.diff(A.row_ptr)))) > 32767
    b = uniform_pm1(8, n)
    ref = orc.pcg(A, b, tol=1e-8)
    for mode in ("exblas", "fpe"):
        x, info = _solve(R, A, b, mode)
        assert info["iterations"] == ref["iters"]
        assert _eq(info["hist"].numpy(), ref["hist"])
        assert _eq(x, ref["x"])


@pytest.mark.parametrize("w", [0, 1, 7, 13, 14, 20])
def test_band_row_lengths_bitexact(R, orc, w):
    """Rows of 2w + 1 entries (shorter at the band's ends): odd widths of the
    solver's sliced-ELL copy, whose last entry sits in a single-entry column,
    read alone (w = 0), after a partial batch of pairs (1, 13, 20) or right
    after full batches (7, 14). Bit-identical to the oracle in both exact
    modes."""
    A = band_csr(300 + w, w)
    b = uniform_pm1(40 + w, A.n)
    ref = orc.pcg(A, b, tol=1e-10, maxit=2000)
    for mode in ("exblas", "fpe"):
        x, info = _solve(R, A, b, mode, tol=1e-10, maxit=2000)
        assert info["status"] == ref["status"]
        assert info["iterations"] == ref["iters"], (w, mode)
        assert _eq(info["hist"].numpy(), ref["hist"])
        assert _eq(x, ref["x"])


def test_status_cases(R, orc):
    A = stencil27_csr(6)
    b = orc.spmv(A, np.ones(A.n))
    # maxit
    for mode in ("exblas", "fpe", "plain"):
        x, info = _solve(R, A, b, mode, maxit=3)
        assert info["status"] == R.WARN_MAXIT and info["iterations"] == 3
    ref = orc.pcg(A, b, maxit=3)
    x, info = _solve(R, A, b, "exblas", maxit=3)
    assert _eq(x, ref["x"]) and _eq(info["hist"].numpy(), ref["hist"])
    # zero right-hand side: zero iterations
    x, info = _solve(R, A, np.zeros(A.n), "exblas")
    assert info["status"] == 0 and info["iterations"] == 0 and not x.any()
    # maxit = 0
    x, info = _solve(R, A, b, "exblas", maxit=0)
    assert info["status"] == R.WARN_MAXIT and info["iterations"] == 0
    # negative diagonal
    bad = CSRHost(A.n, A.row_ptr, A.col_idx, np.where(A.val == 26.0, -26.0, A.val))
    with pytest.raises(R.RpcgError) as e:
        _solve(R, bad, b, "exblas")
    assert e.value.status == R.ERR_NOT_SPD
    # missing diagonal
    nodiag = CSRHost(2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    with pytest.raises(R.RpcgError) as e:
        _solve(R, nodiag, np.ones(2), "exblas")
    assert e.value.status == R.ERR_NOT_SPD
    # non-finite right-hand side
    bn = b.copy()
    bn[3] = np.nan
    with pytest.raises(R.RpcgError) as e:
        _solve(R, A, bn, "exblas")
    assert e.value.status == R.ERR_NONFINITE
    # indefinite: breakdown
    ind = CSRHost(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([1.0, 3.0, 3.0, 1.0]))
    with pytest.raises(R.RpcgError) as e:
        _solve(R, ind, np.array([1.0, -1.0]), "exblas")
    assert e.value.status == R.ERR_BREAKDOWN


def test_empty_system(R):
    A = CSRHost(0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0))
    x, info = _solve(R, A, np.zeros(0), "exblas")
    assert info["status"] == 0 and info["iterations"] == 0


def test_repeat_solves_identical(R, w1):
    """Back-to-back solves (reused workspace, tickets and state) give the same bits."""
    A, b, xs, ref = w1
    xa, ia = _solve(R, A, b, "exblas")
    xb, ib = _solve(R, A, b, "exblas")
    assert _eq(xa, xb) and _eq(ia["hist"].numpy(), ib["hist"].numpy())


def test_timing_fields(R, w1):
    A, b, xs, ref = w1
    x, info = _solve(R, A, b, "exblas", timing=1)
    assert info["k_launches"] == ref["iters"]
    assert info["k_spmv_dot_ms"] > 0 and info["k_update_ms"] > 0 and info["k_direction_ms"] > 0
    assert _eq(x, ref["x"])
    # timing = 2 brackets only the SpMV+dot kernel; timing = k + 1 only that
    # of every k-th iteration; other values are rejected
    x, info = _solve(R, A, b, "exblas", timing=2)
    assert info["k_launches"] == ref["iters"]
    assert info["k_spmv_dot_ms"] > 0 and info["k_update_ms"] == 0 and info["k_direction_ms"] == 0
    assert _eq(x, ref["x"])
    x, info = _solve(R, A, b, "exblas", timing=5)
    assert info["k_launches"] == (ref["iters"] + 3) // 4
    assert info["k_spmv_dot_ms"] > 0 and info["k_update_ms"] == 0 and info["k_direction_ms"] == 0
    assert _eq(x, ref["x"])
    for bad in (-1, 66):
        with pytest.raises(R.RpcgError):
            _solve(R, A, b, "exblas", timing=bad)


def test_64_cube_full_solve_bitexact(R, orc):
    """A full solve to 1e-8 at 64^3 (n = 262,144: many workgroups and slots in
    every kernel), bit-identical to the oracle in both exact modes, with the
    default launch shapes and with grids larger than the chip holds at once."""
    A, b, _ = stencil_problem(64, 3)
    print("pcg 64^3 oracle", flush=True)
    ref = orc.pcg(A, b, tol=1e-8, maxit=2000)
    assert ref["status"] == 0
    for mode in ("exblas", "fpe"):
        for grid, block, sg in ((0, 0, 0), (2048, 256, 4096)):
            print(f"pcg 64^3 {mode} grid={grid} block={block} spmv_grid={sg}", flush=True)
            x, info = _solve(R, A, b, mode, grid_size=grid, block_size=block, spmv_grid_size=sg)
            assert info["status"] == 0 and info["iterations"] == ref["iters"], (mode, grid)
            assert _eq(info["hist"].numpy(), ref["hist"]), (mode, grid)
            assert _eq(x, ref["x"]), (mode, grid)


@pytest.mark.slow
def test_160_cube_first_iterations_bitexact(R, orc):
    """Full-size operator (160^3, the bench configuration): the first three
    iterations match the oracle bit for bit; the full solve converges with
    the tau history consistent with the stopping rule."""
    A, b, xs = stencil_problem(160, 2)
    print("pcg 160^3 maxit=3", flush=True)
    ref = orc.pcg(A, b, tol=1e-8, maxit=3)
    x, info = _solve(R, A, b, "exblas", maxit=3)
    assert _eq(info["hist"].numpy(), ref["hist"])
    assert _eq(x, ref["x"])
    # vector-kernel grids larger than the chip holds at once: workgroups that
    # start after the stopping test has set the done flag must find nothing
    # of the last iteration left to do
    for grid, block in ((1024, 512), (512, 1024), (2048, 256), (4096, 256)):
        for mode in ("exblas", "fpe"):
            print(f"pcg 160^3 maxit=3 {mode} grid={grid} block={block}", flush=True)
            x, info = _solve(R, A, b, mode, maxit=3, grid_size=grid, block_size=block)
            assert _eq(info["hist"].numpy(), ref["hist"]), (mode, grid, block)
            assert _eq(x, ref["x"]), (mode, grid, block)
    print("pcg 160^3 full", flush=True)
    x, info = _solve(R, A, b, "exblas")
    assert info["status"] == 0
    h = info["hist"].numpy()
    assert h[-1] <= info["threshold"] < h[-2]
    idx = np.random.default_rng(0).choice(A.n, 2000, replace=False)
    assert np.max(np.abs(x[idx] - xs[idx])) < 1e-5


@pytest.fixture(scope="module")
def w2(orc):
    """The bench configuration: 27-point operator on 160^3 (n = 4,096,000,
    nnz = 109,215,352), b = A x*, x* ~ U[-1,1) (seed 2), tol 1e-8; the
    oracle's full solve, computed once for the module."""
    A, b, xs = stencil_problem(160, 2)
    print("pcg 160^3 oracle full solve", flush=True)
    ref = orc.pcg(A, b, tol=1e-8, maxit=2000)
    assert ref["status"] == 0
    return A, b, xs, ref


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_160_cube_full_solve_bitexact(R, w2):
    """Section 5.3 / Table 3: the exact variants reproduce the reference at
    every iteration. Here: the whole bench solve (iteration count, every
    tau of the history and every bit of x) equals the oracle in both exact
    modes, with the default launch shapes and with grids larger than the chip
    holds at once."""
    A, b, xs, ref = w2
    Ad = R.CSR.from_host(A)
    bd = torch.from_numpy(b).cuda()
    for mode in ("exblas", "fpe"):
        for grid, block, sg in ((0, 0, 0), (1024, 512, 4096)):
            print(f"pcg 160^3 full {mode} grid={grid} block={block} spmv_grid={sg}", flush=True)
            x, info = R.pcg_solve(Ad, bd, mode=mode, grid_size=grid, block_size=block, spmv_grid_size=sg)
            assert info["status"] == 0 and info["iterations"] == ref["iters"], (mode, grid)
            assert _eq(info["hist"].numpy(), ref["hist"]), (mode, grid)
            assert _eq(x.cpu().numpy(), ref["x"]), (mode, grid)
            if mode == "fpe":
                assert info["fpe_escapes"] == 0


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_160_cube_plain_within_tolerance(R, orc, w2):
    """Plain fp64 at the bench configuration: converges, and at the oracle's
    iteration count its true relative residual (exact row sums) is within
    1e-12 of the oracle's."""
    A, b, xs, ref = w2
    Ad = R.CSR.from_host(A)
    bd = torch.from_numpy(b).cuda()
    print("pcg 160^3 plain", flush=True)
    x, info = R.pcg_solve(Ad, bd, mode="plain")
    assert info["status"] == 0 and abs(info["iterations"] - ref["iters"]) <= 2
    x2, info2 = R.pcg_solve(Ad, bd, mode="plain", maxit=ref["iters"])
    print("pcg 160^3 plain true residuals", flush=True)
    rr_plain = orc.relres_true(A, b, x2.cpu().numpy())
    rr_orc = orc.relres_true(A, b, ref["x"])
    print("160^3 relres plain", rr_plain, "oracle", rr_orc, flush=True)
    assert abs(rr_plain - rr_orc) <= 1e-12
    h = info["hist"].numpy()
    L = min(len(h), len(ref["hist"]))
    assert np.max(np.abs(h[:L] / ref["hist"][:L] - 1)) < 1e-6

"""GPU parity of the binary32 Jacobi-PCG (rpcg_pcg_solve_f32) and of the
mixed-precision refinement (rpcg_ir_solve) against the oracle.

Exact modes: iteration counts, the residual histories and the solutions are
bit-identical to the oracle for every launch configuration. At the full
256^3 size the first inner iterations are compared bit for bit and the
refinement is checked through properties that hold at any size."""

import numpy as np
import pytest

from rpcg_workloads import (CSRHost, random_spd_csr, stencil27_csr, stencil27_rhs_from_int52,
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


def _bits_eq(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.dtype != b.dtype or a.shape != b.shape:
        return False
    return np.array_equal(a.view(np.uint8), b.view(np.uint8))


def stencil_problem(N, seed):
    A = stencil27_csr(N)
    K = uniform_pm1_int52(seed, A.n)
    return A, stencil27_rhs_from_int52(N, K), K * 2.0 ** -52


def _f32_problem(N, seed):
    """27-point operator (exact in binary32) with b = RN32 of a scaled A x*."""
    A, b, _ = stencil_problem(N, seed)
    return A, (b / 64.0).astype(np.float32)


def _solve32(R, A, b32, mode, **kw):
    Ad = R.CSR.from_host(A, dtype=torch.float32)
    x0 = kw.pop("x0", None)
    x, info = R.pcg_solve_f32(Ad, torch.from_numpy(b32).cuda(),
                              None if x0 is None else torch.from_numpy(x0).cuda(), mode=mode, **kw)
    return x.cpu().numpy(), info


@pytest.fixture(scope="module")
def f1(orc):
    A, b32 = _f32_problem(32, 1)
    ref = orc.pcg_f32(A, b32, tol=1e-6, maxit=2000)
    assert ref["status"] == 0
    return A, b32, ref


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_f32_bitexact(R, f1, mode):
    A, b32, ref = f1
    print(f"pcg_f32 32^3 {mode}", flush=True)
    x, info = _solve32(R, A, b32, mode, tol=1e-6)
    assert info["status"] == 0
    assert info["iterations"] == ref["iters"]
    assert _bits_eq(info["hist"].numpy(), ref["hist"])
    assert _bits_eq(x, ref["x"])


LAUNCH = [(64, 1), (128, 256), (512, 13), (1024, 64), (256, 2048)]
SPMV_LAUNCH = [(64, 3), (1024, 7), (512, 64), (256, 1), (64, 4096)]


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_f32_launch_config_invariance(R, f1, mode):
    A, b32, ref = f1
    for (block, grid), (sb, sg) in zip(LAUNCH, SPMV_LAUNCH):
        p = 2 if mode == "exblas" else 6
        narrow = (block + grid) % 2
        print(f"pcg_f32 32^3 {mode} block={block} grid={grid} spmv={sb}x{sg} p={p} no_col16={narrow}", flush=True)
        x, info = _solve32(R, A, b32, mode, tol=1e-6, block_size=block, grid_size=grid, fpe_size=p,
                           spmv_block_size=sb, spmv_grid_size=sg, no_col16=narrow)
        assert info["iterations"] == ref["iters"], (block, grid)
        assert _bits_eq(info["hist"].numpy(), ref["hist"]), (block, grid)
        assert _bits_eq(x, ref["x"]), (block, grid)


def test_f32_160_cube_large_grids(R, orc):
    """Binary32 iteration at 160^3, first three iterations against the oracle,
    with vector-kernel grids larger than the chip holds at once (workgroups
    that start after the stopping test has set the done flag)."""
    A, b32 = _f32_problem(160, 2)
    ref = orc.pcg_f32(A, b32, tol=1e-6, maxit=3)
    for grid, block in ((0, 0), (1024, 512), (4096, 256)):
        for mode in ("exblas", "fpe"):
            print(f"pcg_f32 160^3 maxit=3 {mode} grid={grid} block={block}", flush=True)
            x, info = _solve32(R, A, b32, mode, tol=1e-6, maxit=3, grid_size=grid, block_size=block)
            assert _bits_eq(info["hist"].numpy(), ref["hist"]), (mode, grid, block)
            assert _bits_eq(x, ref["x"]), (mode, grid, block)


@pytest.mark.parametrize("case", ["spd_small", "stencil7", "ragged_n", "nonzero_x0"])
def test_f32_other_systems(R, orc, case):
    x0 = None
    if case == "spd_small":
        A = random_spd_csr(37, 4)
        b32 = uniform_pm1(3, A.n).astype(np.float32)
    elif case == "stencil7":
        A = stencil7_varcoef_csr(13, 8)  # values rounded to binary32 on both sides
        b32 = uniform_pm1(4, A.n).astype(np.float32)
    elif case == "ragged_n":
        A, b32 = _f32_problem(11, 6)
    else:
        A, b32 = _f32_problem(9, 2)
        x0 = uniform_pm1(9, A.n).astype(np.float32)
    ref = orc.pcg_f32(A, b32, x0=x0, tol=1e-5, maxit=3000)
    for mode in ("exblas", "fpe"):
        print(f"pcg_f32 {case} {mode}", flush=True)
        x, info = _solve32(R, A, b32, mode, tol=1e-5, maxit=3000, x0=x0)
        assert info["status"] == ref["status"]
        assert info["iterations"] == ref["iters"], (case, mode)
        assert _bits_eq(info["hist"].numpy(), ref["hist"])
        assert _bits_eq(x, ref["x"])


def test_f32_status_cases(R, orc):
    A, b32 = _f32_problem(6, 3)
    x, info = _solve32(R, A, b32, "exblas", maxit=3, tol=1e-7)
    assert info["status"] == R.WARN_MAXIT and info["iterations"] == 3
    ref = orc.pcg_f32(A, b32, tol=1e-7, maxit=3)
    assert _bits_eq(x, ref["x"])
    x, info = _solve32(R, A, np.zeros(A.n, np.float32), "exblas")
    assert info["status"] == 0 and info["iterations"] == 0 and not x.any()
    bad = CSRHost(A.n, A.row_ptr, A.col_idx, np.where(A.val == 26.0, -26.0, A.val))
    with pytest.raises(R.RpcgError) as e:
        _solve32(R, bad, b32, "exblas")
    assert e.value.status == R.ERR_NOT_SPD
    bn = b32.copy()
    bn[5] = np.inf
    with pytest.raises(R.RpcgError) as e:
        _solve32(R, A, bn, "exblas")
    assert e.value.status == R.ERR_NONFINITE


# ---------------------------------------------------------------------------
# refinement

def _ir(R, A, b, mode="exblas", x0=None, **kw):
    Ad = R.CSR.from_host(A)
    x, info = R.ir_solve(Ad, torch.from_numpy(b).cuda(), None if x0 is None else torch.from_numpy(x0).cuda(),
                         mode=mode, **kw)
    return x.cpu().numpy(), info


def _check_ir(res, x, info):
    assert info["status"] == res["status"]
    assert info["outer"] == res["outer"]
    assert info["inner_iterations"] == res["inner"]
    assert _bits_eq(info["rr_hist"].numpy(), res["hist"])
    assert _bits_eq(x, res["x"])


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_ir_bitexact(R, orc, mode):
    A, b, xs = stencil_problem(20, 7)
    res = orc.ir(A, b, tol=1e-10, tol_in=1e-4)
    assert res["status"] == 0 and res["outer"] >= 2
    print(f"ir 20^3 {mode}", flush=True)
    x, info = _ir(R, A, b, mode, tol=1e-10, maxit=50)
    _check_ir(res, x, info)
    assert orc.relres_true(A, b, x) <= 1e-10


def test_ir_fixed_inner_tolerance(R, orc):
    """adaptive_inner = 0: every inner solve to tol_inner, as the oracle's
    fixed-tolerance refinement; it overshoots the target on the last step."""
    A, b, xs = stencil_problem(20, 7)
    res = orc.ir(A, b, tol=1e-10, tol_in=1e-4, adaptive=False)
    ad = orc.ir(A, b, tol=1e-10, tol_in=1e-4, adaptive=True)
    assert res["inner"] > ad["inner"]
    print("ir 20^3 fixed inner tolerance", flush=True)
    x, info = _ir(R, A, b, tol=1e-10, maxit=50, adaptive_inner=False)
    _check_ir(res, x, info)


def test_ir_error_vs_fp64_oracle(R, orc):
    """The refinement's solution against the binary64 exact-dot PCG solution of
    the oracle (same tolerance): the stated error is at the 1e-9 level."""
    A, b, xs = stencil_problem(24, 3)
    ref = orc.pcg(A, b, tol=1e-10, maxit=3000)
    x, info = _ir(R, A, b, tol=1e-10)
    assert info["status"] == 0
    err = np.max(np.abs(x - ref["x"])) / np.max(np.abs(ref["x"]))
    print("ir 24^3: max relative deviation from the fp64 oracle solution", err, flush=True)
    assert err < 1e-8
    assert orc.relres_true(A, b, x) <= 1e-10


def test_ir_launch_config_invariance(R, orc):
    A, b, _ = stencil_problem(13, 4)  # n = 2197: ragged last slice
    res = orc.ir(A, b, tol=1e-11, tol_in=1e-3)
    for (block, grid), (sb, sg) in zip(LAUNCH, SPMV_LAUNCH):
        print(f"ir 13^3 block={block} grid={grid} spmv={sb}x{sg}", flush=True)
        x, info = _ir(R, A, b, tol=1e-11, tol_inner=1e-3, block_size=block, grid_size=grid,
                      spmv_block_size=sb, spmv_grid_size=sg, no_col16=(block // 64) % 2)
        _check_ir(res, x, info)


def test_ir_binary64_values(R, orc):
    """Values not representable in binary32: inner solves on their rounding,
    outer residual on the binary64 values; bit-identical to the oracle."""
    A0 = stencil27_csr(10)
    A = CSRHost(A0.n, A0.row_ptr, A0.col_idx, A0.val / 3.0 + np.where(A0.val > 0, 0.1, 0.0))
    b = orc.spmv(A, uniform_pm1(12, A.n))
    res = orc.ir(A, b, tol=1e-12, tol_in=1e-4)
    assert res["status"] == 0
    for mode in ("exblas", "fpe"):
        print(f"ir 10^3 non-binary32 values {mode}", flush=True)
        x, info = _ir(R, A, b, mode, tol=1e-12)
        _check_ir(res, x, info)


@pytest.mark.parametrize("case", ["spd_small", "stencil7", "nonzero_x0", "outer_maxit", "zero_rhs",
                                  "inner_maxit"])
def test_ir_other_cases(R, orc, case):
    x0 = None
    kw = dict(tol=1e-10, maxit_out=50, tol_in=1e-4, maxit_in=2000)
    if case == "spd_small":
        A = random_spd_csr(41, 5)
        b = uniform_pm1(13, A.n)
    elif case == "stencil7":
        A = stencil7_varcoef_csr(12, 9)
        b = uniform_pm1(14, A.n)
    elif case == "nonzero_x0":
        A, b, _ = stencil_problem(9, 5)
        x0 = uniform_pm1(15, A.n)
    elif case == "outer_maxit":
        A, b, _ = stencil_problem(9, 6)
        kw["maxit_out"] = 1
    elif case == "zero_rhs":
        A = stencil27_csr(5)
        b = np.zeros(A.n)
    else:
        A, b, _ = stencil_problem(9, 8)
        kw["maxit_in"] = 4  # every inner solve stops at its maxit; accepted
    res = orc.ir(A, b, x0=x0, **kw)
    print(f"ir {case}: oracle status {res['status']} outer {res['outer']} inner {res['inner']}", flush=True)
    x, info = _ir(R, A, b, x0=x0, tol=kw["tol"], maxit=kw["maxit_out"], tol_inner=kw["tol_in"],
                  maxit_inner=kw["maxit_in"], raise_on_error=False)
    _check_ir(res, x, info)
    if case == "outer_maxit":
        assert info["status"] == R.WARN_MAXIT and info["outer"] == 1
    if case == "zero_rhs":
        assert info["outer"] == 0 and not x.any()


def test_ir_errors(R, orc):
    A = stencil27_csr(6)
    bad = CSRHost(A.n, A.row_ptr, A.col_idx, np.where(A.val == 26.0, -26.0, A.val))
    b = np.ones(A.n)
    with pytest.raises(R.RpcgError) as e:
        _ir(R, bad, b)
    assert e.value.status == R.ERR_NOT_SPD
    bn = b.copy()
    bn[7] = np.nan
    with pytest.raises(R.RpcgError) as e:
        _ir(R, A, bn)
    assert e.value.status == R.ERR_NONFINITE
    assert orc.ir(A, bn)["status"] == R.ERR_NONFINITE


def test_ir_timing_fields(R):
    A, b, _ = stencil_problem(16, 2)
    x, info = _ir(R, A, b, timing=1)
    assert info["status"] == 0
    assert info["k_launches"] == info["inner_iterations"]
    assert info["k_residual_ms"] > 0 and info["k_spmv_dot_ms"] > 0
    assert info["total_ms"] >= info["inner_ms"]


@pytest.mark.slow
def test_256_cube_refinement(R, orc):
    """Full-size mixed-precision configuration (256^3): the first two
    iterations of the first inner binary32 solve match the oracle bit for bit;
    the whole refinement reaches 1e-10 with a monotone <r,r> history, a true
    binary64 residual (numpy, error far below the bound) under 1e-10 and a
    solution within 1e-8 of the generating x*."""
    A, b, xs = stencil_problem(256, 2)
    rr = orc.exdot(b, b)
    s = orc.ir_scale(rr)
    rf = np.ldexp(b, -s).astype(np.float32)
    print("pcg_f32 256^3 maxit=2", flush=True)
    ref = orc.pcg_f32(A, rf, tol=1e-4, maxit=2)
    x, info = _solve32(R, A, rf, "exblas", tol=1e-4, maxit=2)
    assert _bits_eq(info["hist"].numpy(), ref["hist"])
    assert _bits_eq(x, ref["x"])
    print("ir 256^3 full", flush=True)
    Ad = R.CSR.from_host(A)
    xd, info = R.ir_solve(Ad, torch.from_numpy(b).cuda(), tol=1e-10)
    assert info["status"] == 0
    h = info["rr_hist"].numpy()
    assert np.all(h[1:] < h[:-1]) and h[-1] <= info["threshold"]
    xg = xd.cpu().numpy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    Ax = np.bincount(rows, weights=A.val * xg[A.col_idx], minlength=A.n)
    rel = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    print("ir 256^3: outer", info["outer"], "inner", info["inner_iterations"], "relres", rel, flush=True)
    assert rel < 1.01e-10
    assert np.max(np.abs(xg - xs)) < 1e-8

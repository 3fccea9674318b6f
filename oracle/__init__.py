"""CPU oracle for the reproducible Jacobi-PCG hot path (ctypes binding).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the library. It shares no code with the
GPU path. The C source states what each function computes and which part of
the paper it follows.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpcg_oracle.c")
_LIB = os.path.join(_HERE, "librpcg_oracle.so")

OK, WARN_MAXIT, ERR_INVALID, ERR_NOT_SPD, ERR_BREAKDOWN, ERR_NONFINITE = 0, 1, -1, -4, -5, -6

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: no contraction of a*b+c, hardware fma for fma()."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-mfma", "-fopenmp", "-fPIC", "-shared",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.rpcg_oracle_exdot.restype = ctypes.c_double
        L.rpcg_oracle_exdot.argtypes = [ctypes.c_int64, P, P]
        L.rpcg_oracle_exact_limbs.restype = ctypes.c_int
        L.rpcg_oracle_exdot_exact.restype = ctypes.c_int
        L.rpcg_oracle_exdot_exact.argtypes = [ctypes.c_int64, P, P, P, P]
        L.rpcg_oracle_round_limbs.restype = ctypes.c_double
        L.rpcg_oracle_round_limbs.argtypes = [P, ctypes.c_int]
        L.rpcg_oracle_spmv.restype = None
        L.rpcg_oracle_spmv.argtypes = [ctypes.c_int32, P, P, P, P, P]
        L.rpcg_oracle_true_residual.restype = None
        L.rpcg_oracle_true_residual.argtypes = [ctypes.c_int32, P, P, P, P, P, P]
        L.rpcg_oracle_pcg.restype = ctypes.c_int
        L.rpcg_oracle_pcg.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                      P, P, P, P, P]
        L.rpcg_oracle_exdot_f32.restype = ctypes.c_float
        L.rpcg_oracle_exdot_f32.argtypes = [ctypes.c_int64, P, P]
        L.rpcg_oracle_spmv_f32.restype = None
        L.rpcg_oracle_spmv_f32.argtypes = [ctypes.c_int32, P, P, P, P, P]
        L.rpcg_oracle_pcg_f32.restype = ctypes.c_int
        L.rpcg_oracle_pcg_f32.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_double, ctypes.c_int32, P, P,
                                          P, P, P, P]
        L.rpcg_oracle_ir_scale.restype = ctypes.c_int
        L.rpcg_oracle_ir_scale.argtypes = [ctypes.c_double]
        L.rpcg_oracle_pcg_factored.restype = ctypes.c_int
        L.rpcg_oracle_pcg_factored.argtypes = [ctypes.c_int32, P, P, P, P, P, P, P, P, P, ctypes.c_double, P, P,
                                               ctypes.c_double, ctypes.c_int32, P, P, P, P, P]
        L.rpcg_oracle_ir.restype = ctypes.c_int
        L.rpcg_oracle_ir.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P, P, P, P]
        L.rpcg_oracle_set_threads.restype = ctypes.c_int
        L.rpcg_oracle_set_threads.argtypes = [ctypes.c_int32]
        L.rpcg_oracle_get_threads.restype = ctypes.c_int
        L.rpcg_cpu_plain_pcg.restype = ctypes.c_int
        L.rpcg_cpu_plain_pcg.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_double, ctypes.c_int32, P]
        _lib = L
    return _lib


def set_threads(t: int) -> int:
    """Threads of the oracle's parallel loops (< 1: the OpenMP default); returns the count in effect."""
    return lib().rpcg_oracle_set_threads(int(t))


def get_threads() -> int:
    return lib().rpcg_oracle_get_threads()


def cpu_plain_pcg(A, b, tol=1e-8, maxit=2000):
    """Host comparison loop: the same iteration with ordinary (threaded) binary64
    dots. Not a reference; returns dict(x, iters, status)."""
    b = _f64(b)
    x = np.zeros(A.n, dtype=np.float64)
    iters = ctypes.c_int32(0)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val)
    st = lib().rpcg_cpu_plain_pcg(A.n, _p(rp), _p(ci), _p(va), _p(b), _p(x), float(tol), int(maxit),
                                  ctypes.byref(iters))
    return dict(x=x, iters=iters.value, status=st)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def exdot(x, y) -> float:
    """Correctly rounded exact dot product."""
    x, y = _f64(x), _f64(y)
    assert x.shape == y.shape
    return lib().rpcg_oracle_exdot(x.size, _p(x), _p(y))


def exdot_exact(x, y) -> int:
    """Exact dot product as an integer E: sum x_i y_i = E * 2^-2148."""
    x, y = _f64(x), _f64(y)
    L = lib()
    nl = L.rpcg_oracle_exact_limbs()
    limbs = np.zeros(nl, dtype=np.uint32)
    sign = ctypes.c_int(0)
    rc = L.rpcg_oracle_exdot_exact(x.size, _p(x), _p(y), _p(limbs), ctypes.byref(sign))
    if rc != 0:
        raise ValueError("non-finite input")
    v = int.from_bytes(limbs.astype("<u4").tobytes(), "little")
    return -v if sign.value else v


EXACT_LSB_EXP = -2148


def round_exact(E: int) -> float:
    """Round E * 2^-2148 to the nearest double (ties to even) with the oracle's rounding."""
    L = lib()
    nl = L.rpcg_oracle_exact_limbs()
    mag = abs(E)
    limbs = np.frombuffer(mag.to_bytes(4 * nl, "little"), dtype="<u4").copy()
    return L.rpcg_oracle_round_limbs(_p(limbs), 1 if E < 0 else 0)


def spmv(A, x):
    x = _f64(x)
    y = np.empty(A.n, dtype=np.float64)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val)
    lib().rpcg_oracle_spmv(A.n, _p(rp), _p(ci), _p(va), _p(x), _p(y))
    return y


def true_residual(A, b, x):
    """r_i = RN(b_i - sum_j a_ij x_j) with exact row sums."""
    b, x = _f64(b), _f64(x)
    r = np.empty(A.n, dtype=np.float64)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val)
    lib().rpcg_oracle_true_residual(A.n, _p(rp), _p(ci), _p(va), _p(b), _p(x), _p(r))
    return r


def relres_true(A, b, x) -> float:
    """sqrt(<r,r>) / sqrt(<b,b>) with r the exact-row-sum residual and exact dots."""
    r = true_residual(A, b, x)
    bb = exdot(b, b)
    return float(np.sqrt(exdot(r, r)) / np.sqrt(bb)) if bb > 0 else float(np.sqrt(exdot(r, r)))


def pcg(A, b, x0=None, tol=1e-8, maxit=2000, trace=False):
    """Jacobi-PCG. Returns dict(x, iters, hist, status[, trace_r, trace_d, trace_x])."""
    n = A.n
    b = _f64(b)
    x = np.zeros(n, dtype=np.float64) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit + 1, dtype=np.float64)
    iters = ctypes.c_int32(0)
    tr = td = tx = None
    if trace:
        tr = np.zeros((maxit + 1) * n, dtype=np.float64)
        td = np.zeros_like(tr)
        tx = np.zeros_like(tr)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val)
    st = lib().rpcg_oracle_pcg(n, _p(rp), _p(ci), _p(va), _p(b), _p(x), float(tol), int(maxit),
                               _p(hist), ctypes.byref(iters), _p(tr), _p(td), _p(tx))
    L = iters.value
    out = dict(x=x, iters=L, hist=hist[:L + 1].copy(), status=st)
    if trace:
        out["trace_r"] = tr.reshape(maxit + 1, n)[:L + 1]
        out["trace_d"] = td.reshape(maxit + 1, n)[:L + 1]
        out["trace_x"] = tx.reshape(maxit + 1, n)[:L + 1]
    return out


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def exdot_f32(x, y) -> np.float32:
    """Exact dot product of binary32 vectors rounded once to binary32."""
    x, y = _f32(x), _f32(y)
    assert x.shape == y.shape
    return np.float32(lib().rpcg_oracle_exdot_f32(x.size, _p(x), _p(y)))


def spmv_f32(A, x):
    """binary32 fmaf chains; A.val is taken as binary32 (exact for the stencils used)."""
    x = _f32(x)
    y = np.empty(A.n, dtype=np.float32)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f32(A.val)
    lib().rpcg_oracle_spmv_f32(A.n, _p(rp), _p(ci), _p(va), _p(x), _p(y))
    return y


def pcg_f32(A, b, x0=None, tol=1e-4, maxit=2000, trace=False):
    """Jacobi-PCG entirely in binary32. Returns dict(x, iters, hist, status,
    thr[, trace_r, trace_d, trace_x])."""
    n = A.n
    b = _f32(b)
    x = np.zeros(n, dtype=np.float32) if x0 is None else _f32(x0).copy()
    hist = np.zeros(maxit + 1, dtype=np.float64)
    iters = ctypes.c_int32(0)
    thr = ctypes.c_float(0.0)
    tr = td = tx = None
    if trace:
        tr = np.zeros((maxit + 1) * n, dtype=np.float32)
        td = np.zeros_like(tr)
        tx = np.zeros_like(tr)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f32(A.val)
    st = lib().rpcg_oracle_pcg_f32(n, _p(rp), _p(ci), _p(va), _p(b), _p(x), float(tol), int(maxit),
                                   _p(hist), ctypes.byref(iters), _p(tr), _p(td), _p(tx), ctypes.byref(thr))
    L = iters.value
    out = dict(x=x, iters=L, hist=hist[:L + 1].copy(), status=st, thr=np.float32(thr.value))
    if trace:
        out["trace_r"] = tr.reshape(maxit + 1, n)[:L + 1]
        out["trace_d"] = td.reshape(maxit + 1, n)[:L + 1]
        out["trace_x"] = tx.reshape(maxit + 1, n)[:L + 1]
    return out


def ir_scale(rr: float) -> int:
    return lib().rpcg_oracle_ir_scale(float(rr))


def ir(A, b, x0=None, tol=1e-10, maxit_out=50, tol_in=1e-4, maxit_in=2000, adaptive=True):
    """Mixed-precision refinement (binary32 inner PCG on the values rounded to
    binary32, binary64 outer loop on the values as given); adaptive: the inner
    tolerance of a step is max(tol_in, 0.25 sqrt(thr / rr)).
    Returns dict(x, outer, inner, hist (rr per outer step), tin (inner
    tolerance per correction), status)."""
    n = A.n
    b = _f64(b)
    x = np.zeros(n, dtype=np.float64) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit_out + 1, dtype=np.float64)
    tin = np.zeros(maxit_out + 1, dtype=np.float64)
    outer, inner = ctypes.c_int32(0), ctypes.c_int32(0)
    rp, ci, va = _i32(A.row_ptr), _i32(A.col_idx), _f64(A.val)
    st = lib().rpcg_oracle_ir(n, _p(rp), _p(ci), _p(va), _p(b), _p(x), float(tol), int(maxit_out),
                              float(tol_in), int(maxit_in), int(bool(adaptive)), _p(hist), ctypes.byref(outer),
                              ctypes.byref(inner), _p(tin))
    k = outer.value
    return dict(x=x, outer=k, inner=inner.value, hist=hist[:k + 1].copy(), tin=tin[:k].copy(), status=st)


def pcg_factored(A, G, Gt, eps, b, x0=None, tol=1e-8, maxit=2000, trace=False):
    """PCG with M^-1 = G G^T + eps I (G^T given explicitly as Gt).
    Returns dict(x, iters, hist, status[, trace_r, trace_d, trace_x])."""
    n = A.n
    b = _f64(b)
    x = np.zeros(n, dtype=np.float64) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit + 1, dtype=np.float64)
    iters = ctypes.c_int32(0)
    tr = td = tx = None
    if trace:
        tr = np.zeros((maxit + 1) * n, dtype=np.float64)
        td = np.zeros_like(tr)
        tx = np.zeros_like(tr)
    arrs = []
    for M in (A, G, Gt):
        arrs += [_i32(M.row_ptr), _i32(M.col_idx), _f64(M.val)]
    st = lib().rpcg_oracle_pcg_factored(n, *[_p(a) for a in arrs], float(eps), _p(b), _p(x), float(tol), int(maxit),
                                        _p(hist), ctypes.byref(iters), _p(tr), _p(td), _p(tx))
    L = iters.value
    out = dict(x=x, iters=L, hist=hist[:L + 1].copy(), status=st)
    if trace:
        out["trace_r"] = tr.reshape(maxit + 1, n)[:L + 1]
        out["trace_d"] = td.reshape(maxit + 1, n)[:L + 1]
        out["trace_x"] = tx.reshape(maxit + 1, n)[:L + 1]
    return out


def transpose_csr(M):
    """Explicit transpose of a square CSR (rows of M^T in ascending column order);
    a storage conversion with no arithmetic."""
    n = M.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(M.row_ptr, dtype=np.int64)))
    cols = np.asarray(M.col_idx, dtype=np.int64)
    order = np.lexsort((rows, cols))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, cols + 1, 1)
    from rpcg_workloads import CSRHost
    return CSRHost(n, np.cumsum(rp).astype(np.int32), rows[order].astype(np.int32),
                   np.asarray(M.val, dtype=np.float64)[order])

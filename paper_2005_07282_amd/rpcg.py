"""Python binding of librpcg.so: argument marshalling only.

Every arithmetic step runs in the library's HIP kernels; torch provides the
device memory (tensors) and the stream. The binding refuses to run if the
library is missing, is not built for this GPU, or a tensor is not a
contiguous CUDA/HIP tensor of the right dtype.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpcg.so")

MODES = {"plain": 0, "fpe": 1, "exblas": 2}

OK, WARN_MAXIT, WARN_FPE_INEXACT = 0, 1, 2
ERR_INVALID, ERR_HIP, ERR_OOM, ERR_NOT_SPD, ERR_BREAKDOWN, ERR_NONFINITE = -1, -2, -3, -4, -5, -6

ACC_DIGITS = 68
ACC_EXP0 = -1088


class RpcgError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: status {status} ({status_string(status)})")
        self.status = status


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("fpe_size", ctypes.c_int32),
                ("early_exit", ctypes.c_int32), ("fpe_fallback", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("grid_size", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("xcd_parts", ctypes.c_int32), ("spmv_block_size", ctypes.c_int32),
                ("spmv_grid_size", ctypes.c_int32), ("no_col16", ctypes.c_int32), ("tau_history", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("tau0", ctypes.c_double),
                ("tau_final", ctypes.c_double), ("threshold", ctypes.c_double),
                ("fpe_escapes", ctypes.c_int64), ("fallbacks", ctypes.c_int64),
                ("setup_ms", ctypes.c_double), ("loop_ms", ctypes.c_double),
                ("k_spmv_dot_ms", ctypes.c_double), ("k_update_ms", ctypes.c_double),
                ("k_direction_ms", ctypes.c_double), ("k_launches", ctypes.c_int32),
                ("grid_size", ctypes.c_int32), ("block_size", ctypes.c_int32)]


class _IrOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("adaptive_inner", ctypes.c_int32),
                ("rr_history", ctypes.c_void_p), ("inner", _Opts)]


class _IrResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer", ctypes.c_int32), ("inner_iterations", ctypes.c_int32),
                ("last_inner_status", ctypes.c_int32), ("rr0", ctypes.c_double), ("rr_final", ctypes.c_double),
                ("threshold", ctypes.c_double), ("fpe_escapes", ctypes.c_int64), ("setup_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("inner_ms", ctypes.c_double), ("outer_ms", ctypes.c_double),
                ("k_residual_ms", ctypes.c_double), ("k_spmv_dot_ms", ctypes.c_double),
                ("k_update_ms", ctypes.c_double), ("k_direction_ms", ctypes.c_double),
                ("k_launches", ctypes.c_int32), ("pad1", ctypes.c_int32)]


class _BatchTuning(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("tile_slices", ctypes.c_int32), ("grid_size", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("graph_iterations", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("ms_per_iteration", ctypes.c_double)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("graph_launches", ctypes.c_int32), ("max_iterations", ctypes.c_int32),
                ("repartitions", ctypes.c_int32), ("total_iterations", ctypes.c_int64), ("setup_ms", ctypes.c_double),
                ("loop_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


_lib = None
_ctx = {}


def lib():
    """Load librpcg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2005_07282_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.rpcg_opts_default.argtypes = [ctypes.POINTER(_Opts)]
        L.rpcg_opts_default.restype = None
        L.rpcg_status_string.argtypes = [ctypes.c_int]
        L.rpcg_status_string.restype = ctypes.c_char_p
        L.rpcg_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        L.rpcg_create.restype = ctypes.c_int
        L.rpcg_destroy.argtypes = [P]
        L.rpcg_destroy.restype = None
        L.rpcg_exdot.argtypes = [P, ctypes.c_int, I64, P, P, P, ctypes.POINTER(_Opts), ctypes.POINTER(_Result), P]
        L.rpcg_exdot.restype = ctypes.c_int
        L.rpcg_exdot_noalloc.argtypes = [ctypes.c_int, I64, P, P, P, ctypes.POINTER(_Opts), ctypes.POINTER(_Result), P]
        L.rpcg_exdot_noalloc.restype = ctypes.c_int
        L.rpcg_fpe_size_auto.argtypes = [P, ctypes.POINTER(_Csr), P, P, P, P]
        L.rpcg_fpe_size_auto.restype = ctypes.c_int
        L.rpcg_spmv.argtypes = [P, ctypes.POINTER(_Csr), P, P, P]
        L.rpcg_spmv.restype = ctypes.c_int
        L.rpcg_smat_create.argtypes = [P, ctypes.POINTER(_Csr), ctypes.POINTER(P), P]
        L.rpcg_smat_create.restype = ctypes.c_int
        L.rpcg_smat_spmv.argtypes = [P, P, P, P]
        L.rpcg_smat_spmv.restype = ctypes.c_int
        L.rpcg_smat_destroy.argtypes = [P]
        L.rpcg_smat_destroy.restype = None
        L.rpcg_pcg_solve.argtypes = [P, ctypes.c_int, ctypes.POINTER(_Csr), P, P, ctypes.POINTER(_Opts),
                                     ctypes.POINTER(_Result), P]
        L.rpcg_pcg_solve.restype = ctypes.c_int
        L.rpcg_pcg_solve_factored.argtypes = [P, ctypes.c_int, ctypes.POINTER(_Csr), ctypes.POINTER(_Csr),
                                              ctypes.POINTER(_Csr), ctypes.c_double, P, P, ctypes.POINTER(_Opts),
                                              ctypes.POINTER(_Result), P]
        L.rpcg_pcg_solve_factored.restype = ctypes.c_int
        L.rpcg_pcg_solve_f32.argtypes = [P, ctypes.c_int, ctypes.POINTER(_Csr), P, P, ctypes.POINTER(_Opts),
                                         ctypes.POINTER(_Result), P]
        L.rpcg_pcg_solve_f32.restype = ctypes.c_int
        L.rpcg_ir_opts_default.argtypes = [ctypes.POINTER(_IrOpts)]
        L.rpcg_ir_opts_default.restype = None
        L.rpcg_ir_solve.argtypes = [P, ctypes.c_int, ctypes.POINTER(_Csr), P, P, ctypes.POINTER(_IrOpts),
                                    ctypes.POINTER(_IrResult), P]
        L.rpcg_ir_solve.restype = ctypes.c_int
        L.rpcg_batch_create.argtypes = [P, ctypes.c_int, I32, P, ctypes.POINTER(_Opts), ctypes.POINTER(P), P]
        L.rpcg_batch_create.restype = ctypes.c_int
        L.rpcg_batch_destroy.argtypes = [P]
        L.rpcg_batch_destroy.restype = None
        L.rpcg_batch_get_tuning.argtypes = [P, ctypes.POINTER(_BatchTuning)]
        L.rpcg_batch_get_tuning.restype = ctypes.c_int
        L.rpcg_batch_set_tuning.argtypes = [P, ctypes.POINTER(_BatchTuning)]
        L.rpcg_batch_set_tuning.restype = ctypes.c_int
        L.rpcg_batch_tune.argtypes = [P, P, I32, ctypes.POINTER(_BatchTuning), P]
        L.rpcg_batch_tune.restype = ctypes.c_int
        L.rpcg_batch_solve.argtypes = [P, P, P, P, P, ctypes.POINTER(_BatchStats), P]
        L.rpcg_batch_solve.restype = ctypes.c_int
        L.rpcg_lp_pattern_nnz.argtypes = [I32]
        L.rpcg_lp_pattern_nnz.restype = I64
        L.rpcg_lp_pattern.argtypes = [I32, P, P, P, P]
        L.rpcg_lp_pattern.restype = ctypes.c_int
        L.rpcg_lp_create.argtypes = [P, I32, I32, ctypes.POINTER(P)]
        L.rpcg_lp_create.restype = ctypes.c_int
        L.rpcg_lp_destroy.argtypes = [P]
        L.rpcg_lp_destroy.restype = None
        L.rpcg_lp_set_params.argtypes = [P, P]
        L.rpcg_lp_set_params.restype = ctypes.c_int
        L.rpcg_lp_get_params.argtypes = [P, P]
        L.rpcg_lp_get_params.restype = ctypes.c_int
        L.rpcg_lp_forward.argtypes = [P, I32, P, P, P]
        L.rpcg_lp_forward.restype = ctypes.c_int
        L.rpcg_lp_factor.argtypes = [P, I32, P, P, P, P]
        L.rpcg_lp_factor.restype = ctypes.c_int
        L.rpcg_lp_loss_grad.argtypes = [P, I32, P, P, I32, ctypes.c_double, P, P, P]
        L.rpcg_lp_loss_grad.restype = ctypes.c_int
        L.rpcg_lp_backward.argtypes = [P, I32, P, P, P, P]
        L.rpcg_lp_backward.restype = ctypes.c_int
        L.rpcg_lp_train_step.argtypes = [P, I32, P, P, I32, ctypes.c_double, ctypes.c_float, P, P]
        L.rpcg_lp_train_step.restype = ctypes.c_int
        L.rpcg_exdot_partial.argtypes = [P, I64, P, P, P, P]
        L.rpcg_exdot_partial.restype = ctypes.c_int
        L.rpcg_acc_round.argtypes = [P, P, P, P]
        L.rpcg_acc_round.restype = ctypes.c_int
        _ = I32
        _lib = L
    return _lib


EXPORTED = ["rpcg_opts_default", "rpcg_status_string", "rpcg_create", "rpcg_destroy", "rpcg_exdot", "rpcg_exdot_noalloc",
            "rpcg_fpe_size_auto",
            "rpcg_spmv", "rpcg_smat_create", "rpcg_smat_spmv", "rpcg_smat_destroy", "rpcg_pcg_solve", "rpcg_pcg_solve_factored", "rpcg_pcg_solve_f32", "rpcg_ir_opts_default", "rpcg_ir_solve",
            "rpcg_batch_create", "rpcg_batch_destroy", "rpcg_batch_get_tuning", "rpcg_batch_set_tuning",
            "rpcg_batch_tune", "rpcg_batch_solve", "rpcg_lp_pattern_nnz", "rpcg_lp_pattern", "rpcg_lp_create",
            "rpcg_lp_destroy", "rpcg_lp_set_params", "rpcg_lp_get_params", "rpcg_lp_forward", "rpcg_lp_factor",
            "rpcg_lp_loss_grad", "rpcg_lp_backward", "rpcg_lp_train_step", "rpcg_exdot_partial", "rpcg_acc_round"]


def status_string(s: int) -> str:
    return lib().rpcg_status_string(int(s)).decode()


def context(device: int | None = None):
    """The library context of a device (created once per process)."""
    if device is None:
        device = torch.cuda.current_device()
    if device not in _ctx:
        h = ctypes.c_void_p()
        rc = lib().rpcg_create(ctypes.byref(h), int(device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_create")
        _ctx[device] = h
    return _ctx[device]


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _opts(**kw) -> _Opts:
    o = _Opts()
    lib().rpcg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if v is None:
            continue
        if k == "tau_history":
            _check(v, torch.float64, "tau_history")
            o.tau_history = v.data_ptr()
        elif hasattr(o, k):
            setattr(o, k, v)
        else:
            raise TypeError(f"unknown option {k}")
    return o


def _result_dict(r: _Result) -> dict:
    return {f: getattr(r, f) for f, _ in _Result._fields_}


@dataclass
class CSR:
    """A CSR matrix whose arrays live on the GPU (int32 indices; float64
    values, or float32 values for the binary32 solver)."""
    n: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @staticmethod
    def from_host(A, device="cuda", dtype=torch.float64) -> "CSR":
        """Copy a host CSR to the GPU; dtype=torch.float32 rounds the values
        to nearest binary32 on the host (a storage conversion)."""
        return CSR(int(A.n), torch.as_tensor(A.row_ptr, dtype=torch.int32).to(device),
                   torch.as_tensor(A.col_idx, dtype=torch.int32).to(device),
                   torch.as_tensor(A.val, dtype=torch.float64).to(dtype).to(device))

    def _c(self, dtype=torch.float64) -> _Csr:
        _check(self.row_ptr, torch.int32, "row_ptr")
        _check(self.col_idx, torch.int32, "col_idx")
        _check(self.val, dtype, "val")
        if self.row_ptr.numel() != self.n + 1 or self.val.numel() != self.col_idx.numel():
            raise ValueError("inconsistent CSR sizes")
        return _Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())


def exdot(x: torch.Tensor, y: torch.Tensor, mode: str = "exblas", out: torch.Tensor | None = None,
          sync: bool = True, **opts):
    """<x, y> on the GPU. Returns (out tensor of one double, info dict or None if sync=False)."""
    _check(x, torch.float64, "x")
    _check(y, torch.float64, "y")
    if x.numel() != y.numel() or x.device != y.device:
        raise ValueError("x and y must have the same length and device")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(out, torch.float64, "out")
    o = _opts(**opts)
    r = _Result()
    rc = lib().rpcg_exdot(context(x.device.index), MODES[mode], x.numel(), x.data_ptr(), y.data_ptr(),
                          out.data_ptr(), ctypes.byref(o), ctypes.byref(r) if sync else None,
                          _stream(x.device))
    if rc < 0:
        raise RpcgError(rc, "rpcg_exdot")
    return out, (_result_dict(r) if sync else None)


def exdot_noalloc(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor, mode: str = "exblas", sync: bool = True,
                  **opts):
    """<x, y> into the caller's out (one double on the GPU) through the
    entry point that allocates nothing. Returns the info dict, or None with
    sync=False."""
    _check(x, torch.float64, "x")
    _check(y, torch.float64, "y")
    _check(out, torch.float64, "out")
    if x.numel() != y.numel() or x.device != y.device or out.device != x.device:
        raise ValueError("x, y and out must be on one device and x, y of one length")
    o = _opts(**opts)
    r = _Result()
    with torch.cuda.device(x.device):
        rc = lib().rpcg_exdot_noalloc(MODES[mode], x.numel(), x.data_ptr(), y.data_ptr(), out.data_ptr(),
                                      ctypes.byref(o), ctypes.byref(r) if sync else None, _stream(x.device))
    if rc < 0:
        raise RpcgError(rc, "rpcg_exdot_noalloc")
    return _result_dict(r) if sync else None


def exdot_partial(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Exact <x, y> as RPCG_ACC_DIGITS int64 digits (digit k weighs 2^(32k - 1088))."""
    _check(x, torch.float64, "x")
    _check(y, torch.float64, "y")
    digits = torch.empty(ACC_DIGITS, dtype=torch.int64, device=x.device)
    rc = lib().rpcg_exdot_partial(context(x.device.index), x.numel(), x.data_ptr(), y.data_ptr(),
                                  digits.data_ptr(), _stream(x.device))
    if rc < 0:
        raise RpcgError(rc, "rpcg_exdot_partial")
    return digits


def acc_round(digits: torch.Tensor) -> torch.Tensor:
    _check(digits, torch.int64, "digits")
    out = torch.empty(1, dtype=torch.float64, device=digits.device)
    rc = lib().rpcg_acc_round(context(digits.device.index), digits.data_ptr(), out.data_ptr(),
                              _stream(digits.device))
    if rc < 0:
        raise RpcgError(rc, "rpcg_acc_round")
    return out


def digits_to_int(digits: torch.Tensor) -> int:
    """Exact value of a digit vector as an integer E: value = E * 2^ACC_EXP0."""
    return sum(int(v) << (32 * k) for k, v in enumerate(digits.cpu().tolist()))


def spmv(A: CSR, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    _check(x, torch.float64, "x")
    if y is None:
        y = torch.empty(A.n, dtype=torch.float64, device=x.device)
    _check(y, torch.float64, "y")
    c = A._c()
    rc = lib().rpcg_spmv(context(x.device.index), ctypes.byref(c), x.data_ptr(), y.data_ptr(), _stream(x.device))
    if rc < 0:
        raise RpcgError(rc, "rpcg_spmv")
    return y


class PreparedMatrix:
    """A CSR matrix copied into the sliced-ELL layout for repeated products
    (rpcg_smat_*); products are bit-identical to spmv(). The copy does not
    refer to the CSR arrays afterwards."""

    def __init__(self, A: CSR):
        self.n = A.n
        self.device = A.val.device
        h = ctypes.c_void_p()
        c = A._c()
        rc = lib().rpcg_smat_create(context(self.device.index), ctypes.byref(c), ctypes.byref(h),
                                    _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_smat_create")
        self._h = h

    def spmv(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        _check(x, torch.float64, "x")
        if y is None:
            y = torch.empty(self.n, dtype=torch.float64, device=x.device)
        _check(y, torch.float64, "y")
        rc = lib().rpcg_smat_spmv(self._h, x.data_ptr(), y.data_ptr(), _stream(x.device))
        if rc < 0:
            raise RpcgError(rc, "rpcg_smat_spmv")
        return y

    def close(self):
        if getattr(self, "_h", None):
            lib().rpcg_smat_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_solve(A: CSR, b: torch.Tensor, x0: torch.Tensor | None = None, mode: str = "exblas",
              history: bool = True, raise_on_error: bool = True, **opts):
    """Jacobi-PCG. Returns (x, info); info['hist'] holds tau^(0..L) when history=True."""
    _check(b, torch.float64, "b")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    _check(x, torch.float64, "x")
    o = _opts(**opts)
    hist = None
    if history and o.tau_history is None:
        hist = torch.zeros(o.maxit + 1, dtype=torch.float64, device=b.device)
        o.tau_history = hist.data_ptr()
    c = A._c()
    r = _Result()
    rc = lib().rpcg_pcg_solve(context(b.device.index), MODES[mode], ctypes.byref(c), b.data_ptr(),
                              x.data_ptr(), ctypes.byref(o), ctypes.byref(r), _stream(b.device))
    info = _result_dict(r)
    info["status"] = rc
    if hist is not None:
        info["hist"] = hist[: r.iterations + 1].cpu()
    if rc < 0 and raise_on_error:
        raise RpcgError(rc, "rpcg_pcg_solve")
    return x, info


def pcg_solve_f32(A: CSR, b: torch.Tensor, x0: torch.Tensor | None = None, mode: str = "exblas",
                  history: bool = True, raise_on_error: bool = True, **opts):
    """Jacobi-PCG in binary32 (A.val float32, b float32). Returns (x, info);
    info['hist'] holds tau^(0..L) widened to float64 when history=True."""
    _check(b, torch.float32, "b")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    _check(x, torch.float32, "x")
    o = _opts(**opts)
    hist = None
    if history and o.tau_history is None:
        hist = torch.zeros(o.maxit + 1, dtype=torch.float64, device=b.device)
        o.tau_history = hist.data_ptr()
    c = A._c(torch.float32)
    r = _Result()
    rc = lib().rpcg_pcg_solve_f32(context(b.device.index), MODES[mode], ctypes.byref(c), b.data_ptr(),
                                  x.data_ptr(), ctypes.byref(o), ctypes.byref(r), _stream(b.device))
    info = _result_dict(r)
    info["status"] = rc
    if hist is not None:
        info["hist"] = hist[: r.iterations + 1].cpu()
    if rc < 0 and raise_on_error:
        raise RpcgError(rc, "rpcg_pcg_solve_f32")
    return x, info


def ir_solve(A: CSR, b: torch.Tensor, x0: torch.Tensor | None = None, mode: str = "exblas",
             tol: float = 1e-10, maxit: int = 50, tol_inner: float = 1e-4, maxit_inner: int = 2000,
             adaptive_inner: bool = True, history: bool = True, raise_on_error: bool = True, **inner):
    """Mixed-precision refinement (binary32 inner Jacobi-PCG, binary64 outer
    residual and update). tol/maxit are the outer ones, tol_inner/maxit_inner
    those of every inner solve (with adaptive_inner, tol_inner is the least
    reduction a step asks for; see rpcg_ir_opts); `inner` takes the other
    rpcg_opts fields of the inner solves (expansion length, launch shapes,
    timing). Returns (x, info); info['rr_hist'] holds <r,r> of every outer
    step when history=True."""
    _check(b, torch.float64, "b")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    _check(x, torch.float64, "x")
    o = _IrOpts()
    lib().rpcg_ir_opts_default(ctypes.byref(o))
    o.tol = tol
    o.maxit = maxit
    o.adaptive_inner = int(bool(adaptive_inner))
    o.inner.tol = tol_inner
    o.inner.maxit = maxit_inner
    for k, v in inner.items():
        if v is None:
            continue
        if k in ("tau_history", "tol", "maxit") or not hasattr(o.inner, k):
            raise TypeError(f"unknown inner option {k}")
        setattr(o.inner, k, v)
    hist = None
    if history:
        hist = torch.zeros(maxit + 1, dtype=torch.float64, device=b.device)
        o.rr_history = hist.data_ptr()
    c = A._c()
    r = _IrResult()
    rc = lib().rpcg_ir_solve(context(b.device.index), MODES[mode], ctypes.byref(c), b.data_ptr(), x.data_ptr(),
                             ctypes.byref(o), ctypes.byref(r), _stream(b.device))
    info = {f: getattr(r, f) for f, _ in _IrResult._fields_ if not f.startswith("pad")}
    info["status"] = rc
    if hist is not None:
        info["rr_hist"] = hist[: r.outer + 1].cpu()
    if rc < 0 and raise_on_error:
        raise RpcgError(rc, "rpcg_ir_solve")
    return x, info


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for k, t in enumerate(tensors):
        arr[k] = None if t is None else t.data_ptr()
    return arr


class Batch:
    """Many independent systems solved together (rpcg_batch_*). The CSR
    matrices must stay alive and unchanged while the batch exists."""

    def __init__(self, mats, mode: str = "exblas", **opts):
        if not mats:
            raise ValueError("empty batch")
        self.mats = list(mats)
        dev = self.mats[0].val.device
        self.device = dev
        self.mode = mode
        self._opts = _opts(**opts)
        if self._opts.tau_history:
            raise TypeError("tau_history is given per solve")
        self.maxit = self._opts.maxit
        arr = (_Csr * len(self.mats))()
        for k, A in enumerate(self.mats):
            arr[k] = A._c()
        self._csr = arr
        h = ctypes.c_void_p()
        rc = lib().rpcg_batch_create(context(dev.index), MODES[mode], len(self.mats), ctypes.cast(arr, ctypes.c_void_p),
                                     ctypes.byref(self._opts), ctypes.byref(h), _stream(dev))
        if rc != 0:
            raise RpcgError(rc, "rpcg_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().rpcg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tuning(self) -> dict:
        t = _BatchTuning()
        rc = lib().rpcg_batch_get_tuning(self._h, ctypes.byref(t))
        if rc != 0:
            raise RpcgError(rc, "rpcg_batch_get_tuning")
        return {f: getattr(t, f) for f, _ in _BatchTuning._fields_ if f != "pad0"}

    def set_tuning(self, **kw):
        t = _BatchTuning()
        lib().rpcg_batch_get_tuning(self._h, ctypes.byref(t))
        for k, v in kw.items():
            if not hasattr(t, k) or k == "pad0":
                raise TypeError(f"unknown tuning field {k}")
            setattr(t, k, v)
        rc = lib().rpcg_batch_set_tuning(self._h, ctypes.byref(t))
        if rc != 0:
            raise RpcgError(rc, "rpcg_batch_set_tuning")

    def tune(self, bs, trial_iterations: int = 10) -> dict:
        for b in bs:
            _check(b, torch.float64, "b")
        t = _BatchTuning()
        rc = lib().rpcg_batch_tune(self._h, ctypes.cast(_ptr_array(bs), ctypes.c_void_p), int(trial_iterations),
                                   ctypes.byref(t), _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_batch_tune")
        return {f: getattr(t, f) for f, _ in _BatchTuning._fields_ if f != "pad0"}

    def solve(self, bs, x0s=None, history: bool = True, raise_on_error: bool = True):
        """Returns (xs, infos, stats): per-system solutions and result dicts
        (info['hist'] = tau^(0..L) when history=True) and the batch figures."""
        if len(bs) != len(self.mats):
            raise ValueError("one right-hand side per system")
        xs = []
        for k, b in enumerate(bs):
            _check(b, torch.float64, "b")
            x = torch.zeros_like(b) if x0s is None or x0s[k] is None else x0s[k].clone()
            _check(x, torch.float64, "x")
            xs.append(x)
        hists = [torch.zeros(self.maxit + 1, dtype=torch.float64, device=self.device) for _ in bs] if history else None
        res = (_Result * len(bs))()
        st = _BatchStats()
        rc = lib().rpcg_batch_solve(self._h, ctypes.cast(_ptr_array(bs), ctypes.c_void_p),
                                    ctypes.cast(_ptr_array(xs), ctypes.c_void_p),
                                    ctypes.cast(_ptr_array(hists), ctypes.c_void_p) if hists else None,
                                    ctypes.cast(res, ctypes.c_void_p), ctypes.byref(st), _stream(self.device))
        infos = []
        for k in range(len(bs)):
            d = _result_dict(res[k])
            if hists is not None:
                d["hist"] = hists[k][: res[k].iterations + 1].cpu()
            infos.append(d)
        stats = {f: getattr(st, f) for f, _ in _BatchStats._fields_ if f != "pad0"}
        if rc < 0 and raise_on_error:
            raise RpcgError(rc, "rpcg_batch_solve")
        return xs, infos, stats


def pcg_solve_factored(A: CSR, G: CSR, Gt: CSR, eps: float, b: torch.Tensor, x0: torch.Tensor | None = None,
                       mode: str = "exblas", history: bool = True, raise_on_error: bool = True, **opts):
    """PCG with M^-1 = G G^T + eps I (Gt = G^T given explicitly). Returns (x, info)."""
    _check(b, torch.float64, "b")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    _check(x, torch.float64, "x")
    o = _opts(**opts)
    hist = None
    if history and o.tau_history is None:
        hist = torch.zeros(o.maxit + 1, dtype=torch.float64, device=b.device)
        o.tau_history = hist.data_ptr()
    ca, cg, cgt = A._c(), G._c(), Gt._c()
    r = _Result()
    rc = lib().rpcg_pcg_solve_factored(context(b.device.index), MODES[mode], ctypes.byref(ca), ctypes.byref(cg),
                                       ctypes.byref(cgt), float(eps), b.data_ptr(), x.data_ptr(), ctypes.byref(o),
                                       ctypes.byref(r), _stream(b.device))
    info = _result_dict(r)
    info["status"] = rc
    if hist is not None:
        info["hist"] = hist[: r.iterations + 1].cpu()
    if rc < 0 and raise_on_error:
        raise RpcgError(rc, "rpcg_pcg_solve_factored")
    return x, info


LP_NPARAMS = 10404


def _csr_array(mats):
    arr = (_Csr * len(mats))()
    for k, A in enumerate(mats):
        arr[k] = A._c()
    return arr


class LearnedPreconditioner:
    """The network of rpcg_lp_* for systems on N^3 grids (7-point operators)."""

    def __init__(self, N: int, max_batch: int = 1, device=None, params=None):
        import numpy as np
        self.N = int(N)
        self.max_batch = int(max_batch)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        h = ctypes.c_void_p()
        rc = lib().rpcg_lp_create(context(self.device.index), self.N, self.max_batch, ctypes.byref(h))
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_create")
        self._h = h
        n = self.N ** 3
        nnz = int(lib().rpcg_lp_pattern_nnz(self.N))
        grp = np.zeros(n + 1, np.int32)
        gcol = np.zeros(nnz, np.int32)
        gtrp = np.zeros(n + 1, np.int32)
        gtcol = np.zeros(nnz, np.int32)
        rc = lib().rpcg_lp_pattern(self.N, grp.ctypes.data, gcol.ctypes.data, gtrp.ctypes.data, gtcol.ctypes.data)
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_pattern")
        self.pattern = (grp, gcol, gtrp, gtcol)
        self._grp = torch.from_numpy(grp).to(self.device)
        self._gcol = torch.from_numpy(gcol).to(self.device)
        self._gtrp = torch.from_numpy(gtrp).to(self.device)
        self._gtcol = torch.from_numpy(gtcol).to(self.device)
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "_h", None):
            lib().rpcg_lp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == LP_NPARAMS
        rc = lib().rpcg_lp_set_params(self._h, p.ctypes.data)
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_set_params")

    def get_params(self):
        import numpy as np
        p = np.zeros(LP_NPARAMS, np.float32)
        rc = lib().rpcg_lp_get_params(self._h, p.ctypes.data)
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_get_params")
        return p

    def forward(self, mats):
        o = torch.empty(len(mats), self.N ** 3, 4, dtype=torch.float32, device=self.device)
        arr = _csr_array(mats)
        rc = lib().rpcg_lp_forward(self._h, len(mats), ctypes.cast(arr, ctypes.c_void_p), o.data_ptr(),
                                   _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_forward")
        return o

    def factor(self, mats):
        """[(G, Gt)] as CSR on the device for each system."""
        nnz = self._gcol.numel()
        Gs = [CSR(self.N ** 3, self._grp, self._gcol, torch.empty(nnz, dtype=torch.float64, device=self.device))
              for _ in mats]
        Gts = [CSR(self.N ** 3, self._gtrp, self._gtcol, torch.empty(nnz, dtype=torch.float64, device=self.device))
               for _ in mats]
        arr, ga, gta = _csr_array(mats), _csr_array(Gs), _csr_array(Gts)
        rc = lib().rpcg_lp_factor(self._h, len(mats), ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(ga, ctypes.c_void_p),
                                  ctypes.cast(gta, ctypes.c_void_p), _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_factor")
        return list(zip(Gs, Gts))

    def loss_grad(self, mats, us, eps=1e-6):
        """us: per system a list of vectors. Returns (loss, dL/do [nb][N^3][4] float64)."""
        nu = len(us[0])
        flat = [u for row in us for u in row]
        dout = torch.empty(len(mats), self.N ** 3, 4, dtype=torch.float64, device=self.device)
        loss = ctypes.c_double(0.0)
        arr = _csr_array(mats)
        rc = lib().rpcg_lp_loss_grad(self._h, len(mats), ctypes.cast(arr, ctypes.c_void_p),
                                     ctypes.cast(_ptr_array(flat), ctypes.c_void_p), nu, float(eps), ctypes.byref(loss),
                                     dout.data_ptr(), _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_loss_grad")
        return loss.value, dout

    def backward(self, mats, dout):
        _check(dout, torch.float64, "dout")
        grad = torch.empty(LP_NPARAMS, dtype=torch.float32, device=self.device)
        arr = _csr_array(mats)
        rc = lib().rpcg_lp_backward(self._h, len(mats), ctypes.cast(arr, ctypes.c_void_p), dout.data_ptr(),
                                    grad.data_ptr(), _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_backward")
        return grad

    def train_step(self, mats, us, lr, eps=1e-6):
        nu = len(us[0])
        flat = [u for row in us for u in row]
        loss = ctypes.c_double(0.0)
        arr = _csr_array(mats)
        rc = lib().rpcg_lp_train_step(self._h, len(mats), ctypes.cast(arr, ctypes.c_void_p),
                                      ctypes.cast(_ptr_array(flat), ctypes.c_void_p), nu, float(eps), float(lr),
                                      ctypes.byref(loss), _stream(self.device))
        if rc != 0:
            raise RpcgError(rc, "rpcg_lp_train_step")
        return loss.value


def fpe_size_auto(A: CSR, b: torch.Tensor):
    """(p, R): expansion length chosen from the exponent range R of A and b."""
    _check(b, torch.float64, "b")
    c = A._c()
    p, r = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = lib().rpcg_fpe_size_auto(context(b.device.index), ctypes.byref(c), b.data_ptr(), ctypes.byref(p),
                                  ctypes.byref(r), _stream(b.device))
    if rc != 0:
        raise RpcgError(rc, "rpcg_fpe_size_auto")
    return p.value, r.value

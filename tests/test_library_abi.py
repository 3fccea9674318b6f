"""CPU-side checks of the C-ABI library: it loads, exports every function the
header declares, and its host-only entry points behave (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpcg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpcg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2005_07282_amd import rpcg
    if not os.path.exists(rpcg.LIB_PATH):
        from paper_2005_07282_amd import build
        build.build()
    return rpcg.lib()


def test_header_lists_the_entry_points():
    names = _declared()
    for n in ("rpcg_exdot", "rpcg_spmv", "rpcg_pcg_solve", "rpcg_create", "rpcg_destroy",
              "rpcg_exdot_partial", "rpcg_acc_round", "rpcg_opts_default", "rpcg_status_string",
              "rpcg_pcg_solve_f32", "rpcg_ir_opts_default", "rpcg_ir_solve"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_binding_names_match_header():
    from paper_2005_07282_amd import rpcg
    assert sorted(rpcg.EXPORTED) == _declared()


def test_opts_default_and_status_strings(L):
    from paper_2005_07282_amd import rpcg
    o = rpcg._Opts()
    L.rpcg_opts_default(ctypes.byref(o))
    assert o.tol == 1e-8 and o.maxit == 2000 and o.fpe_size == 0
    assert o.early_exit == 1 and o.fpe_fallback == 1 and o.tau_history is None
    for s in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert rpcg.status_string(s) != "unknown status"
    assert rpcg.status_string(99) == "unknown status"


def test_struct_layout_matches_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what a C
    compiler makes of include/rpcg.h."""
    import subprocess
    from paper_2005_07282_amd import rpcg
    mirrors = {"rpcg_csr": rpcg._Csr, "rpcg_csr_f32": rpcg._Csr, "rpcg_opts": rpcg._Opts,
               "rpcg_result": rpcg._Result, "rpcg_ir_opts": rpcg._IrOpts, "rpcg_ir_result": rpcg._IrResult,
               "rpcg_batch_tuning": rpcg._BatchTuning, "rpcg_batch_stats": rpcg._BatchStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rpcg.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, field, v = line.split()
            got[(cname, field)] = int(v)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_null_arguments_rejected_without_gpu(L):
    from paper_2005_07282_amd import rpcg
    assert L.rpcg_create(None, 0) == rpcg.ERR_INVALID
    assert L.rpcg_exdot(None, 2, 10, None, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_spmv(None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_smat_create(None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_smat_spmv(None, None, None, None) == rpcg.ERR_INVALID
    L.rpcg_smat_destroy(None)
    assert L.rpcg_pcg_solve(None, 2, None, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_acc_round(None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_pcg_solve_f32(None, 2, None, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_ir_solve(None, 2, None, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_batch_create(None, 2, 1, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_batch_solve(None, None, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_batch_tune(None, None, 10, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_batch_set_tuning(None, None) == rpcg.ERR_INVALID
    L.rpcg_batch_destroy(None)
    assert L.rpcg_lp_create(None, 8, 1, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_train_step(None, 1, None, None, 1, 0.0, 0.0, None, None) == rpcg.ERR_INVALID
    L.rpcg_lp_destroy(None)
    assert L.rpcg_pcg_solve_factored(None, 2, None, None, None, 1e-6, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_fpe_size_auto(None, None, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_exdot_partial(None, 10, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_batch_get_tuning(None, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_set_params(None, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_get_params(None, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_forward(None, 1, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_factor(None, 1, None, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_loss_grad(None, 1, None, None, 1, 1e-6, None, None, None) == rpcg.ERR_INVALID
    assert L.rpcg_lp_backward(None, 1, None, None, None, None) == rpcg.ERR_INVALID


def test_status_strings(L):
    """Every status code has its own description; unknown codes get one too."""
    from paper_2005_07282_amd import rpcg
    codes = [0, 1, 2, -1, -2, -3, -4, -5, -6]
    texts = [L.rpcg_status_string(c) for c in codes]
    assert all(t for t in texts) and len(set(texts)) == len(codes)
    assert L.rpcg_status_string(12345)


def test_lp_pattern_host(L):
    import numpy as np
    from paper_2005_07282_amd import rpcg
    N = 3
    nnz = L.rpcg_lp_pattern_nnz(N)
    assert nnz == 4 * 27 - 3 * 9
    a, b, c, d = (np.zeros(28, np.int32), np.zeros(nnz, np.int32), np.zeros(28, np.int32), np.zeros(nnz, np.int32))
    assert L.rpcg_lp_pattern(N, a.ctypes.data, b.ctypes.data, c.ctypes.data, d.ctypes.data) == 0
    import scipy.sparse as sp
    G = sp.csr_matrix((np.ones(nnz), b, a), shape=(27, 27))
    Gt = sp.csr_matrix((np.ones(nnz), d, c), shape=(27, 27))
    assert (G.T != Gt).nnz == 0
    assert sp.triu(G, 1).nnz == 0 and G.diagonal().all()
    assert rpcg.LP_NPARAMS == 10404
    L.rpcg_destroy(None)


def test_ir_opts_default(L):
    from paper_2005_07282_amd import rpcg
    o = rpcg._IrOpts()
    L.rpcg_ir_opts_default(ctypes.byref(o))
    assert o.tol == 1e-10 and o.maxit == 50 and o.rr_history is None and o.adaptive_inner == 1
    assert o.inner.tol == 1e-4 and o.inner.maxit == 2000 and o.inner.fpe_fallback == 1

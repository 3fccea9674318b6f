"""Reproducible Jacobi-preconditioned CG on AMD Instinct MI355X (gfx950).

The library (librpcg.so, C ABI in include/rpcg.h) is built from
paper_2005_07282_amd/csrc by paper_2005_07282_amd/build.py; the binding in
``rpcg`` loads it and fails loudly if it is missing.
"""

from . import rpcg  # noqa: F401
from .rpcg import CSR, exdot, exdot_partial, acc_round, spmv, pcg_solve  # noqa: F401

"""Seeded synthetic inputs for the reproducible Jacobi-PCG hot path.

This module is shared by the CPU oracle tests, the GPU tests and the bench.
It builds matrices and vectors only; it holds none of the method's
arithmetic (no fma chains, no exact dots, no expansions, no rounding of sums):
where a right-hand side ``b = A x*`` is produced, the stencil has integer
coefficients and ``x*`` lies on the 2^-52 grid, so ``b`` is computed in int64
and converted once (one IEEE round-to-nearest conversion per entry).

Random numbers come from a counter-based SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): value ``i`` of
stream ``seed`` is ``mix64(key(seed) + (i + 1) * GOLDEN)``, so any index range
can be generated independently and identically on every machine.
"""

from .gen import (  # noqa: F401
    GOLDEN,
    splitmix64,
    uniform_pm1,
    uniform_pm1_int52,
    stencil27_csr,
    stencil27_rhs_from_int52,
    stencil27_nnz,
    stencil7_varcoef_csr,
    exdot_narrow,
    exdot_wide,
    exdot_conditioned,
    random_spd_csr,
    batch_grid_sizes,
    batch_systems,
    grf_field,
    grf_diffusion_csr,
    band_csr,
    scale_first,
    suitesparse_like,
    suitesparse_like_parts,
    scale_sym,
    SUITESPARSE_LIKE,
    CSRHost,
)

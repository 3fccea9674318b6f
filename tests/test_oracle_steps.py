"""Step-by-step pins of the oracle's PCG loops against exact rational arithmetic.

Every element-wise step of Fig. 1 (S1, S3, S4, S5, S7) and every scalar
(delta, rho, beta, tau, gamma, the threshold) is re-derived here from the
oracle's own trace of the previous iteration, with exact rationals and an
independent correct rounding (``exact_ref.rn`` / ``rn32``), and compared bit
for bit. The readings pinned are those of Section 4.3: SpMV rows as fma
chains from +0 in storage order, the axpy-type updates as single fma
operations, the Jacobi step as the precomputed inverse diagonal times the
residual; the dots are the exact sums rounded once (Sections 2.1, 4.3).

Each test also checks that its inputs discriminate: for every step, the
plausible misreading (a separately rounded multiply and add instead of the
fma, a division by the diagonal instead of the multiply by its inverse, a
threshold formed in binary64 and rounded once) gives a different value for
at least one element, so a mutation of the oracle at that step fails here.
"""

from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np
import pytest

from exact_ref import dot_fraction, rn, rn32
from rpcg_workloads import CSRHost, random_spd_csr, stencil7_varcoef_csr, uniform_pm1


def _bits64(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def _bits32(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def _eq64(a, b):
    return np.array_equal(_bits64(a), _bits64(b))


def _eq32(a, b):
    return np.array_equal(_bits32(a), _bits32(b))


# ---- rational definitions of the steps ------------------------------------

def fma64(a, b, c):
    return rn(F(float(a)) * F(float(b)) + F(float(c)))


def fma32(a, b, c):
    return rn32(F(float(a)) * F(float(b)) + F(float(c)))


def spmv_def(A, x, rnd):
    """Row i: acc = +0, then acc = RN(a_ik x_col + acc) per stored entry in order."""
    y = []
    for i in range(A.n):
        acc = 0.0
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc = rnd(F(float(A.val[k])) * F(float(x[A.col_idx[k]])) + F(acc))
        y.append(acc)
    return y


def diag_of(A):
    out = []
    for i in range(A.n):
        v = None
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            if A.col_idx[k] == i:
                v = float(A.val[k])
        out.append(v)
    return out


def dot_def(x, y, rnd):
    return rnd(dot_fraction([float(v) for v in x], [float(v) for v in y]))


def rn_sqrt(v: F) -> float:
    """Nearest double to sqrt(v), v >= 0: the integer square root with 1200
    extra bits, the remainder kept as a sticky half-unit (a square root of a
    rational that is not exact is irrational, so it never sits on a tie)."""
    if v == 0:
        return 0.0
    k = 1200
    X = v.numerator * (1 << (2 * k)) // v.denominator
    s = math.isqrt(X)
    exact = s * s * v.denominator == v.numerator * (1 << (2 * k))
    val = F(s, 1 << k) if exact else F(2 * s + 1, 1 << (k + 1))
    return rn(val)


def _varcoef(seed):
    return stencil7_varcoef_csr(3, seed)  # n = 27, coefficients exp(N(0,1)): no dyadic values


SYSTEMS = [("varcoef", 11), ("varcoef", 12), ("randspd", 5)]


def _system(kind, seed):
    A = _varcoef(seed) if kind == "varcoef" else random_spd_csr(12, seed)
    b = uniform_pm1(300 + seed, A.n)
    x0 = uniform_pm1(400 + seed, A.n) * 0.25
    return A, b, x0


# ---- binary64 --------------------------------------------------------------

@pytest.mark.parametrize("kind,seed", SYSTEMS)
def test_pcg_f64_every_step(orc, kind, seed):
    A, b, x0 = _system(kind, seed)
    n = A.n
    tol, maxit = 1e-30, 3  # the loop runs all three bodies
    res = orc.pcg(A, b, x0=x0, tol=tol, maxit=maxit, trace=True)
    assert res["iters"] == maxit and res["status"] == orc.WARN_MAXIT
    R, D, X, H = res["trace_r"], res["trace_d"], res["trace_x"], res["hist"]

    dinv = [rn(1 / F(a)) for a in diag_of(A)]
    # setup: r0 = RN(b - (A x0)_i) with the row as an fma chain, z0 = RN(dinv r0), d0 = z0
    w0 = spmv_def(A, x0, rn)
    r = [rn(F(float(bi)) - F(wi)) for bi, wi in zip(b, w0)]
    z = [rn(F(di) * F(ri)) for di, ri in zip(dinv, r)]
    d = list(z)
    x = [float(v) for v in x0]
    assert _eq64(R[0], r) and _eq64(D[0], d) and _eq64(X[0], x)
    beta = dot_def(z, r, rn)
    assert _eq64([H[0]], [dot_def(r, r, rn)])
    bb = dot_def(b, b, rn)
    thr = rn(F(rn(F(tol) * F(tol))) * F(bb))
    assert H[0] > thr

    seen = dict(s3=False, s4=False, s5=False, s7=False)
    for l in range(maxit):
        # continue from the oracle's own state, so every step is checked on its own
        r, d, x = [float(v) for v in R[l]], [float(v) for v in D[l]], [float(v) for v in X[l]]
        w = spmv_def(A, d, rn)                                                 # S1
        delta = dot_def(d, w, rn)                                              # S2
        rho = rn(F(beta) / F(delta))
        x1 = [fma64(rho, di, xi) for di, xi in zip(d, x)]                      # S3
        r1 = [fma64(-rho, wi, ri) for wi, ri in zip(w, r)]                     # S4
        z1 = [rn(F(di) * F(ri)) for di, ri in zip(dinv, r1)]                   # S5
        beta1 = dot_def(z1, r1, rn)                                            # S6
        tau1 = dot_def(r1, r1, rn)                                             # S8
        gamma = rn(F(beta1) / F(beta))
        d1 = [fma64(gamma, di, zi) for di, zi in zip(d, z1)]                   # S7
        assert _eq64(X[l + 1], x1), ("S3", l)
        assert _eq64(R[l + 1], r1), ("S4", l)
        assert _eq64(D[l + 1], d1), ("S5-S7", l)
        assert _eq64([H[l + 1]], [tau1]), ("S8", l)
        # the misreadings differ somewhere
        seen["s3"] |= any(rn(F(rn(F(rho) * F(di))) + F(xi)) != v for di, xi, v in zip(d, x, x1))
        seen["s4"] |= any(rn(F(ri) - F(rn(F(rho) * F(wi)))) != v for wi, ri, v in zip(w, r, r1))
        seen["s5"] |= any(rn(F(ri) / F(a)) != v for ri, a, v in zip(r1, diag_of(A), z1))
        seen["s7"] |= any(rn(F(rn(F(gamma) * F(di))) + F(zi)) != v for di, zi, v in zip(d, z1, d1))
        beta = beta1
    assert all(seen.values()), seen
    assert n == len(R[0])


# ---- binary32 --------------------------------------------------------------

def _f32(v):
    return float(np.float32(v))


@pytest.mark.parametrize("kind,seed", SYSTEMS)
def test_pcg_f32_every_step(orc, kind, seed):
    A, b64, x064 = _system(kind, seed)
    A32 = CSRHost(A.n, A.row_ptr, A.col_idx, np.asarray(A.val, dtype=np.float32).astype(np.float64))
    b = np.asarray(b64, dtype=np.float32)
    x0 = np.asarray(x064, dtype=np.float32)
    tol, maxit = 1e-30, 3
    res = orc.pcg_f32(A32, b, x0=x0, tol=tol, maxit=maxit, trace=True)
    assert res["iters"] == maxit and res["status"] == orc.WARN_MAXIT
    R, D, X, H = res["trace_r"], res["trace_d"], res["trace_x"], res["hist"]

    diag = diag_of(A32)
    dinv = [rn32(1 / F(a)) for a in diag]
    w0 = spmv_def(A32, x0, rn32)
    r = [rn32(F(float(bi)) - F(wi)) for bi, wi in zip(b, w0)]
    z = [rn32(F(di) * F(ri)) for di, ri in zip(dinv, r)]
    assert _eq32(R[0], r) and _eq32(D[0], z) and _eq32(X[0], x0)
    beta = dot_def(z, r, rn32)
    assert float(H[0]) == dot_def(r, r, rn32)
    bb = dot_def(b, b, rn32)
    tol32 = _f32(tol)
    thr = rn32(F(rn32(F(tol32) * F(tol32))) * F(bb))
    assert _eq32([res["thr"]], [thr])

    seen = dict(s3=False, s4=False, s5=False, s7=False)
    for l in range(maxit):
        r, d, x = [float(v) for v in R[l]], [float(v) for v in D[l]], [float(v) for v in X[l]]
        w = spmv_def(A32, d, rn32)
        delta = dot_def(d, w, rn32)
        rho = rn32(F(beta) / F(delta))
        x1 = [fma32(rho, di, xi) for di, xi in zip(d, x)]
        r1 = [fma32(-rho, wi, ri) for wi, ri in zip(w, r)]
        z1 = [rn32(F(di) * F(ri)) for di, ri in zip(dinv, r1)]
        beta1 = dot_def(z1, r1, rn32)
        tau1 = dot_def(r1, r1, rn32)
        gamma = rn32(F(beta1) / F(beta))
        d1 = [fma32(gamma, di, zi) for di, zi in zip(d, z1)]
        assert _eq32(X[l + 1], x1), ("S3", l)
        assert _eq32(R[l + 1], r1), ("S4", l)
        assert _eq32(D[l + 1], d1), ("S5-S7", l)
        assert float(H[l + 1]) == tau1, ("S8", l)
        seen["s3"] |= any(rn32(F(rn32(F(rho) * F(di))) + F(xi)) != v for di, xi, v in zip(d, x, x1))
        seen["s4"] |= any(rn32(F(ri) - F(rn32(F(rho) * F(wi)))) != v for wi, ri, v in zip(w, r, r1))
        seen["s5"] |= any(rn32(F(ri) / F(rn32(1 / F(di)))) != v for ri, di, v in zip(r1, dinv, z1))
        seen["s7"] |= any(rn32(F(rn32(F(gamma) * F(di))) + F(zi)) != v for di, zi, v in zip(d, z1, d1))
        beta = beta1
    assert all(seen.values()), seen


@pytest.mark.parametrize("seed", range(4))
def test_pcg_f32_threshold(orc, seed):
    """thr = RN32(RN32(t t) <b,b>) with t = RN32(tol): checked over many
    tolerances (maxit = 0, so only the setup runs); forming t t <b,b> in
    binary64 and rounding once gives another value for several of them."""
    A = _varcoef(seed + 20)
    A32 = CSRHost(A.n, A.row_ptr, A.col_idx, np.asarray(A.val, dtype=np.float32).astype(np.float64))
    b = np.asarray(uniform_pm1(500 + seed, A.n) * 3.7, dtype=np.float32)
    bb = dot_def(b, b, rn32)
    rng = np.random.default_rng(seed)
    differ = 0
    for tol in 10.0 ** rng.uniform(-7, -1, 40):
        res = orc.pcg_f32(A32, b, tol=float(tol), maxit=0)
        t = _f32(tol)
        want = rn32(F(rn32(F(t) * F(t))) * F(bb))
        assert _eq32([res["thr"]], [want]), tol
        differ += rn32(F(t) * F(t) * F(bb)) != want
    assert differ >= 3, differ


# ---- factored preconditioner ----------------------------------------------

def _lower_factor(A, seed):
    """A sparse lower-triangular G on A's pattern with non-dyadic values of
    moderate size, and its explicit transpose."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    keep = A.col_idx <= rows
    cnt = np.zeros(A.n + 1, dtype=np.int64)
    np.add.at(cnt, rows[keep] + 1, 1)
    vals = rng.uniform(-0.4, 0.4, int(keep.sum()))
    cols = A.col_idx[keep]
    vals[cols == rows[keep]] = rng.uniform(0.3, 0.9, int((cols == rows[keep]).sum()))
    return CSRHost(A.n, np.cumsum(cnt).astype(np.int32), cols.astype(np.int32), vals)


@pytest.mark.parametrize("seed", [11, 12])
def test_pcg_factored_every_step(orc, seed):
    A, b, x0 = _system("varcoef", seed)
    G = _lower_factor(A, seed)
    Gt = orc.transpose_csr(G)
    eps = 0.3141
    tol, maxit = 1e-30, 3
    res = orc.pcg_factored(A, G, Gt, eps, b, x0=x0, tol=tol, maxit=maxit, trace=True)
    assert res["iters"] == maxit
    R, D, X, H = res["trace_r"], res["trace_d"], res["trace_x"], res["hist"]

    def precond(r):
        t = spmv_def(Gt, r, rn)
        s = spmv_def(G, t, rn)
        return [fma64(eps, ri, si) for ri, si in zip(r, s)], s

    w0 = spmv_def(A, x0, rn)
    r = [rn(F(float(bi)) - F(wi)) for bi, wi in zip(b, w0)]
    z, _ = precond(r)
    assert _eq64(R[0], r) and _eq64(D[0], z)
    beta = dot_def(z, r, rn)
    seen = False
    for l in range(maxit):
        r, d, x = [float(v) for v in R[l]], [float(v) for v in D[l]], [float(v) for v in X[l]]
        w = spmv_def(A, d, rn)
        delta = dot_def(d, w, rn)
        rho = rn(F(beta) / F(delta))
        x1 = [fma64(rho, di, xi) for di, xi in zip(d, x)]
        r1 = [fma64(-rho, wi, ri) for wi, ri in zip(w, r)]
        z1, s1 = precond(r1)
        beta1 = dot_def(z1, r1, rn)
        gamma = rn(F(beta1) / F(beta))
        d1 = [fma64(gamma, di, zi) for di, zi in zip(d, z1)]
        assert _eq64(X[l + 1], x1) and _eq64(R[l + 1], r1) and _eq64(D[l + 1], d1), l
        assert _eq64([H[l + 1]], [dot_def(r1, r1, rn)])
        # z = RN(eps r + s) differs from RN(RN(eps r) + s) somewhere
        seen |= any(rn(F(rn(F(eps) * F(ri))) + F(si)) != zi for ri, si, zi in zip(r1, s1, z1))
        beta = beta1
    assert seen


# ---- exact-row residual and the refinement's inner tolerance ---------------

@pytest.mark.parametrize("seed", range(3))
def test_true_residual_rows(orc, seed):
    A = _varcoef(seed + 30)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, A.n) * 2.0 ** rng.integers(-30, 30, A.n)
    b = np.asarray(spmv_def(A, x, rn)) * (1 + rng.uniform(-1e-9, 1e-9, A.n))  # heavy cancellation
    got = orc.true_residual(A, b, x)
    for i in range(A.n):
        s = F(float(b[i]))
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            s -= F(float(A.val[k])) * F(float(x[A.col_idx[k]]))
        assert _bits64([got[i]])[0] == _bits64([rn(s)])[0], i


def test_ir_inner_tolerance_rule(orc):
    """The inner tolerance of every correction is max(tol_in, RN(0.25 RN(sqrt(RN(thr / rr)))))
    with the correctly rounded square root."""
    from rpcg_workloads import stencil27_csr, stencil27_rhs_from_int52, uniform_pm1_int52
    N = 6
    A = stencil27_csr(N)
    b = stencil27_rhs_from_int52(N, uniform_pm1_int52(7, A.n))
    tol, tol_in = 1e-10, 1e-4
    res = orc.ir(A, b, tol=tol, tol_in=tol_in, adaptive=True)
    assert res["status"] == 0 and res["outer"] >= 2
    thr = rn(F(rn(F(tol) * F(tol))) * F(dot_def(b, b, rn)))
    raised = 0
    for k, t in enumerate(res["tin"]):
        rr = float(res["hist"][k])
        need = rn(F(0.25) * F(rn_sqrt(F(rn(F(thr) / F(rr))))))
        assert t == max(tol_in, need), k
        raised += need > tol_in
    assert raised >= 1

"""Pins of the learned-preconditioner oracle (oracle/lpnet.py): bfloat16
rounding against its rational definition, the convolution against explicit
loops, the transposed and weight-gradient convolutions as exact adjoints,
the factor's structure, and the whole gradient (features -> network -> G ->
loss) against central finite differences."""

import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import lpnet
from rpcg_workloads import grf_diffusion_csr, uniform_pm1


def test_bf16_rounding_definition():
    rng = np.random.default_rng(0)
    vals = rng.standard_normal(2000).astype(np.float32) * np.float32(3.0)
    # exact ties: bf16 value plus half an ulp of bf16
    for m in (1.0, 1.5, 1.0078125, -2.75):
        b = np.float32(m).view(np.uint32)
        vals = np.append(vals, (np.uint32(b) | np.uint32(0x8000)).view(np.float32))
    got = lpnet.rn_bf16(vals)
    for v, g in zip(vals, got):
        f = Fraction(float(v))
        if f == 0:
            assert g == 0
            continue
        e = abs(f).numerator.bit_length() - abs(f).denominator.bit_length()
        while Fraction(2) ** e > abs(f):
            e -= 1
        while Fraction(2) ** (e + 1) <= abs(f):
            e += 1
        q = Fraction(2) ** (e - 7)  # 8 significant bits
        lo = (abs(f) // q) * q
        rem = abs(f) - lo
        if rem > q / 2 or (rem == q / 2 and (lo / q) % 2 == 1):
            lo += q
        want = float(lo if f > 0 else -lo)
        assert g == want, (v, g, want)


def test_conv_explicit_loops():
    rng = np.random.default_rng(1)
    N, ci, co = 3, 2, 3
    x = rng.standard_normal((N, N, N, ci))
    W = rng.standard_normal((27, co, ci))
    b = rng.standard_normal(co)
    out = lpnet.conv(x, W, b)
    for z, y, xx, c in itertools.product(range(N), range(N), range(N), range(co)):
        acc = b[c]
        for t, (dz, dy, dx) in enumerate(lpnet.OFFSETS):
            Z, Y, X = z + dz, y + dy, xx + dx
            if 0 <= Z < N and 0 <= Y < N and 0 <= X < N:
                acc += sum(W[t, c, k] * x[Z, Y, X, k] for k in range(ci))
        assert abs(out[z, y, xx, c] - acc) < 1e-12


def test_conv_adjoints():
    rng = np.random.default_rng(2)
    N = 4
    x = rng.standard_normal((N, N, N, 5))
    yv = rng.standard_normal((N, N, N, 3))
    W = rng.standard_normal((27, 3, 5))
    lhs = np.sum(lpnet.conv(x, W, np.zeros(3)) * yv)
    assert abs(lhs - np.sum(x * lpnet.conv_t(yv, W))) < 1e-9 * abs(lhs)
    Wd = rng.standard_normal((27, 3, 5))
    assert abs(np.sum(lpnet.conv(x, Wd, np.zeros(3)) * yv) - np.sum(Wd * lpnet.conv_dw(x, yv))) < 1e-9


def test_factor_structure_and_jacobi_start():
    N = 5
    A, _ = grf_diffusion_csr(N, 3)
    o = np.zeros((N ** 3, 4))
    G, dgdo = lpnet.factor(A, N, o)
    d = A.val[A.col_idx == np.repeat(np.arange(A.n), np.diff(A.row_ptr))]
    assert np.allclose((G @ G.T).toarray(), np.diag(1.0 / d), rtol=2e-7)
    o = np.random.default_rng(3).standard_normal((N ** 3, 4))
    G, _ = lpnet.factor(A, N, o)
    import scipy.sparse as sp
    pat = sp.tril(lpnet._rows(A)) != 0
    assert ((G != 0) != pat).nnz == 0  # exactly the lower triangle of A's pattern


def test_features_per_row():
    N = 4
    A, _ = grf_diffusion_csr(N, 4)
    f = lpnet.features(A, N).reshape(-1, 4)
    for i in range(A.n):
        cols = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        vals = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
        aii = vals[cols == i][0]
        for k, step in enumerate((1, N, N * N)):
            hit = vals[cols == i - step]
            same_line = (k == 0 and i % N > 0) or (k == 1 and (i // N) % N > 0) or (k == 2 and i // (N * N) > 0)
            want = np.log(abs(hit[0]) / aii) if (same_line and hit.size) else lpnet.ABSENT
            assert abs(f[i, k] - want) < 1e-12
        assert f[i, 3] == (7 - cols.size) / 6.0


def test_gradient_finite_differences():
    """Float64 pipeline (no bfloat16 rounding; G entries kept in float64 for the
    check): backward + chain rule against central differences."""
    N, eps = 4, 1e-3
    A, _ = grf_diffusion_csr(N, 7)
    rng = np.random.default_rng(8)
    p = lpnet.init_params(9, scale=1.0).astype(np.float64)
    q = lpnet.split(p)
    q["W3"] = rng.standard_normal(q["W3"].shape) * 0.05
    q["b3"] = rng.standard_normal(4) * 0.1
    p = lpnet.join(q)
    us = [uniform_pm1(20 + k, A.n) for k in range(2)]

    def loss_of(pp):
        c = lpnet.forward(pp, lpnet.features(A, N), bf16=False)
        G, dgdo = _factor64(A, N, c["o"])
        return lpnet.loss_grad(A, G, us, eps)[0], c, G, dgdo

    L0, c, G, dgdo = loss_of(p)
    _, dG = lpnet.loss_grad(A, G, us, eps)
    do = lpnet.do_from_dg(G, dG, dgdo, N)
    g = lpnet.backward(c, do)
    idx = rng.choice(lpnet.NPARAMS, 40, replace=False)
    # the output layer and the biases carry most of the gradient; include some of each
    idx = np.concatenate([idx, [lpnet.NPARAMS - 1, lpnet.NPARAMS - 5, 100, 2000]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (loss_of(p + e)[0] - loss_of(p - e)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 + 1e-4 * abs(fd), (k, fd, g[k])


def _factor64(A, N, o):
    """lpnet.factor without the float32 roundings, for the finite-difference check."""
    import scipy.sparse as sp
    M = lpnet._rows(A)
    n = N ** 3
    d = M.diagonal()
    s = 1.0 / np.sqrt(d)
    o = np.asarray(o, dtype=np.float64).reshape(n, 4)
    i = np.arange(n)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    gd = s * np.exp(np.clip(o[:, 0], -lpnet.OCLAMP, lpnet.OCLAMP))
    rows, cols, vals = [i], [i], [gd]
    dgdo = np.zeros((n, 4))
    dgdo[:, 0] = np.where(np.abs(o[:, 0]) < lpnet.OCLAMP, gd, 0.0)
    for k, (step, has) in enumerate(((1, x > 0), (N, y > 0), (N * N, z > 0)), start=1):
        rows.append(i[has])
        cols.append(i[has] - step)
        vals.append(s[has] * o[has, k])
        dgdo[has, k] = s[has]
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    G.sort_indices()
    return G, dgdo

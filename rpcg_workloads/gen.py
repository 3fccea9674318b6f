"""Generators for the synthetic workloads (host only, numpy).

Workloads follow the paper's experiments: a 3D Poisson matrix from the
27-point finite-difference stencil (Section 5.1), the right-hand side built
from a known vector (Section 5.1 uses ``A * ones``), a zero initial guess;
plus vector pairs for the standalone exact dot product with wide exponent
ranges and prescribed condition numbers (Section 2.1, Section 4.1 cost model
for wide dynamic ranges).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO52 = 1 << 52


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _key(seed: int) -> np.uint64:
    return _mix64(np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ np.uint64(0x6A09E667F3BCC909)],
                           dtype=np.uint64))[0]


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Counter-based stream: element i is mix64(key(seed) + (start + i + 1) * GOLDEN)."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = _key(seed) + idx * GOLDEN
        return _mix64(z)


def uniform_pm1_int52(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Integers K in [-2^52, 2^52): the uniform value on [-1, 1) is K * 2^-52."""
    k = (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.int64)  # 53 random bits
    return k - np.int64(_TWO52)


def uniform_pm1(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles on [-1, 1) on the 2^-52 grid (exact int -> double conversion)."""
    return uniform_pm1_int52(seed, n, start).astype(np.float64) * (2.0 ** -52)


@dataclass
class CSRHost:
    """CSR matrix on the host: int32 row pointers and column indices, values."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def stencil27_nnz(N: int) -> int:
    return (3 * N - 2) ** 3


def _stencil_offsets(kind: int):
    if kind == 27:
        return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    if kind == 7:
        return [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    raise ValueError(kind)


def _stencil_pattern(N: int, kind: int):
    """Column pattern of a Dirichlet stencil on an N^3 grid, rows in z-y-x order.

    Offsets are visited in lexicographic (dz, dy, dx) order, so the column
    indices of every row come out ascending. Returns (row_ptr, col, offset_id)."""
    n = N ** 3
    offs = _stencil_offsets(kind)
    i = np.arange(n, dtype=np.int64)
    z, y, x = i // (N * N), (i // N) % N, i % N
    cols = np.empty((n, len(offs)), dtype=np.int64)
    valid = np.empty((n, len(offs)), dtype=bool)
    for t, (dz, dy, dx) in enumerate(offs):
        ok = (z + dz >= 0) & (z + dz < N) & (y + dy >= 0) & (y + dy < N) & (x + dx >= 0) & (x + dx < N)
        valid[:, t] = ok
        cols[:, t] = i + dz * N * N + dy * N + dx
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[valid]
    oid = np.broadcast_to(np.arange(len(offs)), (n, len(offs)))[valid]
    del cols
    return row_ptr, col, oid, valid


def stencil27_csr(N: int) -> CSRHost:
    """27-point operator on an N^3 grid: 26 on the diagonal, -1 for each in-grid neighbour."""
    n = N ** 3
    if stencil27_nnz(N) >= 2 ** 31:
        raise ValueError("nnz does not fit int32 row pointers")
    row_ptr, col, oid, _ = _stencil_pattern(N, 27)
    val = np.where(oid == 13, 26.0, -1.0)
    return CSRHost(n, row_ptr.astype(np.int32), col.astype(np.int32), val.astype(np.float64))


def stencil27_rhs_from_int52(N: int, K: np.ndarray) -> np.ndarray:
    """b = A x* for x* = K * 2^-52 on the 27-point operator, rounded once per entry.

    (A x*)_i * 2^52 = 27 K_i - sum over the 3x3x3 box around i of K (zero
    outside the grid): an int64 with |value| < 2^58, converted to double by one
    round-to-nearest-even conversion, then scaled by a power of two (exact)."""
    K3 = K.reshape(N, N, N).astype(np.int64)
    P = np.zeros((N + 2, N + 2, N + 2), dtype=np.int64)
    P[1:-1, 1:-1, 1:-1] = K3
    box = np.zeros_like(K3)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                box += P[dz:dz + N, dy:dy + N, dx:dx + N]
    B = 27 * K3 - box
    return (B.astype(np.float64) * (2.0 ** -52)).reshape(-1)


def stencil7_varcoef_csr(N: int, seed: int, sigma: float = 1.0) -> CSRHost:
    """7-point diffusion on an N^3 grid with i.i.d. face coefficients exp(sigma * N(0,1)).

    Every cell face, boundary faces included, carries one coefficient k_f.
    A_ij = -k_f for the face between cells i and j; A_ii = sum of the six faces
    of cell i (boundary faces give Dirichlet coupling to zero). The matrix is
    symmetric and strictly diagonally dominant, hence SPD."""
    rng = np.random.Generator(np.random.PCG64(seed))
    # faces normal to x: (N, N, N+1), y: (N, N+1, N), z: (N+1, N, N)
    kx = np.exp(sigma * rng.standard_normal((N, N, N + 1)))
    ky = np.exp(sigma * rng.standard_normal((N, N + 1, N)))
    kz = np.exp(sigma * rng.standard_normal((N + 1, N, N)))
    diag = (kx[:, :, :-1] + kx[:, :, 1:]) + (ky[:, :-1, :] + ky[:, 1:, :]) + (kz[:-1, :, :] + kz[1:, :, :])
    # off-diagonal value for each of the 7 offsets, in (dz,dy,dx) lexicographic order
    offv = {
        (-1, 0, 0): -kz[:-1, :, :], (1, 0, 0): -kz[1:, :, :],
        (0, -1, 0): -ky[:, :-1, :], (0, 1, 0): -ky[:, 1:, :],
        (0, 0, -1): -kx[:, :, :-1], (0, 0, 1): -kx[:, :, 1:],
        (0, 0, 0): diag,
    }
    row_ptr, col, oid, valid = _stencil_pattern(N, 7)
    offs = _stencil_offsets(7)
    vals = np.stack([offv[o].reshape(-1) for o in offs], axis=1)
    val = vals[valid]
    return CSRHost(N ** 3, row_ptr.astype(np.int32), col.astype(np.int32), val.astype(np.float64))


def exdot_narrow(seed: int, n: int):
    """Vector pair with values uniform on [-1, 1) (the PCG-like, narrow-range case)."""
    return uniform_pm1(2 * seed, n), uniform_pm1(2 * seed + 1, n)


def _wide_bits(seed: int, n: int, emin: int, emax: int) -> np.ndarray:
    """Doubles +-m * 2^e: m with 52 random fraction bits, e uniform in [emin, emax], random sign."""
    r1 = splitmix64(seed, n)
    r2 = splitmix64(seed ^ 0x5DEECE66D, n)
    span = np.uint64(emax - emin + 1)
    e = (r2 % span).astype(np.int64) + emin
    sign = (r2 >> np.uint64(63)).astype(np.uint64)
    mant = r1 >> np.uint64(12)
    bits = (sign << np.uint64(63)) | ((e + 1023).astype(np.uint64) << np.uint64(52)) | mant
    return bits.view(np.float64)


def exdot_wide(seed: int, n: int, emin: int = -200, emax: int = 200):
    """Vector pair whose exponents are uniform over [emin, emax] with random signs."""
    return _wide_bits(2 * seed, n, emin, emax), _wide_bits(2 * seed + 1, n, emin, emax)


def exdot_conditioned(seed: int, n: int, cond: float, emin: int = -200, emax: int = 200):
    """Wide-exponent vector pair whose dot product has condition number about ``cond``.

    cond = sum|x_i y_i| / |sum x_i y_i|. For cond == 1 the signs of y copy the
    signs of x, so every product is positive. For cond > 1 the vectors hold
    mirrored pairs whose products cancel exactly, (x, y) and
    (x * 2^t, -y * 2^-t), plus two signal entries (2^a, 2^b) and (2^a, 2^(b-1))
    whose products sum to 1.5 * 2^(a+b), chosen so that this is near
    sum|x_i y_i| / cond; positions are then shuffled by a seeded permutation.
    The exact dot product is therefore the representable value 1.5 * 2^(a+b),
    returned as the third element (None for cond == 1)."""
    if n < 4 and cond != 1.0:
        raise ValueError("need n >= 4")
    if cond == 1.0:
        x, y = exdot_wide(seed, n, emin, emax)
        y = np.where(np.signbit(x) != np.signbit(y), -y, y)
        return x, y, None
    h = (n - 2) // 2
    xa, ya = exdot_wide(seed, h, emin, emax)
    t = (splitmix64(seed + 7777, h) % np.uint64(17)).astype(np.int64) - 8
    xb = np.ldexp(xa, t)
    yb = -np.ldexp(ya, -t)
    # approximate magnitude of sum|x_i y_i| (only used to place the signal)
    mag = 2.0 * float(np.sum(np.abs(xa * ya)))
    target = int(np.floor(np.log2(mag / cond)))
    a = target // 2
    b = target - a
    sig_x = np.array([2.0 ** a, 2.0 ** a])
    sig_y = np.array([2.0 ** b, 2.0 ** (b - 1)])
    x = np.concatenate([xa, xb, sig_x])
    y = np.concatenate([ya, yb, sig_y])
    if x.size < n:  # odd n: pad with an exact zero product
        x = np.concatenate([x, [0.0]])
        y = np.concatenate([y, [1.0]])
    perm = np.argsort(splitmix64(seed + 99991, n), kind="stable")
    exact = 1.5 * 2.0 ** (a + b)
    return x[perm], y[perm], exact


def random_spd_csr(n: int, seed: int, density: float = 0.3) -> CSRHost:
    """Small integer SPD matrix A = B^T B + I (int64, exact) in CSR form with sorted columns."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.integers(-2, 3, size=(n, n)) * (rng.random((n, n)) < density)
    A = B.T @ B + np.eye(n, dtype=np.int64)
    rows, cols = np.nonzero(A)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return CSRHost(n, row_ptr.astype(np.int32), cols.astype(np.int32), A[rows, cols].astype(np.float64))


def batch_grid_sizes(seed: int, count: int = 64, lo: int = 16, hi: int = 96) -> list:
    """Grid sizes N_s, uniform integers in [lo, hi] (the batched workload's
    cubic grids), from the counter-based stream (modulo bias below 2^-57)."""
    r = splitmix64(seed, count) % np.uint64(hi - lo + 1)
    return [int(v) + lo for v in r]


def batch_systems(seed: int, count: int = 64, lo: int = 16, hi: int = 96, sigma: float = 1.0):
    """The batched workload: `count` 7-point variable-coefficient systems on
    N_s^3 grids (N_s from batch_grid_sizes) with right-hand sides uniform on
    [-1, 1). System s uses matrix seed 1000 * seed + s and vector seed
    2000 * seed + s. Returns a list of (N_s, CSRHost, b)."""
    out = []
    for s, N in enumerate(batch_grid_sizes(seed, count, lo, hi)):
        A = stencil7_varcoef_csr(N, 1000 * seed + s, sigma)
        out.append((N, A, uniform_pm1(2000 * seed + s, A.n)))
    return out


def grf_field(N: int, seed: int, ell: float = 8.0) -> np.ndarray:
    """Stationary Gaussian random field on an N^3 grid with unit variance and
    Gaussian correlation exp(-|h|^2 / (2 ell^2)) (in cells), by FFT filtering
    of seeded white noise (periodic; the workload uses it as a texture)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((N, N, N))
    k = 2.0 * np.pi * np.fft.fftfreq(N)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    filt = np.exp(-0.25 * ell * ell * (kx * kx + ky * ky + kz * kz))  # square root of the spectral density
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g -= g.mean()
    s = g.std()
    return g / s if s > 0 else g


def grf_diffusion_csr(N: int, seed: int, sigma: float = 1.5, ell: float = 8.0):
    """7-point diffusion on an N^3 grid with log-normal cell coefficients
    c = exp(sigma * GRF) (grf_field). Face coefficient = harmonic mean of the
    two cells it separates; a boundary face takes its cell's coefficient
    (Dirichlet coupling to zero). A_ij = -k_face, A_ii = sum of the six faces.
    Returns (CSRHost, c) with the cell coefficients c (N, N, N)."""
    c = np.exp(sigma * grf_field(N, seed, ell))

    def hmean(a, b):
        return 2.0 * a * b / (a + b)

    kx = np.empty((N, N, N + 1))
    ky = np.empty((N, N + 1, N))
    kz = np.empty((N + 1, N, N))
    kx[:, :, 1:-1] = hmean(c[:, :, :-1], c[:, :, 1:])
    kx[:, :, 0], kx[:, :, -1] = c[:, :, 0], c[:, :, -1]
    ky[:, 1:-1, :] = hmean(c[:, :-1, :], c[:, 1:, :])
    ky[:, 0, :], ky[:, -1, :] = c[:, 0, :], c[:, -1, :]
    kz[1:-1, :, :] = hmean(c[:-1, :, :], c[1:, :, :])
    kz[0, :, :], kz[-1, :, :] = c[0, :, :], c[-1, :, :]
    diag = (kx[:, :, :-1] + kx[:, :, 1:]) + (ky[:, :-1, :] + ky[:, 1:, :]) + (kz[:-1, :, :] + kz[1:, :, :])
    offv = {
        (-1, 0, 0): -kz[:-1, :, :], (1, 0, 0): -kz[1:, :, :],
        (0, -1, 0): -ky[:, :-1, :], (0, 1, 0): -ky[:, 1:, :],
        (0, 0, -1): -kx[:, :, :-1], (0, 0, 1): -kx[:, :, 1:],
        (0, 0, 0): diag,
    }
    row_ptr, col, oid, valid = _stencil_pattern(N, 7)
    offs = _stencil_offsets(7)
    vals = np.stack([offv[o].reshape(-1) for o in offs], axis=1)
    val = vals[valid]
    A = CSRHost(N ** 3, row_ptr.astype(np.int32), col.astype(np.int32), val.astype(np.float64))
    return A, c


def band_csr(n: int, w: int) -> CSRHost:
    """Symmetric band matrix with half-bandwidth w (the paper's weak-scaling
    transform, bandL = bandU = w, nnz = (2w+1) n - w (w+1)): -1 on every
    off-diagonal position of the band, 2w + 1 on the diagonal (strictly
    diagonally dominant, hence SPD; the eigenvalues lie between 1 and the
    maximum of the Toeplitz symbol 2w + 2 - sin((w + 1/2) t) / sin(t / 2),
    about 1.43 (2w + 1) for large w). Columns ascending."""
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(i - w, 0)
    hi = np.minimum(i + w, n - 1)
    counts = hi - lo + 1
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz >= 2 ** 31:
        raise ValueError("nnz does not fit int32 row pointers")
    col = np.empty(nnz, dtype=np.int32)
    val = np.full(nnz, -1.0)
    step = 1 << 16
    for s0 in range(0, n, step):  # row blocks, to bound the temporaries
        s1 = min(n, s0 + step)
        c = counts[s0:s1]
        seg = slice(int(row_ptr[s0]), int(row_ptr[s1]))
        if np.all(c == 2 * w + 1):
            col[seg] = (lo[s0:s1, None] + np.arange(2 * w + 1)[None, :]).ravel()
        else:
            pos = np.arange(row_ptr[s0], row_ptr[s1]) - np.repeat(row_ptr[s0:s1], c)
            col[seg] = np.repeat(lo[s0:s1], c) + pos
    val[row_ptr[:-1] + (i - lo)] = float(2 * w + 1)
    return CSRHost(n, row_ptr.astype(np.int32), col, val)


def scale_first(A: CSRHost, sigma: float) -> CSRHost:
    """The paper's ill-conditioned generator: the first row and the first
    column multiplied by sigma (A' = S A S, S = diag(sigma, 1, ..., 1)); with
    sigma a power of two the scaling is exact."""
    val = A.val.copy()
    val[int(A.row_ptr[0]):int(A.row_ptr[1])] *= sigma
    val[np.flatnonzero(A.col_idx == 0)] *= sigma
    return CSRHost(A.n, A.row_ptr, A.col_idx, val)


def suitesparse_like_parts(seed: int, nnz: int, cond: float, kappa_b: float = 1e6):
    """The two factors of a SuiteSparse-shaped stand-in (only the paper's
    printed nonzero counts and condition numbers are used, Section 5.4).

    B: n = max(100, nnz // 32) rows and nnz nonzeros (up to parity): the
    graph Laplacian of a random subset of the edges of a band of the
    narrowest half-width h that holds them (so the spectrum spreads like
    that of a mesh, not of an expander), edge weights in (0, 1], plus
    delta = 2 * mean(diagonal) / kappa_b on the diagonal, then rows and
    columns permuted at random. cond(B) is about min(kappa_b, that of the
    Laplacian), and Jacobi does not remove it.

    e: integer exponents of D = diag(2^e_i), uniform in [0, E] with
    4^(E-1) = cond / min(cond, kappa_b): the part of the condition number
    that Jacobi undoes."""
    n = max(100, nnz // 32)
    m = min(max(0, (nnz - n) // 2), n * (n - 1) // 2)  # distinct off-diagonal pairs
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 0
    while n * h - h * (h + 1) // 2 < m:
        h += 1
    # the band's pairs (i, i + j), j = 1..h, numbered row by row
    j = np.arange(1, h + 1)
    counts = np.clip(n - j, 0, None)
    off = np.concatenate([[0], np.cumsum(counts)])
    pick = np.sort(rng.choice(int(off[-1]), size=m, replace=False))
    jj = np.searchsorted(off, pick, side="right")  # 1-based distance
    ii = pick - off[jj - 1]
    perm = rng.permutation(n)
    r, c = perm[ii], perm[ii + jj]
    r, c = np.minimum(r, c), np.maximum(r, c)
    v = -rng.random(m) - 2.0 ** -20
    import scipy.sparse as sp
    U = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    Bo = (U + U.T).tocsr()
    d = np.asarray(abs(Bo).sum(axis=1)).reshape(-1)
    kb = min(float(cond), float(kappa_b))
    d = d + 2.0 * d.mean() / kb
    B = (Bo + sp.diags(d)).tocsr()
    B.sort_indices()
    E = max(0, int(round(np.log2(float(cond) / kb) / 2)) + 1)
    e = rng.integers(0, E + 1, n)
    Bh = CSRHost(n, B.indptr.astype(np.int32), B.indices.astype(np.int32), B.data.astype(np.float64))
    return Bh, e


def scale_sym(A: CSRHost, e: np.ndarray) -> CSRHost:
    """D A D with D = diag(2^e_i) (exact while nothing overflows or goes subnormal)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    return CSRHost(A.n, A.row_ptr, A.col_idx, np.ldexp(A.val, e[rows] + e[A.col_idx]))


def suitesparse_like(seed: int, nnz: int, cond: float, kappa_b: float = 1e6) -> CSRHost:
    """D B D from suitesparse_like_parts: about nnz nonzeros, condition number
    about cond."""
    B, e = suitesparse_like_parts(seed, nnz, cond, kappa_b)
    return scale_sym(B, e)


# (nonzeros, condition number) pairs printed in the paper's SuiteSparse tables
# (Section 5.4), in the order printed
SUITESPARSE_LIKE = [(32399, 2.22e18), (26198, 9.00e15), (27520, 1.03e14), (1015156, 7.61e11), (1021159, 1.10e9),
                    (219024, 6.28e9), (83883, 5.64e8), (72356, 3.56e7), (1666, 3.89e6), (97707, 4.78e5),
                    (56126, 1.49e4)]

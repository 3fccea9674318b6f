"""CPU oracle of the learned preconditioner (numpy).

TEST INFRASTRUCTURE ONLY: used by the tests and never by the library. It
shares no code with the GPU path.

The preconditioner is M^-1 = G G^T + eps I with G on the lower-triangle
pattern of a 7-point operator on an N^3 grid (rows in z-y-x order). G comes
from a three-layer 3x3x3 convolutional network over per-cell features:

  features f (4 channels): ln(|a_ij| / a_ii) for the -x, -y, -z neighbour j
      (-4 where the neighbour is absent), and (number of absent neighbours) / 6
  h1 = relu(conv1(f) + b1)   16 channels
  h2 = relu(conv2(h1) + b2)  16 channels
  o  = conv3(h2) + b3        4 channels
  s_i = RN32(1 / sqrt(a_ii));  G_ii = s_i exp(clamp(o_0, -4, 4));
  G_i,j(k) = s_i o_k for the -x, -y, -z neighbour j(k) (k = 1, 2, 3)

Convolutions use zero padding; tap t = 9 (dz+1) + 3 (dy+1) + (dx+1) reads the
cell at offset (dz, dy, dx). Weights are stored [tap][out][in]. In the
network's reduced-precision form (bf16=True) the weights, the features and
the hidden activations (after relu) are rounded to bfloat16 (nearest, ties to
even) and everything is accumulated in float64 here (float32 on the GPU), so
the two agree to accumulation-order rounding.

Training loss for one system and vectors u_m: with v = A u, y = G^T v,
r = G y + eps v - u, L = mean_m |r|^2 / |u|^2; its gradient on the pattern of
G is dL/dG_ij = mean_m (2 / |u|^2) (r_i y_j + v_i (G^T r)_j).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

CIN, HID, COUT, TAPS = 4, 16, 4, 27
ABSENT = -4.0
OCLAMP = 4.0
SHAPES = [("W1", (TAPS, HID, CIN)), ("b1", (HID,)), ("W2", (TAPS, HID, HID)), ("b2", (HID,)),
          ("W3", (TAPS, COUT, HID)), ("b3", (COUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def split(p):
    out, k = {}, 0
    for name, shape in SHAPES:
        m = int(np.prod(shape))
        out[name] = np.asarray(p[k:k + m]).reshape(shape)
        k += m
    return out


def join(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def rn_bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even); returns float64."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _rows(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))


def features(A, N):
    """Per-cell input features, float64 array (N, N, N, 4)."""
    M = _rows(A)
    n = N ** 3
    d = M.diagonal()
    i = np.arange(n)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    f = np.empty((n, 4))
    for k, (step, has) in enumerate(((1, x > 0), (N, y > 0), (N * N, z > 0))):
        a = np.zeros(n)
        a[has] = np.asarray(M[i[has], i[has] - step]).reshape(-1)
        ok = has & (a != 0)
        f[:, k] = ABSENT
        f[ok, k] = np.log(np.abs(a[ok]) / d[ok])
    f[:, 3] = (7 - np.diff(A.row_ptr)) / 6.0
    return f.reshape(N, N, N, 4)


def conv(xin, W, b):
    """Zero-padded 3x3x3 convolution: x (N, N, N, Cin), W (27, Cout, Cin), b (Cout,)."""
    N = xin.shape[0]
    P = np.zeros((N + 2, N + 2, N + 2, xin.shape[3]))
    P[1:-1, 1:-1, 1:-1] = xin
    out = np.zeros((N, N, N, W.shape[1])) + b
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        sl = P[1 + dz:1 + dz + N, 1 + dy:1 + dy + N, 1 + dx:1 + dx + N]
        out += sl @ W[t].T
    return out


def conv_t(dout, W):
    """Adjoint of conv with respect to its input: sum over taps of W[t]^T dout(cell - offset)."""
    N = dout.shape[0]
    P = np.zeros((N + 2, N + 2, N + 2, dout.shape[3]))
    P[1:-1, 1:-1, 1:-1] = dout
    out = np.zeros((N, N, N, W.shape[2]))
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        sl = P[1 - dz:1 - dz + N, 1 - dy:1 - dy + N, 1 - dx:1 - dx + N]
        out += sl @ W[t]
    return out


def conv_dw(xin, dout):
    """Weight gradient: dW[t][co][ci] = sum over cells of dout[cell][co] xin[cell + offset][ci]."""
    N = xin.shape[0]
    P = np.zeros((N + 2, N + 2, N + 2, xin.shape[3]))
    P[1:-1, 1:-1, 1:-1] = xin
    dW = np.zeros((TAPS, dout.shape[3], xin.shape[3]))
    D = dout.reshape(-1, dout.shape[3])
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        sl = P[1 + dz:1 + dz + N, 1 + dy:1 + dy + N, 1 + dx:1 + dx + N].reshape(-1, xin.shape[3])
        dW[t] = D.T @ sl
    return dW


def forward(p, f, bf16=True):
    q = split(p)
    rb = rn_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3 = rb(q["W1"]), rb(q["W2"]), rb(q["W3"])
    fi = rb(f)
    pre1 = conv(fi, W1, q["b1"])
    h1 = rb(np.maximum(pre1, 0.0))
    pre2 = conv(h1, W2, q["b2"])
    h2 = rb(np.maximum(pre2, 0.0))
    o = conv(h2, W3, q["b3"])
    return dict(f=fi, pre1=pre1, h1=h1, pre2=pre2, h2=h2, o=o, W1=W1, W2=W2, W3=W3, bf16=bf16)


def backward(cache, do):
    """Parameter gradient (flat, float64) for the output gradient do (N, N, N, 4)."""
    rb = rn_bf16 if cache["bf16"] else (lambda v: np.asarray(v, dtype=np.float64))
    d3 = rb(do)
    g = {"W3": conv_dw(cache["h2"], d3), "b3": d3.reshape(-1, COUT).sum(axis=0)}
    d2 = rb(conv_t(d3, cache["W3"]) * (cache["pre2"] > 0))
    g["W2"], g["b2"] = conv_dw(cache["h1"], d2), d2.reshape(-1, HID).sum(axis=0)
    d1 = rb(conv_t(d2, cache["W2"]) * (cache["pre1"] > 0))
    g["W1"], g["b1"] = conv_dw(cache["f"], d1), d1.reshape(-1, HID).sum(axis=0)
    return join(g)


def factor(A, N, o):
    """G (CSR, rows with ascending columns) and the derivative factors of its
    entries with respect to o: returns (G, dgdo) with dgdo (n, 4)."""
    M = _rows(A)
    n = N ** 3
    d = M.diagonal()
    s = (1.0 / np.sqrt(d)).astype(np.float32).astype(np.float64)
    o = np.asarray(o, dtype=np.float64).reshape(n, 4)
    i = np.arange(n)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    oc = np.clip(o[:, 0], -OCLAMP, OCLAMP)
    gdiag = (s * np.exp(oc).astype(np.float32)).astype(np.float32).astype(np.float64)
    rows, cols, vals = [i], [i], [gdiag]
    dgdo = np.zeros((n, 4))
    dgdo[:, 0] = np.where(np.abs(o[:, 0]) < OCLAMP, gdiag, 0.0)
    for k, (step, has) in enumerate(((1, x > 0), (N, y > 0), (N * N, z > 0)), start=1):
        rows.append(i[has])
        cols.append(i[has] - step)
        vals.append((s[has] * o[has, k]).astype(np.float32).astype(np.float64))
        dgdo[has, k] = s[has]
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    G.sort_indices()
    return G, dgdo


def loss_grad(A, G, us, eps):
    """Loss and dL/dG on the pattern of G (a CSR with G's structure)."""
    M = _rows(A)
    L = 0.0
    dG = sp.csr_matrix(G.shape)
    Gc = G.tocoo()
    dvals = np.zeros(Gc.nnz)
    for u in us:
        u = np.asarray(u, dtype=np.float64)
        v = M @ u
        y = G.T @ v
        r = G @ y + eps * v - u
        q = G.T @ r
        uu = u @ u
        L += (r @ r) / uu
        dvals += (2.0 / uu) * (r[Gc.row] * y[Gc.col] + v[Gc.row] * q[Gc.col])
    m = len(us)
    dG = sp.csr_matrix((dvals / m, (Gc.row, Gc.col)), shape=G.shape)
    return L / m, dG


def do_from_dg(G, dG, dgdo, N):
    """Chain rule from dL/dG (on the pattern) to dL/do (N, N, N, 4)."""
    n = N ** 3
    i = np.arange(n)
    x, y, z = i % N, (i // N) % N, i // (N * N)
    do = np.zeros((n, 4))
    do[:, 0] = np.asarray(dG[i, i]).reshape(-1) * dgdo[:, 0]
    for k, (step, has) in enumerate(((1, x > 0), (N, y > 0), (N * N, z > 0)), start=1):
        do[has, k] = np.asarray(dG[i[has], i[has] - step]).reshape(-1) * dgdo[has, k]
    return do.reshape(N, N, N, 4)


def init_params(seed, scale=1.0):
    """He-style initialisation of the hidden layers; the output layer starts at
    zero, so the initial G is s_i on the diagonal (Jacobi's D^-1/2)."""
    rng = np.random.default_rng(seed)
    q = {}
    q["W1"] = rng.standard_normal((TAPS, HID, CIN)) * scale * np.sqrt(2.0 / (TAPS * CIN))
    q["b1"] = np.zeros(HID)
    q["W2"] = rng.standard_normal((TAPS, HID, HID)) * scale * np.sqrt(2.0 / (TAPS * HID))
    q["b2"] = np.zeros(HID)
    q["W3"] = np.zeros((TAPS, COUT, HID))
    q["b3"] = np.zeros(COUT)
    return join(q).astype(np.float32)

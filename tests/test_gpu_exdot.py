"""GPU parity of rpcg_exdot, rpcg_exdot_partial and rpcg_acc_round against the
oracle: exact modes bit-for-bit, for every launch configuration; plain mode
within the standard error bound of a floating-point dot."""

import math
import struct

import numpy as np
import pytest

from rpcg_workloads import exdot_conditioned, exdot_narrow, exdot_wide

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bits(v):
    return struct.unpack("<Q", struct.pack("<d", float(v)))[0]


def _same(a, b):
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return _bits(a) == _bits(b)


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.context(0)
    return rpcg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _case(kind, n, seed):
    if kind == "narrow":
        return exdot_narrow(seed, n)
    if kind == "wide":
        return exdot_wide(seed, n)
    cond = float(kind.split(":")[1])
    x, y, _ = exdot_conditioned(seed, max(n, 4), cond)
    return x, y


SIZES = [0, 1, 2, 3, 63, 64, 65, 255, 1000, 4097, 65539, 1 << 20]
KINDS = ["narrow", "wide", "cond:1e0", "cond:1e8", "cond:1e16", "cond:1e24", "cond:1e32"]


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
@pytest.mark.parametrize("kind", KINDS)
def test_exact_modes_bitexact(R, orc, mode, kind):
    print(f"exdot {mode} {kind}", flush=True)
    for i, n in enumerate(SIZES):
        if kind.startswith("cond") and n < 4:
            continue
        x, y = _case(kind, n, 100 + i)
        want = orc.exdot(x, y)
        out, info = R.exdot(_dev(x), _dev(y), mode=mode)
        got = out.item()
        assert _same(got, want), (mode, kind, n, got, want, info)
        assert info["status"] == 0, info


LAUNCH = [(64, 1), (64, 3), (128, 17), (256, 1), (256, 100), (512, 333), (1024, 2048), (256, 4096)]


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_launch_config_invariance(R, orc, mode):
    x, y = exdot_wide(7, 100003)
    want = orc.exdot(x, y)
    X, Y = _dev(x), _dev(y)
    for block, grid in LAUNCH:
        for p in (1, 3, 4, 8):
            print(f"exdot {mode} block={block} grid={grid} p={p}", flush=True)
            out, info = R.exdot(X, Y, mode=mode, block_size=block, grid_size=grid, fpe_size=p)
            assert _same(out.item(), want), (block, grid, p)


def test_mixed_ranges_switch_paths(R, orc):
    """Narrow, wide, narrow segments: in exblas mode each lane moves from its
    expansion to adding the products straight into the accumulator and back
    as the overflow rate changes; the result stays the exact dot for any
    launch shape (the switching points move with the shape)."""
    parts = [exdot_narrow(21, 300000), exdot_wide(22, 300000), exdot_narrow(23, 300001)]
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    want = orc.exdot(x, y)
    X, Y = _dev(x), _dev(y)
    for block, grid in ((0, 0), (64, 1), (256, 37), (1024, 1024), (512, 4096)):
        print(f"exdot mixed ranges block={block} grid={grid}", flush=True)
        out, info = R.exdot(X, Y, mode="exblas", block_size=block, grid_size=grid)
        assert _same(out.item(), want), (block, grid)


def test_fpe_escapes_and_fallback(R, orc):
    """Wide data overflows short expansions (Section 4.3 warning); with the
    fallback the result is still the exact dot, without it a warning is raised."""
    x, y = exdot_wide(3, 50000)
    want = orc.exdot(x, y)
    X, Y = _dev(x), _dev(y)
    out, info = R.exdot(X, Y, mode="fpe", fpe_size=2)
    assert info["fpe_escapes"] > 0 and info["fallbacks"] == 1 and info["status"] == 0
    assert _same(out.item(), want)
    out, info = R.exdot(X, Y, mode="fpe", fpe_size=2, fpe_fallback=0)
    assert info["status"] == R.WARN_FPE_INEXACT and info["fallbacks"] == 0
    # narrow data: no escapes at p = 4 (the PCG-like case)
    xn, yn = exdot_narrow(3, 50000)
    out, info = R.exdot(_dev(xn), _dev(yn), mode="fpe", fpe_size=4)
    assert info["fpe_escapes"] == 0 and info["fallbacks"] == 0
    assert _same(out.item(), orc.exdot(xn, yn))


def test_fpe8_holds_424_bits(R, orc):
    """Section 4.2: an expansion of eight doubles represents at least
    8 x 53 = 424 bits. Eight terms with random 53-bit significands, every
    term just below the previous one, form one 424-bit string: the merge of
    the eight products into one expansion keeps all of them at p = 8 (no
    escape, exact without the fallback) and loses one term at p = 7. (A run
    of equal bits would not do: 2^a - 2^b needs only two terms.)"""
    rng = np.random.default_rng(42)
    x = np.array([float(rng.integers(2 ** 52, 2 ** 53)) * 2.0 ** (-53 * k) for k in range(8)])
    y = np.ones(8)
    want = orc.exdot(x, y)
    X, Y = _dev(x), _dev(y)
    out, info = R.exdot(X, Y, mode="fpe", fpe_size=8, fpe_fallback=0, block_size=64, grid_size=1)
    assert info["fpe_escapes"] == 0 and info["status"] == 0
    assert _same(out.item(), want)
    out, info = R.exdot(X, Y, mode="fpe", fpe_size=7, fpe_fallback=0, block_size=64, grid_size=1)
    assert info["fpe_escapes"] >= 1 and info["status"] == R.WARN_FPE_INEXACT


def test_early_exit_changes_nothing(R, orc):
    x, y = exdot_narrow(9, 30001)
    want = orc.exdot(x, y)
    for mode in ("exblas", "fpe"):
        for ee in (0, 1):
            out, _ = R.exdot(_dev(x), _dev(y), mode=mode, early_exit=ee)
            assert _same(out.item(), want)


def test_plain_mode_error_bound(R, orc):
    """Plain fp64: |s - exact| <= gamma_n * sum|x_i y_i| (Higham's dot bound,
    n here being the depth of the summation tree, bounded by the length)."""
    for kind in ("narrow", "wide"):
        x, y = _case(kind, 200000, 5)
        exact = orc.exdot(x, y)
        absdot = orc.exdot(np.abs(x), np.abs(y))
        out, _ = R.exdot(_dev(x), _dev(y), mode="plain")
        n = x.size
        u = 2.0 ** -53
        assert abs(out.item() - exact) <= (n * u / (1 - n * u)) * absdot


def test_plain_mode_not_reproducible_across_configs(R):
    """The paper's point (Section 5.3): the regular reduction changes with the
    parallel configuration, the exact ones do not."""
    x, y, _ = exdot_conditioned(12, 1 << 18, 1e16)
    X, Y = _dev(x), _dev(y)
    vals = {R.exdot(X, Y, mode="plain", block_size=b, grid_size=g)[0].item() for b, g in LAUNCH}
    assert len(vals) > 1
    vals = {R.exdot(X, Y, mode="exblas", block_size=b, grid_size=g)[0].item() for b, g in LAUNCH}
    assert len(vals) == 1


def test_exact_domain_edges(R, orc):
    tiny = 5e-324
    # a product below 2^-969: TwoProd's error is not representable -> warning
    out, info = R.exdot(_dev(np.array([3 * tiny, 1.0])), _dev(np.array([0.5, 1.0])), mode="exblas")
    assert info["status"] == R.WARN_FPE_INEXACT
    # non-finite input -> error status and NaN
    x = np.ones(1000)
    x[17] = np.inf
    with pytest.raises(R.RpcgError) as e:
        R.exdot(_dev(x), _dev(np.ones(1000)), mode="exblas")
    assert e.value.status == R.ERR_NONFINITE
    # large cancellation and results near the top of the range stay exact
    x = np.array([2.0 ** 1000, 1.0, -(2.0 ** 1000), 2.0 ** -1000])
    y = np.array([2.0 ** 20, 1.0, 2.0 ** 20, 1.0])
    for mode in ("exblas", "fpe"):
        out, info = R.exdot(_dev(x), _dev(y), mode=mode)
        assert _same(out.item(), orc.exdot(x, y))
    # ties to even at the rounding point
    e = 2.0 ** -53
    for xs, want in (([1.0, e], 1.0), ([1.0, 3 * e], 1.0 + 2.0 ** -51), ([1.0, e, 2.0 ** -200], 1.0 + 2.0 ** -52)):
        for mode in ("exblas", "fpe"):
            out, _ = R.exdot(_dev(np.array(xs)), _dev(np.ones(len(xs))), mode=mode)
            assert out.item() == want


def test_partial_digits_equal_oracle_integer(R, orc):
    for kind, n in (("wide", 77777), ("narrow", 5000), ("cond:1e32", 10001)):
        x, y = _case(kind, n, 31)
        digits = R.exdot_partial(_dev(x), _dev(y))
        E_gpu = R.digits_to_int(digits)  # value = E_gpu * 2^-1088
        E_orc = orc.exdot_exact(x, y)    # value = E_orc * 2^-2148
        assert E_orc == E_gpu * (1 << (2148 - 1088))
        # digits are normalized (0 <= d < 2^32 below the top word)
        d = digits.cpu().numpy()
        assert np.all((d[:-1] >= 0) & (d[:-1] < 2 ** 32))
        # rounding the digits gives the exact dot
        assert _same(R.acc_round(digits).item(), orc.exdot(x, y))


def test_partial_digits_sum_across_pieces(R, orc):
    """The multi-GPU design: integer sums of per-piece digit vectors, rounded
    once, equal the dot of the whole (any split, any order)."""
    x, y = exdot_wide(44, 300000)
    X, Y = _dev(x), _dev(y)
    cuts = [0, 1, 99999, 150000, 299999, 300000]
    total = torch.zeros(68, dtype=torch.int64, device="cuda")
    for a, b in zip(cuts[:-1], cuts[1:]):
        total += R.exdot_partial(X[a:b].contiguous(), Y[a:b].contiguous())
    assert _same(R.acc_round(total).item(), orc.exdot(x, y))


def test_acc_round_random_integers(R, orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        top = int(rng.integers(0, 67))
        words = rng.integers(0, 2 ** 32, size=68, dtype=np.uint64).astype(np.int64)
        words[top + 1:] = 0
        lo = int(rng.integers(0, top + 1))
        words[:lo] = 0
        if rng.random() < 0.5:
            words[top] = -words[top] if words[top] else -1
        d = torch.from_numpy(words).to("cuda")
        E = sum(int(v) << (32 * k) for k, v in enumerate(words.tolist()))
        want = orc.round_exact(E * (1 << (2148 - 1088)))
        assert _same(R.acc_round(d).item(), want), (top, lo)


def test_large_closed_form(R):
    """At 2^24 elements the conditioned construction gives the exact dot in
    closed form; both exact modes return it for cond 1e16 and 1e32."""
    for cond in (1e16, 1e32):
        x, y, exact = exdot_conditioned(77, 1 << 24, cond)
        for mode in ("exblas", "fpe"):
            out, info = R.exdot(_dev(x), _dev(y), mode=mode)
            assert out.item() == exact, (cond, mode, info)


@pytest.mark.slow
def test_full_size_wide_exponents(R, orc):
    """The benchmark's workload at full size: 2^28 pairs with exponents
    uniform over 2^+-200 (the bench's seeds and chunks), in the launch
    configuration the bench times; both exact modes return the oracle's
    exact dot, summed over the chunks as exact integers and rounded once."""
    ne, chunk = 1 << 28, 1 << 24
    X = torch.empty(ne, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    E = 0
    for c0 in range(0, ne, chunk):
        xs, ys = exdot_wide(1000 + c0 // chunk, chunk)
        X[c0:c0 + chunk].copy_(torch.from_numpy(xs))
        Y[c0:c0 + chunk].copy_(torch.from_numpy(ys))
        E += orc.exdot_exact(xs, ys)
    want = orc.round_exact(E)
    for mode in ("exblas", "fpe"):
        print(f"exdot 2^28 wide {mode}", flush=True)
        out, info = R.exdot(X, Y, mode=mode)
        assert _same(out.item(), want), mode
    del X, Y
    torch.cuda.empty_cache()


def test_async_call_without_result(R, orc):
    x, y = exdot_narrow(2, 10000)
    out, info = R.exdot(_dev(x), _dev(y), mode="exblas", sync=False)
    assert info is None
    torch.cuda.synchronize()
    assert _same(out.item(), orc.exdot(x, y))


def _direct_edges(threads: int, seed: int):
    """Input that sends every lane of a launch with `threads` lanes into the
    direct path of the exact dot (wide-exponent products overflow the lane's
    expansion on every add for 20 element pairs per lane, i.e. more than one
    measurement window), followed, while the lanes stay direct, by the edge
    cases of that path: subnormal operands times large ones (the ex = 0
    branch), products of few significant bits below 2^-969 (added as two
    doubles, exact; they raise the inexact-domain warning), and products
    near 2^1021 that cancel (the top accumulator words)."""
    rng = np.random.default_rng(seed)
    px, py = exdot_wide(seed, 2 * 20 * threads)
    m = 2 * 40 * threads
    kind = rng.integers(0, 3, m)
    x = np.empty(m)
    y = np.empty(m)
    sub = kind == 0
    x[sub] = np.ldexp(rng.integers(1, 1 << 52, int(sub.sum())).astype(np.float64), -1074)
    y[sub] = np.ldexp(1.0 + rng.random(int(sub.sum())), rng.integers(980, 1023, int(sub.sum())))
    tiny = kind == 1
    a = rng.integers(-600, -400, int(tiny.sum()))
    b = rng.integers(-1070, -970, int(tiny.sum())) - a
    x[tiny] = np.ldexp(rng.choice([-1.0, 1.0, 3.0, -5.0], int(tiny.sum())), a)
    y[tiny] = np.ldexp(rng.choice([1.0, -1.0, 0.75], int(tiny.sum())), b)
    wide = kind == 2
    wx, wy = exdot_wide(seed + 1, int(wide.sum()))
    x[wide], y[wide] = wx, wy
    # two cancelling products of about 1.5 * 2^1021 (sum of magnitudes below 2^1023)
    hx = 1.5 * 2.0 ** 511
    x[5], y[5] = hx, 2.0 ** 510 * (1 + 2.0 ** -40)
    x[m // 2 + 7], y[m // 2 + 7] = -hx, 2.0 ** 510
    tx, ty = exdot_wide(seed + 2, 2 * 10 * threads)
    return np.concatenate([px, x, tx]), np.concatenate([py, y, ty])


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_direct_path_edge_cases(R, orc, mode):
    """The exact dot's direct path on its edge cases equals the oracle bit for
    bit under several launch shapes (each input built for its shape so that
    the edge cases reach lanes in direct mode)."""
    for grid, block in ((1, 64), (2, 128), (4, 256), (3, 1024), (0, 0)):
        threads = grid * block if grid else 1024  # default shape: sized for 1024 lanes only
        x, y = _direct_edges(threads, 300 + grid + block)
        want = orc.exdot(x, y)
        print(f"exdot direct-path edges {mode} grid={grid} block={block} n={x.size}", flush=True)
        out, info = R.exdot(_dev(x), _dev(y), mode=mode, grid_size=grid, block_size=block)
        assert _same(out.item(), want), (mode, grid, block, out.item(), want)
        assert info["status"] == R.WARN_FPE_INEXACT, info  # the tiny products
        if mode == "fpe" and grid:
            assert info["fpe_escapes"] > x.size // 4  # direct adds count as escapes

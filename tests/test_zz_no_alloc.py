"""GPU test of rpcg_exdot_noalloc, the dot-product entry point that
allocates nothing (its scratch is a static device array): it must return
what rpcg_exdot returns, bit for bit, on consecutive calls that reuse the
array, the second with a smaller input, in every mode."""

import numpy as np
import pytest
import torch

from rpcg_workloads import exdot_narrow, exdot_wide

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.lib()
    return rpcg


def _bits(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("mode", ["exblas", "fpe", "plain"])
@pytest.mark.parametrize("data", ["narrow", "wide"])
def test_noalloc_matches_exdot_on_consecutive_calls(R, mode, data):
    dev = torch.device("cuda:0")
    gen = exdot_narrow if data == "narrow" else exdot_wide
    for n, seed in ((3_000_001, 91), (40_013, 92)):  # second call smaller than the first
        print(f"noalloc {mode} {data} n={n}", flush=True)
        xh, yh = gen(seed, n)
        x, y = torch.from_numpy(xh).to(dev), torch.from_numpy(yh).to(dev)
        ref, info_ref = R.exdot(x, y, mode=mode)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        info = R.exdot_noalloc(x, y, out, mode=mode)
        assert np.array_equal(_bits(out), _bits(ref)), (mode, data, n, out.item(), ref.item())
        assert info["status"] == info_ref["status"]
        assert info["fpe_escapes"] == info_ref["fpe_escapes"]
        assert info["grid_size"] == info_ref["grid_size"]
        if mode != "plain":
            import oracle
            assert out.item() == oracle.exdot(xh, yh)


def test_noalloc_launch_shapes_and_limit(R):
    dev = torch.device("cuda:0")
    xh, yh = exdot_wide(93, 1_000_003)
    x, y = torch.from_numpy(xh).to(dev), torch.from_numpy(yh).to(dev)
    ref, _ = R.exdot(x, y, mode="exblas")
    out = torch.empty(1, dtype=torch.float64, device=dev)
    for grid, block in ((1, 64), (2048, 256), (37, 1024)):
        print(f"noalloc shape grid={grid} block={block}", flush=True)
        R.exdot_noalloc(x, y, out, mode="exblas", grid_size=grid, block_size=block)
        assert np.array_equal(_bits(out), _bits(ref)), (grid, block)
    with pytest.raises(R.RpcgError):
        R.exdot_noalloc(x, y, out, mode="exblas", grid_size=2049)
    # empty input and an asynchronous call ordered after it on the same stream
    e = torch.empty(0, dtype=torch.float64, device=dev)
    R.exdot_noalloc(e, e, out, mode="fpe")
    assert out.item() == 0.0 and not np.signbit(out.item())
    assert R.exdot_noalloc(x, y, out, mode="fpe", sync=False) is None
    torch.cuda.synchronize()
    assert np.array_equal(_bits(out), _bits(ref))

"""GPU parity of the batched solver (rpcg_batch_*): each system's iteration
count, tau history and solution are bit-identical to solving it alone
(rpcg_pcg_solve) and to the oracle, whatever the batch order, composition,
schedule or autotuner choice."""

import numpy as np
import pytest

from rpcg_workloads import (CSRHost, batch_systems, random_spd_csr, stencil27_csr, stencil7_varcoef_csr,
                            uniform_pm1)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.context(0)
    return rpcg


def _eq(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def small_batch():
    """Uneven systems: 7-point variable coefficients on 3^3..16^3 grids (ragged
    slices), a 27-point operator, a random SPD matrix."""
    systems = []
    for k, N in enumerate((5, 9, 12, 3, 16, 7)):
        A = stencil7_varcoef_csr(N, 300 + k)
        systems.append((A, uniform_pm1(400 + k, A.n)))
    A = stencil27_csr(6)
    systems.append((A, uniform_pm1(410, A.n)))
    A = random_spd_csr(29, 11)
    systems.append((A, uniform_pm1(411, A.n)))
    return systems


@pytest.fixture(scope="module")
def sb(orc):
    systems = small_batch()
    refs = [orc.pcg(A, b, tol=1e-10, maxit=3000) for A, b in systems]
    for r in refs:
        assert r["status"] == 0
    return systems, refs


def _run(R, systems, mode="exblas", tuning=None, tol=1e-10, maxit=3000, history=True, **opts):
    mats = [R.CSR.from_host(A) for A, _ in systems]
    bs = [torch.from_numpy(b).cuda() for _, b in systems]
    B = R.Batch(mats, mode=mode, tol=tol, maxit=maxit, **opts)
    if tuning:
        B.set_tuning(**tuning)
    xs, infos, stats = B.solve(bs, history=history, raise_on_error=False)
    B.close()
    return [x.cpu().numpy() for x in xs], infos, stats


def _check(infos, xs, refs, idx=None):
    idx = range(len(refs)) if idx is None else idx
    for k, j in enumerate(idx):
        assert infos[k]["status"] == refs[j]["status"], j
        assert infos[k]["iterations"] == refs[j]["iters"], j
        assert _eq(infos[k]["hist"].numpy(), refs[j]["hist"]), j
        assert _eq(xs[k], refs[j]["x"]), j


@pytest.mark.parametrize("mode", ["exblas", "fpe"])
def test_batch_matches_oracle(R, sb, mode):
    systems, refs = sb
    print(f"batch of {len(systems)} systems, {mode}", flush=True)
    xs, infos, stats = _run(R, systems, mode)
    _check(infos, xs, refs)
    assert stats["status"] == 0 and stats["max_iterations"] == max(r["iters"] for r in refs)
    assert stats["total_iterations"] == sum(r["iters"] for r in refs)


def test_batch_matches_solo_solves(R, sb):
    systems, refs = sb
    xs, infos, _ = _run(R, systems)
    for k, (A, b) in enumerate(systems):
        x1, i1 = R.pcg_solve(R.CSR.from_host(A), torch.from_numpy(b).cuda(), tol=1e-10, maxit=3000)
        assert i1["iterations"] == infos[k]["iterations"]
        assert _eq(i1["hist"].numpy(), infos[k]["hist"].numpy())
        assert _eq(x1.cpu().numpy(), xs[k])


def test_batch_order_and_composition(R, sb):
    systems, refs = sb
    order = [4, 0, 7, 2, 6, 1]
    print("batch reordered subset", order, flush=True)
    xs, infos, _ = _run(R, [systems[j] for j in order])
    _check(infos, xs, refs, order)
    xs, infos, _ = _run(R, [systems[5]])
    _check(infos, xs, refs, [5])


TUNINGS = [
    dict(policy=0, grid_size=1, block_size=64, graph_iterations=1),
    dict(policy=0, grid_size=7, block_size=1024, graph_iterations=5),
    dict(policy=0, grid_size=3000, block_size=256, graph_iterations=8),
    dict(policy=1, tile_slices=1, grid_size=5, block_size=128, graph_iterations=3),
    dict(policy=1, tile_slices=3, grid_size=300, block_size=512, graph_iterations=64),
    dict(policy=1, tile_slices=1000, grid_size=2, block_size=256, graph_iterations=2),
]


def test_batch_schedules_do_not_change_results(R, sb):
    systems, refs = sb
    for t in TUNINGS:
        print("batch tuning", t, flush=True)
        xs, infos, _ = _run(R, systems, tuning=t)
        _check(infos, xs, refs)


def test_batch_autotuner(R, sb):
    systems, refs = sb
    mats = [R.CSR.from_host(A) for A, _ in systems]
    bs = [torch.from_numpy(b).cuda() for _, b in systems]
    B = R.Batch(mats, tol=1e-10, maxit=3000)
    t = B.tune(bs, trial_iterations=5)
    print("autotuner chose", t, flush=True)
    assert t["ms_per_iteration"] > 0 and t["policy"] in (0, 1)
    xs, infos, _ = B.solve(bs)
    _check(infos, [x.cpu().numpy() for x in xs], refs)
    # a second solve replays the captured graph; without histories it is recaptured
    xs2, infos2, _ = B.solve(bs, history=False)
    for k in range(len(refs)):
        assert _eq(xs2[k].cpu().numpy(), refs[k]["x"]) and infos2[k]["iterations"] == refs[k]["iters"]
    xs3, infos3, _ = B.solve(bs)
    _check(infos3, [x.cpu().numpy() for x in xs3], refs)
    B.close()
    # a new batch of the same sizes starts from the recorded tuning
    B2 = R.Batch(mats, tol=1e-10, maxit=3000)
    got = B2.tuning
    B2.close()
    assert all(got[k] == t[k] for k in ("policy", "tile_slices", "grid_size", "block_size"))


def test_batch_statuses_per_system(R, orc):
    A = stencil7_varcoef_csr(6, 21)
    b = uniform_pm1(22, A.n)
    bad = CSRHost(A.n, A.row_ptr, A.col_idx, np.where(A.val > 0, -A.val, A.val))
    bn = b.copy()
    bn[4] = np.nan
    empty = CSRHost(0, np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0))
    systems = [(A, b), (bad, b), (A, np.zeros(A.n)), (A, bn), (empty, np.zeros(0)), (A, b)]
    xs, infos, stats = _run(R, systems, tol=1e-10, maxit=3000)
    ref = orc.pcg(A, b, tol=1e-10, maxit=3000)
    for k in (0, 5):
        assert infos[k]["status"] == 0 and infos[k]["iterations"] == ref["iters"] and _eq(xs[k], ref["x"])
    assert infos[1]["status"] == R.ERR_NOT_SPD
    assert infos[2]["status"] == 0 and infos[2]["iterations"] == 0 and not xs[2].any()
    assert infos[3]["status"] == R.ERR_NONFINITE
    assert infos[4]["status"] == 0 and infos[4]["iterations"] == 0
    assert stats["status"] == R.ERR_NONFINITE  # the lowest error


def test_batch_maxit_and_plain(R, sb, orc):
    systems, refs = sb
    xs, infos, stats = _run(R, systems, maxit=7)
    for k, (A, b) in enumerate(systems):
        r = orc.pcg(A, b, tol=1e-10, maxit=7)
        assert infos[k]["iterations"] == r["iters"] and _eq(xs[k], r["x"])
        assert infos[k]["status"] == (R.WARN_MAXIT if r["iters"] == 7 else 0)
    xs, infos, stats = _run(R, systems, mode="plain")
    for k, (A, b) in enumerate(systems):
        assert infos[k]["status"] == 0
        assert abs(infos[k]["iterations"] - refs[k]["iters"]) <= 3
        assert orc.relres_true(A, b, xs[k]) < 1e-9


@pytest.mark.slow
def test_batch_64_systems(R, orc):
    """The batched workload (64 systems, grids 16^3..96^3, seed 7): sampled
    systems are bit-identical to their solo solves, the smallest to the oracle."""
    systems = batch_systems(7)
    print("batch 64: solving", flush=True)
    xs, infos, stats = _run(R, [(A, b) for _, A, b in systems])
    assert stats["status"] == 0
    sizes = [N for N, _, _ in systems]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 3, 40})
    for k in pick:
        N, A, b = systems[k]
        print(f"batch 64: solo check of system {k} (N={N})", flush=True)
        x1, i1 = R.pcg_solve(R.CSR.from_host(A), torch.from_numpy(b).cuda(), tol=1e-10, maxit=3000)
        assert i1["iterations"] == infos[k]["iterations"]
        assert _eq(i1["hist"].numpy(), infos[k]["hist"].numpy())
        assert _eq(x1.cpu().numpy(), xs[k])
    k = int(np.argmin(sizes))
    ref = orc.pcg(systems[k][1], systems[k][2], tol=1e-10, maxit=3000)
    assert infos[k]["iterations"] == ref["iters"] and _eq(xs[k], ref["x"])

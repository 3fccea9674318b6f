"""GPU checks of the learned preconditioner against the CPU oracle
(oracle/lpnet.py): network outputs, loss and output gradient, parameter
gradient (tolerances: the two sides round to bfloat16 at the same points and
differ in accumulation order); G invariant to the batch it is computed in;
training steps reproducible; the preconditioned solve with the network's G
bit-identical to the oracle given G."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import lpnet
from rpcg_workloads import CSRHost, grf_diffusion_csr, uniform_pm1

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_07282_amd import rpcg
    rpcg.context(0)
    return rpcg


def params(seed, w3=0.05):
    rng = np.random.default_rng(seed)
    q = lpnet.split(lpnet.init_params(seed).astype(np.float64))
    q["W3"] = rng.standard_normal(q["W3"].shape) * w3
    q["b1"] = rng.standard_normal(16) * 0.1
    q["b2"] = rng.standard_normal(16) * 0.1
    q["b3"] = rng.standard_normal(4) * 0.1
    return lpnet.join(q).astype(np.float32)


def systems(N, seeds):
    return [grf_diffusion_csr(N, s)[0] for s in seeds]


@pytest.fixture(scope="module")
def net10(R):
    net = R.LearnedPreconditioner(10, max_batch=3)
    net.set_params(params(1))
    return net


def test_forward_matches_oracle(R, net10):
    N = 10
    As = systems(N, [11, 12])
    o = net10.forward([R.CSR.from_host(A) for A in As]).cpu().numpy()
    p = params(1).astype(np.float64)
    for k, A in enumerate(As):
        ref = lpnet.forward(p, lpnet.features(A, N), bf16=True)["o"].reshape(-1, 4)
        scale = np.abs(ref).max()
        err = np.abs(o[k] - ref)
        print(f"forward system {k}: max |diff| / max |o| = {err.max() / scale:.2e}, "
              f"elements off by > 1e-3 relative: {np.mean(err > 1e-3 * scale):.4f}", flush=True)
        assert err.max() <= 3e-2 * scale
        assert np.mean(err > 1e-3 * scale) < 0.01


@pytest.mark.parametrize("nu", [2, 4, 9])
def test_loss_grad_matches_oracle(R, net10, nu):
    """Loss and dL/do against the oracle; nu = 4 takes the device's
    four-vector path, 2 and 9 the general one (9: two passes of eight and one
    over the interleaved vectors)."""
    N = 10
    As = systems(N, [13])
    mats = [R.CSR.from_host(A) for A in As]
    us = [[uniform_pm1(30 + m, As[0].n) for m in range(nu)]]
    ud = [[torch.from_numpy(u).cuda() for u in row] for row in us]
    loss, dout = net10.loss_grad(mats, ud, eps=1e-6)
    o = net10.forward(mats).cpu().numpy()[0]
    G, dgdo = lpnet.factor(As[0], N, o)
    L, dG = lpnet.loss_grad(As[0], G, us[0], 1e-6)
    do = lpnet.do_from_dg(G, dG, dgdo, N).reshape(-1, 4)
    print(f"nu={nu}: loss gpu {loss:.12g} oracle {L:.12g}", flush=True)
    # the exponential of the diagonal output is the only step not correctly
    # rounded on both sides (last-bit differences of G_ii)
    assert abs(loss - L) <= 1e-6 * abs(L)
    d = dout.cpu().numpy()[0]
    print(f"dL/do: max |diff| / max = {np.max(np.abs(d - do)) / np.max(np.abs(do)):.2e}", flush=True)
    assert np.max(np.abs(d - do)) <= 1e-5 * np.max(np.abs(do))


def test_backward_matches_oracle(R, net10):
    N = 10
    As = systems(N, [14, 15])
    mats = [R.CSR.from_host(A) for A in As]
    rng = np.random.default_rng(5)
    dout = rng.standard_normal((2, N ** 3, 4))
    g = net10.backward(mats, torch.from_numpy(dout).cuda()).cpu().numpy().astype(np.float64)
    p = params(1).astype(np.float64)
    ref = np.zeros(lpnet.NPARAMS)
    for k, A in enumerate(As):
        c = lpnet.forward(p, lpnet.features(A, N), bf16=True)
        ref += lpnet.backward(c, dout[k].reshape(N, N, N, 4))
    off = 0
    for name, shape in lpnet.SHAPES:
        m = int(np.prod(shape))
        a, b = g[off:off + m], ref[off:off + m]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"gradient {name}: relative difference {rel:.2e}", flush=True)
        assert rel < 2e-2, name
        off += m


def test_forward_backward_ragged_blocks(R):
    """N = 21 cuts the kernels' tiles raggedly: forward and adjoint passes
    take one full and one 5-cell tile along x, y-groups of 4 lines with a
    remainder and z-runs of 16 + 5 planes; the weight gradient one 32-cell
    x-segment holding 21 cells; halos on every side."""
    N = 21
    net = R.LearnedPreconditioner(N, max_batch=2)
    net.set_params(params(3))
    As = systems(N, [31, 32])
    mats = [R.CSR.from_host(A) for A in As]
    o = net.forward(mats).cpu().numpy()
    p = params(3).astype(np.float64)
    rng = np.random.default_rng(9)
    dout = rng.standard_normal((2, N ** 3, 4))
    g = net.backward(mats, torch.from_numpy(dout).cuda()).cpu().numpy().astype(np.float64)
    net.close()
    ref_g = np.zeros(lpnet.NPARAMS)
    for k, A in enumerate(As):
        c = lpnet.forward(p, lpnet.features(A, N), bf16=True)
        ref = c["o"].reshape(-1, 4)
        scale = np.abs(ref).max()
        err = np.abs(o[k] - ref)
        print(f"N=21 forward system {k}: max |diff| / max |o| = {err.max() / scale:.2e}", flush=True)
        assert err.max() <= 3e-2 * scale
        assert np.mean(err > 1e-3 * scale) < 0.01
        ref_g += lpnet.backward(c, dout[k].reshape(N, N, N, 4))
    off = 0
    for name, shape in lpnet.SHAPES:
        m = int(np.prod(shape))
        rel = np.linalg.norm(g[off:off + m] - ref_g[off:off + m]) / np.linalg.norm(ref_g[off:off + m])
        print(f"N=21 gradient {name}: relative difference {rel:.2e}", flush=True)
        assert rel < 2e-2, name
        off += m


def test_weight_gradient_two_segments(R):
    """N = 37: the weight gradient's x-segments of 32 cells are one full and
    one of 5 cells, so the staged x halo crosses a segment boundary."""
    N = 37
    net = R.LearnedPreconditioner(N, max_batch=1)
    net.set_params(params(4))
    A = systems(N, [33])[0]
    mats = [R.CSR.from_host(A)]
    rng = np.random.default_rng(11)
    dout = rng.standard_normal((1, N ** 3, 4))
    g = net.backward(mats, torch.from_numpy(dout).cuda()).cpu().numpy().astype(np.float64)
    net.close()
    p = params(4).astype(np.float64)
    c = lpnet.forward(p, lpnet.features(A, N), bf16=True)
    ref = lpnet.backward(c, dout[0].reshape(N, N, N, 4))
    off = 0
    for name, shape in lpnet.SHAPES:
        m = int(np.prod(shape))
        rel = np.linalg.norm(g[off:off + m] - ref[off:off + m]) / np.linalg.norm(ref[off:off + m])
        print(f"N=37 gradient {name}: relative difference {rel:.2e}", flush=True)
        assert rel < 2e-2, name
        off += m


def test_loss_grad_batch_above_16(R):
    """18 systems x 3 vectors in one call (the matrix table holds more than
    the 16 matrices one feature launch takes) give the per-system losses and
    output gradients: the batch loss is their mean, each system's gradient
    its own divided by the batch size (to rounding: the scale factors and
    the order of the loss sum differ)."""
    N = 6
    nb, nu = 18, 3
    net = R.LearnedPreconditioner(N, max_batch=nb)
    net.set_params(params(5))
    As = systems(N, list(range(60, 60 + nb)))
    mats = [R.CSR.from_host(A) for A in As]
    us = [[torch.from_numpy(uniform_pm1(500 + 7 * k + m, As[0].n)).cuda() for m in range(nu)] for k in range(nb)]
    loss, dout = net.loss_grad(mats, us, eps=1e-6)
    losses = []
    for k in range(nb):
        lk, dk = net.loss_grad([mats[k]], [us[k]], eps=1e-6)
        losses.append(lk)
        a, b = dout[k].cpu().numpy(), dk[0].cpu().numpy() / nb
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), k
    net.close()
    ref = float(np.mean(losses))
    print(f"batch loss {loss:.15g}, mean of per-system losses {ref:.15g}", flush=True)
    assert abs(loss - ref) <= 1e-12 * abs(ref)


def test_lp_limits(R):
    """Batches beyond what the kernels' grids index are rejected up front."""
    with pytest.raises(R.RpcgError) as ei:
        R.LearnedPreconditioner(2, max_batch=70000)
    assert ei.value.status == R.ERR_INVALID
    N = 4
    net = R.LearnedPreconditioner(N, max_batch=2)
    A = systems(N, [70])[0]
    mats = [R.CSR.from_host(A)]
    u = torch.from_numpy(uniform_pm1(3, A.n)).cuda()
    with pytest.raises(R.RpcgError) as ei:
        net.loss_grad(mats, [[u] * 65536])
    assert ei.value.status == R.ERR_INVALID
    net.close()


def test_factor_independent_of_batch(R, net10):
    N = 10
    As = systems(N, [16, 17, 18])
    mats = [R.CSR.from_host(A) for A in As]
    together = net10.factor(mats)
    alone = net10.factor([mats[1]])[0]
    G1, Gt1 = together[1]
    assert torch.equal(G1.val, alone[0].val) and torch.equal(Gt1.val, alone[1].val)
    # G^T is the transpose of G, entry for entry
    grp, gcol, gtrp, gtcol = net10.pattern
    Gs = sp.csr_matrix((G1.val.cpu().numpy(), gcol, grp), shape=(N ** 3, N ** 3))
    Gts = sp.csr_matrix((Gt1.val.cpu().numpy(), gtcol, gtrp), shape=(N ** 3, N ** 3))
    assert (Gs.T != Gts).nnz == 0


def test_forward_large_batch_and_bad_diagonal(R):
    """Batches above one launch's 16 matrices give the outputs of the systems
    alone; a non-positive diagonal is reported, and a later good batch is
    not affected by the earlier report."""
    N = 6
    net = R.LearnedPreconditioner(N, max_batch=18)
    net.set_params(params(3))
    As = systems(N, list(range(40, 58)))
    mats = [R.CSR.from_host(A) for A in As]
    together = net.forward(mats).cpu()
    for k in (0, 15, 16, 17):
        alone = net.forward([mats[k]]).cpu()[0]
        assert torch.equal(together[k], alone), k
    bad = As[5]
    val = bad.val.copy()
    rows = np.repeat(np.arange(bad.n), np.diff(bad.row_ptr))
    val[np.flatnonzero(bad.col_idx == rows)[7]] = -1.0
    badm = R.CSR.from_host(CSRHost(bad.n, bad.row_ptr, bad.col_idx, val))
    with pytest.raises(R.RpcgError) as ei:
        net.forward(mats[:17] + [badm])
    assert ei.value.status == R.ERR_NOT_SPD
    again = net.forward(mats).cpu()
    assert torch.equal(again, together)


def test_training_reproducible_and_learning(R):
    N = 12
    As = systems(N, [21, 22, 23, 24])
    mats = [R.CSR.from_host(A) for A in As]
    us = []
    for k, A in enumerate(As):
        # Krylov vectors: early Jacobi-PCG iterates of a random right-hand side
        b = torch.from_numpy(uniform_pm1(40 + k, A.n)).cuda()
        row = []
        for it in (3, 10):
            x, _ = R.pcg_solve(mats[k], b, mode="exblas", maxit=it, tol=1e-14, history=False, raise_on_error=False)
            row.append(x)
        us.append(row)
    runs = []
    for rep in range(2):
        net = R.LearnedPreconditioner(N, max_batch=4, params=lpnet.init_params(3))
        losses = [net.train_step(mats, us, lr=1e-3) for _ in range(30)]
        runs.append((losses, net.get_params()))
        net.close()
    (l1, p1), (l2, p2) = runs
    print("loss", l1[0], "->", l1[-1], flush=True)
    assert l1 == l2 and np.array_equal(p1, p2)  # fixed-order reductions: bit-reproducible training
    assert l1[-1] < 0.5 * l1[0]


def test_solve_with_network_factor_bitexact(R, orc, net10):
    N = 10
    A = systems(N, [19])[0]
    (G, Gt), = net10.factor([R.CSR.from_host(A)])
    grp, gcol, gtrp, gtcol = net10.pattern
    Gh = CSRHost(N ** 3, grp, gcol, G.val.cpu().numpy())
    Gth = CSRHost(N ** 3, gtrp, gtcol, Gt.val.cpu().numpy())
    b = uniform_pm1(50, A.n)
    ref = orc.pcg_factored(A, Gh, Gth, 1e-6, b, tol=1e-10, maxit=3000)
    x, info = R.pcg_solve_factored(R.CSR.from_host(A), G, Gt, 1e-6, torch.from_numpy(b).cuda(), tol=1e-10,
                                   maxit=3000, raise_on_error=False)
    assert info["status"] == ref["status"] and info["iterations"] == ref["iters"]
    assert np.array_equal(info["hist"].numpy(), ref["hist"])
    assert np.array_equal(x.cpu().numpy(), ref["x"])


def test_factored_solve_64_cube_large_grids(R, orc):
    """The factored iteration at 64^3 (262,144 rows) with the network's G,
    first five iterations against the oracle, with vector-kernel grids
    larger than the chip holds at once."""
    N = 64
    net = R.LearnedPreconditioner(N, max_batch=1)
    net.set_params(params(1))
    A = systems(N, [23])[0]
    (G, Gt), = net.factor([R.CSR.from_host(A)])
    grp, gcol, gtrp, gtcol = net.pattern
    Gh = CSRHost(N ** 3, grp, gcol, G.val.cpu().numpy())
    Gth = CSRHost(N ** 3, gtrp, gtcol, Gt.val.cpu().numpy())
    b = uniform_pm1(51, A.n)
    ref = orc.pcg_factored(A, Gh, Gth, 1e-6, b, tol=1e-10, maxit=5)
    for grid, block in ((0, 0), (2048, 512), (4096, 256)):
        print(f"factored 64^3 maxit=5 grid={grid} block={block}", flush=True)
        x, info = R.pcg_solve_factored(R.CSR.from_host(A), G, Gt, 1e-6, torch.from_numpy(b).cuda(), tol=1e-10,
                                       maxit=5, raise_on_error=False, grid_size=grid, block_size=block)
        assert info["iterations"] == ref["iters"], (grid, block)
        assert np.array_equal(info["hist"].numpy(), ref["hist"]), (grid, block)
        assert np.array_equal(x.cpu().numpy(), ref["x"]), (grid, block)
    net.close()


@pytest.mark.slow
def test_trained_network_beats_jacobi(R):
    """The committed parameters (trained on 2,000 instances of 64^3) against
    Jacobi on held-out instances: fewer exact-dot PCG iterations to 1e-10, the
    same solution to 1e-8."""
    from paper_2005_07282_amd import learned
    ev = learned.Dataset(R, torch, 64, [learned.EVAL_SEED0 + 150 + k for k in range(4)], torch.device("cuda:0"))
    net = R.LearnedPreconditioner(64, max_batch=1, params=learned.load_params())
    rows = learned.evaluate(R, torch, net, ev)
    net.close()
    for r in rows:
        print("held-out: Jacobi", r["jacobi_it"], "learned", r["learned_it"], flush=True)
        assert r["status"] == (0, 0)
        assert r["learned_it"] < 0.8 * r["jacobi_it"]
        assert r["max_rel_diff"] < 1e-8

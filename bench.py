"""Benchmark: reproducible Jacobi-PCG iterations/s and exact-dot GB/s on one MI355X.

A step is one PCG iteration (SpMV + <d,w>, the three updates with the
Jacobi preconditioner and the two fused dots, the direction update) on the
27-point Poisson operator of a 160^3 grid (n = 4,096,000, nnz = 109,215,352,
fp64 CSR), exact-dot ("exblas") mode, inputs resident in HBM. The plain-fp64
and FPE modes and the standalone exact dot (2^28-element vector pairs with
exponents uniform over 2^-200..2^200, and U[-1,1) pairs) are measured beside
it in the same run; the CPU oracle is timed on a bounded sample.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reproducible PCG iters/s + exdot GB/s (%HBM peak) vs plain fp64, 160^3 27-pt"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def k1_bytes(n, nnz):
    """Algorithmic bytes of one SpMV+dot launch: val and col (12 per entry),
    row pointers 4(n+1), the direction vector read once (8n), w written (8n)."""
    return 12 * nnz + 4 * (n + 1) + 16 * n


K1_SOURCES = ("pcg_spmv_dot.hip", "sell_spmv.hpp", "reduce.hpp", "numerics.hpp", "kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pcg_160cube_hbm_traffic.md")
# the timed loop brackets the SpMV+dot launch of every 4th iteration with HIP
# events (the kernel's mean duration over those launches; fewer events in the loop)
K1_TIMING_STRIDE = 4


def k1_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in K1_SOURCES:
        with open(os.path.join(ROOT, "paper_2005_07282_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def k1_traffic():
    """HBM bytes per SpMV+dot launch from the committed counter summary, or None
    if it is missing or was taken on different kernel sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("k_pcg_spmv_dot source_hash="):
            kv = dict(tok.split("=", 1) for tok in line.split()[1:])
            if kv.get("source_hash") == k1_source_hash():
                return int(kv["traffic_bytes"])
    return None


def time_spmv(rpcg, torch, Ad, n, nnz, reps=20, prepared=False):
    """The exported SpMV on the caller's CSR (rpcg_spmv), or with
    prepared=True on a prepared sliced-ELL copy (rpcg_smat_spmv; the copy's
    creation timed once, apart): median of reps event-timed calls against
    the CSR algorithmic bytes 12 nnz + 4 (n+1) + 8 n (x read once) + 8 n (y
    written)."""
    import numpy as np
    dev = Ad.row_ptr.device
    x = torch.ones(n, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    extra = {}
    if prepared:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = rpcg.PreparedMatrix(Ad)
        extra["create_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        call, name = (lambda: M.spmv(x, y)), "k_sell_spmv (rpcg_smat_spmv)"
    else:
        M = None
        call, name = (lambda: rpcg.spmv(Ad, x, y)), "k_spmv_csr (rpcg_spmv)"
    for _ in range(5):
        call()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    if M is not None:
        M.close()
    tm = float(np.median(times))
    byt = 12 * nnz + 4 * (n + 1) + 16 * n
    gbs = byt / (tm * 1e-3) / 1e9
    del x, y
    return {"kernel": name, "ms": round(tm, 5), "bytes": byt, "GB_s": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), **extra}


def iteration_bytes(n, nnz):
    """Algorithmic bytes of one fused PCG iteration (three kernels): K1, then
    K2 reading w, r, dinv and writing r, z (40 n), then K3 reading d, z, x
    and writing d, x (40 n): 12 nnz + 4 (n+1) + 96 n."""
    return k1_bytes(n, nnz) + 40 * n + 40 * n


def measure_stream_read(torch, dev, nbytes=2 << 30, reps=10):
    """Read bandwidth of a plain streaming reduction on this GPU (torch's own
    sum kernel over one binary64 vector of nbytes), as a measured ceiling
    beside the nominal HBM peak: bytes / fastest of reps timed calls."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    torch.sum(x)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.sum(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x
    torch.cuda.empty_cache()
    return nbytes / (best * 1e-3) / 1e9


def run_mixed_precision(N, rpcg, torch, dev):
    """Mixed-precision refinement on the 27-point operator of an N^3 grid
    (binary32 inner Jacobi-PCG to 1e-4 with exact binary32 dots, binary64
    exact residual and update, to 1e-10 relative residual) against plain and
    exact-dot binary64 PCG to the same tolerance, every solve end to end."""
    import numpy as np
    from rpcg_workloads import stencil27_csr, stencil27_rhs_from_int52, uniform_pm1_int52
    log(f"[bench] mixed precision: generating 27-point operator on {N}^3")
    A = stencil27_csr(N)
    K = uniform_pm1_int52(2, A.n)
    b = stencil27_rhs_from_int52(N, K)
    xs = K * 2.0 ** -52
    del K
    n, nnz = A.n, A.nnz
    Ad = rpcg.CSR.from_host(A, dev)
    bd = torch.from_numpy(b).to(dev)
    del A
    tol = 1e-10

    def true_rr(x):
        # exact <r,r> of r = b - A x (rows summed exactly): a refinement call with no correction step
        _, i = rpcg.ir_solve(Ad, bd, x, tol=tol, maxit=0, history=False, raise_on_error=False)
        return i["rr0"]

    bb = float(rpcg.exdot(bd, bd)[0].item())
    log("[bench] mixed precision: warmup")
    rpcg.ir_solve(Ad, bd, tol=tol, maxit=1, maxit_inner=5, history=False, raise_on_error=False)
    rpcg.pcg_solve(Ad, bd, mode="plain", tol=tol, maxit=5, history=False, raise_on_error=False)
    out = {"workload": f"27-point Poisson {N}^3 (n={n}, nnz={nnz}), b = A x*, x* ~ U[-1,1) seed 2, x0 = 0, "
                       f"relative residual 1e-10",
           "inner": "binary32 Jacobi-PCG, exact binary32 dots (exblas), tol 1e-4"}
    sol = {}
    for mode in ("plain", "exblas"):
        log(f"[bench] mixed precision: binary64 {mode} PCG to {tol}")
        torch.cuda.synchronize()
        x, info = rpcg.pcg_solve(Ad, bd, mode=mode, tol=tol, maxit=6000, history=False, timing=1)
        torch.cuda.synchronize()
        sol[mode] = x
        ms = info["setup_ms"] + info["loop_ms"]
        out[f"fp64_{mode}"] = {"iterations": info["iterations"], "solve_ms": round(ms, 2),
                               "setup_ms": round(info["setup_ms"], 2),
                               "ms_per_iteration": round(info["loop_ms"] / max(1, info["iterations"]), 5),
                               "k_spmv_dot_ms": round(info["k_spmv_dot_ms"] / max(1, info["k_launches"]), 5),
                               "true_relres": float(np.sqrt(true_rr(x) / bb))}
        log(f"[bench]   {info['iterations']} it, {ms:.1f} ms")
    log("[bench] mixed precision: refinement")
    torch.cuda.synchronize()
    x, info = rpcg.ir_solve(Ad, bd, mode="exblas", tol=tol, tol_inner=1e-4, history=True)
    torch.cuda.synchronize()
    _, it = rpcg.ir_solve(Ad, bd, mode="exblas", tol=tol, tol_inner=1e-4, history=False, timing=1)
    xe = sol["exblas"]
    scale = float(xe.abs().max())
    xs_d = torch.from_numpy(xs).to(dev)
    inner_it = max(1, it["k_launches"])
    k1_32 = it["k_spmv_dot_ms"] / inner_it
    k1_32_bytes = 8 * nnz + 4 * (n + 1) + 8 * n  # CSR with binary32 values: val + col, row pointers, d, w
    out["refinement"] = {
        "outer": info["outer"], "inner_iterations": info["inner_iterations"],
        "solve_ms": round(info["total_ms"], 2), "setup_ms": round(info["setup_ms"], 2),
        "inner_ms": round(info["inner_ms"], 2), "outer_ms": round(info["outer_ms"], 2),
        "rr_history": [float(v) for v in info["rr_hist"].tolist()],
        "true_relres": float(np.sqrt(info["rr_final"] / bb)),
        "max_rel_diff_vs_fp64_exblas": float((x - xe).abs().max()) / scale,
        "max_abs_err_vs_x_star": float((x - xs_d).abs().max()),
        "inner_ms_per_iteration": round((it["k_spmv_dot_ms"] + it["k_update_ms"] + it["k_direction_ms"])
                                        / inner_it, 5),
        "inner_k_spmv_dot_ms": round(k1_32, 5),
        "inner_k_spmv_dot_GB_s": round(k1_32_bytes / (k1_32 * 1e-3) / 1e9, 1),
        "k_residual_ms_per_step": round(it["k_residual_ms"] / max(1, it["outer"] + 1), 4),
    }
    out["fp64_exblas"]["max_abs_err_vs_x_star"] = float((xe - xs_d).abs().max())
    out["speedup_vs_fp64_plain"] = round(out["fp64_plain"]["solve_ms"] / info["total_ms"], 3)
    out["speedup_vs_fp64_exblas"] = round(out["fp64_exblas"]["solve_ms"] / info["total_ms"], 3)
    log(f"[bench]   refinement: {info['outer']} outer, {info['inner_iterations']} inner, "
        f"{info['total_ms']:.1f} ms; speedup vs plain fp64 {out['speedup_vs_fp64_plain']}")
    del Ad, bd, sol, x, xe, xs_d
    torch.cuda.empty_cache()
    return out


def run_batched(seed, rpcg, torch, dev):
    """64 independent 7-point variable-coefficient systems on N^3 grids, N
    uniform in 16..96, exact dots, tol 1e-8: one batched solve (autotuned
    schedule, captured iteration graphs) against the same systems solved one
    after another with rpcg_pcg_solve."""
    from rpcg_workloads import batch_systems
    log(f"[bench] batched: generating 64 systems (seed {seed})")
    systems = batch_systems(seed)
    mats = [rpcg.CSR.from_host(A, dev) for _, A, _ in systems]
    bs = [torch.from_numpy(b).to(dev) for _, _, b in systems]
    rows = [A.n for _, A, _ in systems]
    nnz = [A.nnz for _, A, _ in systems]
    tol, maxit = 1e-8, 2000
    torch.cuda.synchronize()
    t = time.perf_counter()
    B = rpcg.Batch(mats, mode="exblas", tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t) * 1e3
    log("[bench] batched: autotuning")
    tuning = B.tune(bs, trial_iterations=10)
    log(f"[bench]   chose {tuning}")
    B.solve(bs, history=False)  # warm-up (graph capture)
    torch.cuda.synchronize()
    t = time.perf_counter()
    xs, infos, st = B.solve(bs, history=False)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t) * 1e3
    log(f"[bench]   batched solve {batch_ms:.1f} ms, {st['total_iterations']} iterations in total")
    solo_ms = 0.0
    same = 0
    rpcg.pcg_solve(mats[0], bs[0], mode="exblas", tol=tol, maxit=maxit, history=False)
    for k in range(len(mats)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x1, i1 = rpcg.pcg_solve(mats[k], bs[k], mode="exblas", tol=tol, maxit=maxit, history=False)
        torch.cuda.synchronize()
        solo_ms += (time.perf_counter() - t) * 1e3
        same += int(i1["iterations"] == infos[k]["iterations"] and torch.equal(x1, xs[k]))
    B.close()
    row_it = sum(r * i["iterations"] for r, i in zip(rows, infos))
    # algorithmic bytes of one iteration of a system (as for the single solve): 12 nnz + 4 (n+1) + 104 n
    it_bytes = sum((12 * z + 4 * (r + 1) + 104 * r) * i["iterations"] for r, z, i in zip(rows, nnz, infos))
    out = {
        "workload": f"64 systems, 7-point diffusion with exp(N(0,1)) face coefficients on N^3 grids, N uniform "
                    f"in 16..96 (seed {seed}; n = {sum(rows)}, nnz = {sum(nnz)} in total), b ~ U[-1,1), "
                    f"exact dots, tol {tol}",
        "tuning": {k: v for k, v in tuning.items()},
        "create_ms": round(create_ms, 2),
        "solve_ms": round(batch_ms, 2),
        "loop_ms": round(st["loop_ms"], 2),
        "graph_launches": st["graph_launches"],
        "iterations_total": st["total_iterations"],
        "iterations_max": st["max_iterations"],
        "solo_solves_ms": round(solo_ms, 2),
        "speedup_vs_solo": round(solo_ms / batch_ms, 3),
        "row_iterations_per_s": round(row_it / (batch_ms * 1e-3), 1),
        "algorithmic_GB_s": round(it_bytes / (st["loop_ms"] * 1e-3) / 1e9, 1),
        "systems_bit_identical_to_solo": same,
    }
    log(f"[bench]   solo solves {solo_ms:.1f} ms; speedup {out['speedup_vs_solo']}; identical {same}/64")
    del mats, bs, xs
    torch.cuda.empty_cache()
    return out


def run_stress(n, w, n_ill, w_ill, rpcg, torch, dev):
    """The paper's stress workloads. Band transform (Section 5.1, bandL =
    bandU = w, b = A 1, x0 = 0, tol 1e-8): plain, exact-dot and FPE PCG, per
    iteration cost and overheads. Ill-conditioned band (Section 5.3: first
    row and column scaled by 2^16, condition number about 1e12, at the size
    of Table 3): tau history of the exact modes against plain's, as Table 3
    prints it."""
    import numpy as np
    from rpcg_workloads import band_csr, scale_first

    def band_system(nn, ww, sigma):
        A = band_csr(nn, ww)
        if sigma != 1.0:
            A = scale_first(A, sigma)
        Ad = rpcg.CSR.from_host(A, dev)
        nnz = int(A.row_ptr[-1])
        del A
        bd = rpcg.spmv(Ad, torch.ones(nn, dtype=torch.float64, device=dev))  # integers: exact in any order
        return Ad, bd, nnz

    def solve(Ad, bd, mode, p=0):
        rpcg.pcg_solve(Ad, bd, mode=mode, maxit=2, tol=1e-8, fpe_size=p, history=False, raise_on_error=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = rpcg.pcg_solve(Ad, bd, mode=mode, tol=1e-8, maxit=20000, fpe_size=p, history=True, timing=1)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) * 1e3
        it = max(1, info["iterations"])
        return x, info, {"iterations": info["iterations"], "solve_ms": round(wall, 2),
                         "setup_ms": round(info["setup_ms"], 2),
                         "ms_per_iteration": round(info["loop_ms"] / it, 5),
                         "k_spmv_dot_ms": round(info["k_spmv_dot_ms"] / max(1, info["k_launches"]), 5),
                         "fpe_escapes": info["fpe_escapes"], "fallbacks": info["fallbacks"]}

    out = {}
    log(f"[bench] stress: band n={n} w={w}")
    t = time.time()
    Ad, bd, nnz = band_system(n, w, 1.0)
    log(f"[bench]   nnz={nnz} ({time.time() - t:.1f}s)")
    p_auto, rng = rpcg.fpe_size_auto(Ad, bd)
    runs, xs, hs = {}, {}, {}
    for mode, p in (("plain", 0), ("exblas", 0), ("fpe", p_auto)):
        xs[mode], info, runs[mode] = solve(Ad, bd, mode, p)
        hs[mode] = info["hist"]
        log(f"[bench]   {mode}: {runs[mode]['iterations']} it, {runs[mode]['ms_per_iteration']} ms/it")
    k1_bytes_band = 10 * nnz + 4 * (n + 1) + 16 * n  # 16-bit codes + values, row pointers, d, w (SELL-64)
    spmv_band = time_spmv(rpcg, torch, Ad, n, nnz)
    log(f"[bench]   rpcg_spmv on the band: {spmv_band['ms']} ms, {spmv_band['GB_s']} GB/s")
    smat_band = time_spmv(rpcg, torch, Ad, n, nnz, prepared=True)
    log(f"[bench]   rpcg_smat_spmv on the band: {smat_band['ms']} ms, {smat_band['GB_s']} GB/s")
    out["band"] = {
        "workload": f"band matrix n={n}, bandL = bandU = {w} (nnz={nnz}), 2w+1 on the diagonal, -1 in the band, "
                    f"b = A 1, x0 = 0, tol 1e-8",
        "rpcg_spmv": spmv_band,
        "rpcg_smat_spmv": smat_band,
        "fpe_size_auto": p_auto, "exponent_range": rng,
        "runs": runs,
        "exblas_over_plain": round(runs["exblas"]["ms_per_iteration"] / runs["plain"]["ms_per_iteration"], 4),
        "fpe_over_plain": round(runs["fpe"]["ms_per_iteration"] / runs["plain"]["ms_per_iteration"], 4),
        "k_spmv_dot_GB_s_exblas": round(k1_bytes_band / (runs["exblas"]["k_spmv_dot_ms"] * 1e-3) / 1e9, 1),
        "exblas_fpe_identical": bool(torch.equal(xs["exblas"], xs["fpe"]) and torch.equal(hs["exblas"], hs["fpe"])),
    }
    del Ad, bd, xs
    torch.cuda.empty_cache()
    if n_ill > 0:
        sigma = 2.0 ** 16
        log(f"[bench] stress: ill-conditioned band n={n_ill} w={w_ill} sigma=2^16")
        t = time.time()
        Ad, bd, nnz = band_system(n_ill, w_ill, sigma)
        log(f"[bench]   nnz={nnz} ({time.time() - t:.1f}s)")
        p_auto, rng = rpcg.fpe_size_auto(Ad, bd)
        runs, xs, hs = {}, {}, {}
        for mode, p in (("plain", 0), ("exblas", 0), ("fpe", p_auto)):
            xs[mode], info, runs[mode] = solve(Ad, bd, mode, p)
            hs[mode] = info["hist"].numpy()
            log(f"[bench]   {mode}: {runs[mode]['iterations']} it")
        escapes = {}
        for p in range(1, 9):
            xp, info = rpcg.pcg_solve(Ad, bd, mode="fpe", tol=1e-8, maxit=20000, fpe_size=p, history=False)
            escapes[str(p)] = {"escapes": info["fpe_escapes"], "fallbacks": info["fallbacks"],
                               "identical_to_exblas": bool(torch.equal(xp, xs["exblas"]))}
        he, hp = hs["exblas"], hs["plain"]
        k = min(len(he), len(hp))
        show = sorted({0, 2, 9, 10, k // 2, len(he) - 1} & set(range(len(he))))
        out["ill_conditioned"] = {
            "workload": f"band matrix n={n_ill}, bandL = bandU = {w_ill} (nnz={nnz}), first row and column "
                        f"scaled by 2^16 (condition number about {sigma ** 2 * (2 * w_ill + 1):.1e}), "
                        f"b = A 1, x0 = 0, tol 1e-8",
            "fpe_size_auto": p_auto, "exponent_range": rng,
            "runs": runs,
            "exblas_fpe_identical": bool(torch.equal(xs["exblas"], xs["fpe"]) and np.array_equal(he, hs["fpe"])),
            "fpe_escapes_by_p": escapes,
            "plain_tau_entries_differing": int(np.sum(he[:k].view(np.uint64) != hp[:k].view(np.uint64))),
            "plain_tau_max_rel_diff": float(np.max(np.abs(hp[:k] - he[:k]) / he[:k])),
            "tau_hex": {str(j): {"exact": float(he[j]).hex(),
                                 "plain": float(hp[j]).hex() if j < len(hp) else None} for j in show},
        }
        del Ad, bd, xs
        torch.cuda.empty_cache()
    return out


EXDOT_KINDS = ("narrow", "wide", "cond:1e0", "cond:1e8", "cond:1e16", "cond:1e24", "cond:1e32")
EXDOT_CHUNK_LOG2 = 20


def exdot_chunk(kind, seed, n):
    """One chunk of an exdot input distribution (host, rpcg_workloads)."""
    from rpcg_workloads import exdot_conditioned, exdot_narrow, exdot_wide
    if kind == "narrow":
        return exdot_narrow(seed, n)
    if kind == "wide":
        return exdot_wide(seed, n)
    x, y, _ = exdot_conditioned(seed, n, float(kind.split(":")[1]))
    return x, y


def fill_exdot(kind, ne, torch, dev, seed=1000):
    """x, y of ne elements on the device: tile k is one 2^20-element chunk of
    the distribution (one host draw per kind), its pairs reordered by a
    seeded permutation of its own and x scaled by 2^s_k, s_k cycling through
    -3..3 (-1..1 for the narrow kind). The exponent range and the condition
    number Sum|x_i y_i| / |Sum x_i y_i| of any whole number of tiles stay
    those of the chunk (a permutation changes neither sum, the scale
    multiplies both alike), while no two tiles hold the same values at the
    same positions, so a lane's grid-stride walk meets no repeated pairs."""
    c = 1 << EXDOT_CHUNK_LOG2
    xs, ys = exdot_chunk(kind, seed, c)
    xc = torch.from_numpy(xs).to(dev)
    yc = torch.from_numpy(ys).to(dev)
    X = torch.empty(ne, dtype=torch.float64, device=dev)
    Y = torch.empty(ne, dtype=torch.float64, device=dev)
    span = 3 if kind == "narrow" else 7
    gen = torch.Generator(device=dev)
    for k in range(ne // c):
        gen.manual_seed(seed * 100003 + k)
        perm = torch.randperm(c, generator=gen, device=dev)
        X[k * c:(k + 1) * c].copy_(xc[perm] * 2.0 ** ((k % span) - span // 2))
        Y[k * c:(k + 1) * c].copy_(yc[perm])
    return X, Y


def time_exdot(rpcg, torch, X, Y, mode, reps, warm=10):
    """Median, min and max of reps event-timed calls (after warm calls) and the
    counters of one synchronous call."""
    import numpy as np
    out = torch.empty(1, dtype=torch.float64, device=X.device)
    stream = torch.cuda.current_stream()
    for _ in range(warm):
        rpcg.exdot(X, Y, mode=mode, out=out, sync=False)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rpcg.exdot(X, Y, mode=mode, out=out, sync=False)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    _, info = rpcg.exdot(X, Y, mode=mode, out=out)
    return float(np.median(times)), float(min(times)), float(max(times)), info


def run_exdot_grid(log2_max, reps, rpcg, torch, dev, kinds=EXDOT_KINDS):
    """Standalone exact dot over lengths 2^20..2^log2_max (every second power)
    and the seven input distributions, in the three modes: GB/s of the 16 n
    algorithmic bytes and the fraction of the 8 TB/s HBM peak."""
    ne = 1 << log2_max
    sizes = [1 << k for k in range(EXDOT_CHUNK_LOG2, log2_max + 1, 2)]
    if sizes[-1] != ne:
        sizes.append(ne)
    grid = {}
    for kind in kinds:
        log(f"[bench] exdot grid {kind}: filling 2^{log2_max}")
        X, Y = fill_exdot(kind, ne, torch, dev)
        grid[kind] = {}
        for n in sizes:
            row = {}
            for mode in ("exblas", "fpe", "plain"):
                tm, tmin, tmax, info = time_exdot(rpcg, torch, X[:n], Y[:n], mode, reps)
                gbs = 16 * n / (tm * 1e-3) / 1e9
                row[mode] = {"ms": round(tm, 5), "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                             "GB_s_best": round(16 * n / (tmin * 1e-3) / 1e9, 1),
                             "GB_s_worst": round(16 * n / (tmax * 1e-3) / 1e9, 1),
                             "escapes": info["fpe_escapes"], "status": info["status"]}
            grid[kind][f"2^{n.bit_length() - 1}"] = row
            log(f"[bench]   n=2^{n.bit_length() - 1}: " +
                ", ".join(f"{m} {row[m]['GB_s']:.0f}" for m in row) + " GB/s")
        del X, Y
        torch.cuda.empty_cache()
    return {"workload": "two binary64 vectors of n elements, tiles of one 2^20-element chunk, each tile permuted "
                        "(seeded) and scaled by a power of two "
                        "(narrow: U[-1,1); wide: exponents uniform in [-200, 200], random signs; cond:c: wide "
                        "pairs with cancelling mirrored pairs and a signal giving condition number about c)",
            "reps": reps, "grid": grid}


def cpu_model():
    try:
        import subprocess
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(A, b, N, iters, reps):
    """The oracle (exact dots) on this machine's host cores on a bounded sample
    of the same solve: at one thread, and at all threads (median of reps);
    and the host plain loop (ordinary dots) at all threads beside it."""
    import numpy as np
    import oracle
    if not os.path.exists(oracle._LIB):
        oracle.build()
    all_threads = oracle.set_threads(0)

    def rate(fn, k):
        t0 = time.perf_counter()
        fn(0)
        t1 = time.perf_counter()
        r = fn(k)
        t2 = time.perf_counter()
        return r, r["iters"] / ((t2 - t1) - (t1 - t0))

    exact = lambda k: oracle.pcg(A, b, tol=1e-8, maxit=k)
    plain = lambda k: oracle.cpu_plain_pcg(A, b, tol=1e-8, maxit=k)
    oracle.set_threads(1)
    log(f"[bench] oracle on the host: {iters} iterations at 1 thread")
    r1, one = rate(exact, iters)
    oracle.set_threads(all_threads)
    rN = exact(iters)
    same = bool(np.array_equal(r1["x"].view(np.uint64), rN["x"].view(np.uint64))
                and np.array_equal(r1["hist"].view(np.uint64), rN["hist"].view(np.uint64)))
    log(f"[bench] oracle on the host: {reps} x {4 * iters} iterations at {all_threads} threads")
    rates = sorted(rate(exact, 4 * iters)[1] for _ in range(reps))
    log(f"[bench] host plain loop: {reps} x {8 * iters} iterations at {all_threads} threads")
    prates = sorted(rate(plain, 8 * iters)[1] for _ in range(reps))
    med, pmed = float(np.median(rates)), float(np.median(prates))
    log(f"[bench]   oracle {one:.2f} it/s (1 thread), {med:.2f} it/s ({all_threads} threads); plain {pmed:.2f} it/s")
    return {"value": round(med, 4), "unit": "iterations/s", "cores": all_threads, "kind": "oracle",
            "sample": f"first {4 * iters} PCG iterations of the {N}^3 exact-dot solve (setup timed separately "
                      f"and subtracted), C oracle with OpenMP, median of {reps} runs; at 1 thread the first "
                      f"{iters}",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "oracle_1_thread": round(one, 4), "oracle_all_threads_min_max": [round(rates[0], 4), round(rates[-1], 4)],
            "identical_bits_1_vs_all_threads": same,
            "cpu_plain": {"value": round(pmed, 4), "unit": "iterations/s", "cores": all_threads,
                          "sample": f"first {8 * iters} iterations, same loop with ordinary OpenMP dot sums, "
                                    f"median of {reps} runs"},
            "exact_over_plain": round(pmed / med, 3)}


LP_FWD_FLOP_PER_CELL = 2 * 27 * (4 * 16 + 16 * 16 + 16 * 4)  # three convolutions, algorithmic


def run_learned(n_eval, rpcg, torch, dev):
    """Learned preconditioner (committed trained parameters) against Jacobi:
    exact-dot PCG to 1e-10 on held-out 64^3 log-normal diffusion instances;
    throughput of the bfloat16 MFMA network (forward, training step)."""
    from paper_2005_07282_amd import learned
    if not os.path.exists(learned.PARAMS_FILE):
        log("[bench] learned preconditioner: no trained parameters, skipped")
        return None
    N = 64
    params = learned.load_params()
    log(f"[bench] learned preconditioner: {n_eval} held-out instances of {N}^3")
    ev = learned.Dataset(rpcg, torch, N, [learned.EVAL_SEED0 + k for k in range(n_eval)], dev)
    net = rpcg.LearnedPreconditioner(N, max_batch=8, params=params)
    learned.evaluate(rpcg, torch, net, ev, limit=1)  # warm-up
    rows = learned.evaluate(rpcg, torch, net, ev)
    out = learned.summarize(rows)
    # network throughput: forward of 8 systems; one training step on 8 systems (separate copy)
    nb = min(8, n_eval)
    mats = ev.mats[:nb]
    net.forward(mats)
    reps = 9

    def median_ms(fn):
        # each call is timed on its own (the forward waits for its result);
        # the median keeps an occasional host-side stall out of the figure
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return sorted(ts)[reps // 2]

    fwd_ms = median_ms(lambda: net.forward(mats))
    from rpcg_workloads import uniform_pm1
    us = [[torch.from_numpy(uniform_pm1(900 + 7 * k + j, ev.n)).to(dev) for j in range(4)] for k in range(nb)]
    tnet = rpcg.LearnedPreconditioner(N, max_batch=nb, params=params)
    tnet.train_step(mats, us, lr=0.0)
    step_ms = median_ms(lambda: tnet.train_step(mats, us, lr=0.0))
    tnet.close()
    net.close()
    flop = LP_FWD_FLOP_PER_CELL * ev.n * nb
    out.update({
        "workload": f"7-point diffusion, exp(1.5 GRF) coefficients (correlation 8 cells), {N}^3, held-out grid seeds "
                    f"{learned.EVAL_SEED0}..{learned.EVAL_SEED0 + n_eval - 1}, b ~ U[-1,1), exact dots, tol 1e-10, "
                    f"M^-1 = G G^T + 1e-6 I",
        "forward_ms_8_systems": round(fwd_ms, 3),
        "forward_TFLOP_s_bf16": round(flop / (fwd_ms * 1e-3) / 1e12, 2),
        "forward_frac_of_bf16_peak": round(flop / (fwd_ms * 1e-3) / 2.5e15, 4),
        "train_step_ms_8_systems_4_vectors": round(step_ms, 3),
        "throughput_timing": f"median of {reps} single calls",
    })
    log(f"[bench]   iterations Jacobi {out['jacobi_iterations_mean']:.1f}, learned {out['learned_iterations_mean']:.1f}; "
        f"time ratio {out['time_ratio_incl_factor']:.3f}")
    del ev
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=160, help="N of the N^3 grid")
    ap.add_argument("--reps", type=int, default=5, help="timed loops per mode (the median is reported)")
    ap.add_argument("--exdot-log2", type=int, default=28)
    ap.add_argument("--exdot-reps", type=int, default=20)
    ap.add_argument("--exdot-only", action="store_true", help="only the exdot grid; prints its JSON")
    ap.add_argument("--exdot-kinds", default=",".join(EXDOT_KINDS),
                    help="comma-separated input distributions of the exdot grid")
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ir-grid", type=int, default=256,
                    help="N of the N^3 grid of the mixed-precision refinement section (0 = skip)")
    ap.add_argument("--batch-seed", type=int, default=7,
                    help="seed of the batched workload (64 systems, 16^3..96^3); -1 = skip")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched section and print its JSON (for a separate kernel trace)")
    ap.add_argument("--lp-eval", type=int, default=20,
                    help="held-out 64^3 instances for the learned-preconditioner section (0 = skip)")
    ap.add_argument("--lp-only", action="store_true",
                    help="run only the learned-preconditioner section and print its JSON")
    ap.add_argument("--stress-n", type=int, default=4_000_000,
                    help="rows of the band stress matrix (bandL = bandU = 100); 0 skips the stress section")
    ap.add_argument("--stress-ill-n", type=int, default=159 ** 3,
                    help="rows of the ill-conditioned band matrix (bandL = bandU = 200); 0 skips it")
    ap.add_argument("--stress-only", action="store_true", help="only the stress section; prints its JSON")
    ap.add_argument("--mixed-only", action="store_true",
                    help="run only the mixed-precision section and print its JSON (for a separate kernel trace)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for hardware counters: a few exblas iterations on the N^3 operator "
                         "and a 1 GiB device-to-device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU decomposition is a design, see the documentation", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2005_07282_amd import rpcg
    from rpcg_workloads import (stencil27_csr, stencil27_rhs_from_int52,
                                uniform_pm1_int52)

    if not os.path.exists(rpcg.LIB_PATH):
        raise SystemExit("librpcg.so is not built (run __graft_entry__.build())")
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rpcg.context(0)
    if args.mixed_only:
        print(json.dumps(run_mixed_precision(args.ir_grid, rpcg, torch, dev)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(run_batched(args.batch_seed, rpcg, torch, dev)), flush=True)
        return
    if args.lp_only:
        print(json.dumps(run_learned(args.lp_eval, rpcg, torch, dev)), flush=True)
        return
    if args.exdot_only:
        print(json.dumps(run_exdot_grid(args.exdot_log2, args.exdot_reps, rpcg, torch, dev,
                                        args.exdot_kinds.split(","))), flush=True)
        return
    if args.stress_only:
        print(json.dumps(run_stress(args.stress_n, 100, args.stress_ill_n, 200, rpcg, torch, dev)), flush=True)
        return

    N = args.grid
    log(f"[bench] generating 27-point operator on {N}^3")
    t = time.time()
    A = stencil27_csr(N)
    K = uniform_pm1_int52(2, A.n)
    b = stencil27_rhs_from_int52(N, K)
    del K
    n, nnz = A.n, A.nnz
    Ad = rpcg.CSR.from_host(A, dev)
    bd = torch.from_numpy(b).to(dev)
    log(f"[bench] n={n} nnz={nnz} ({time.time() - t:.1f}s)")

    if args.profile_pass:
        src = torch.zeros(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        x, info = rpcg.pcg_solve(Ad, bd, mode="exblas", maxit=5, tol=1e-8, history=False)
        torch.cuda.synchronize()
        log(f"[bench] profile pass: copy of {src.numel() * 8} bytes, {info['iterations']} exblas iterations")
        return

    def solve(mode, maxit, timing=0):
        torch.cuda.synchronize()
        x, info = rpcg.pcg_solve(Ad, bd, mode=mode, maxit=maxit, tol=1e-8, timing=timing, history=False)
        torch.cuda.synchronize()
        return x, info

    def median_run(runs):
        """The run whose loop time is the median of the repetitions."""
        order = sorted(runs, key=lambda r: r["loop_ms"])
        return order[len(order) // 2]

    res, spread = {}, {}
    reps = max(1, args.reps)
    for mode in ("exblas", "fpe", "plain"):
        log(f"[bench] PCG {mode}: warmup {args.warmup} iterations")
        solve(mode, max(1, args.warmup))
        log(f"[bench] PCG {mode}: timing {reps} x {args.steps} iterations")
        # every mode is timed alike: HIP events around the SpMV+dot launch of
        # every K1_TIMING_STRIDE-th iteration only
        runs = [solve(mode, args.steps, timing=K1_TIMING_STRIDE + 1)[1] for _ in range(reps)]
        for info in runs:
            if info["iterations"] != args.steps:
                log(f"[bench] note: {mode} stopped after {info['iterations']} iterations")
        res[mode] = median_run(runs)
        its = sorted(r["iterations"] / r["loop_ms"] * 1e3 for r in runs)
        spread[mode] = {"median": round(float(np.median(its)), 2), "min": round(its[0], 2), "max": round(its[-1], 2)}
        log(f"[bench]   {res[mode]['iterations']} it; it/s median {spread[mode]['median']} "
            f"(min {spread[mode]['min']}, max {spread[mode]['max']})")
    # the same iterations with no events at all (what the events cost), and
    # with every kernel bracketed (durations of the update and direction kernels)
    bare_runs = [solve("exblas", args.steps, timing=0)[1] for _ in range(reps)]
    bare = median_run(bare_runs)
    its = sorted(r["iterations"] / r["loop_ms"] * 1e3 for r in bare_runs)
    spread["exblas_no_events"] = {"median": round(float(np.median(its)), 2), "min": round(its[0], 2),
                                  "max": round(its[-1], 2)}
    inst = median_run([solve("exblas", args.steps, timing=1)[1] for _ in range(reps)])
    # the headline: the loop with no events in it (the median of the bare
    # repetitions); the kernel durations come from the bracketed loops
    ex = res["exblas"]
    L = bare["iterations"]
    ms_per_step = bare["loop_ms"] / L
    value = L / (bare["loop_ms"] / 1e3)
    k1_ms = ex["k_spmv_dot_ms"] / max(1, ex["k_launches"])
    k2_ms = inst["k_update_ms"] / max(1, inst["k_launches"])
    k3_ms = inst["k_direction_ms"] / max(1, inst["k_launches"])
    k1_gbs = k1_bytes(n, nnz) / (k1_ms * 1e-3) / 1e9
    it_gbs = iteration_bytes(n, nnz) / (ms_per_step * 1e-3) / 1e9
    per_it = {m: res[m]["loop_ms"] / res[m]["iterations"] for m in res}

    # full solve to 1e-8 (the paper's stopping rule) for the iteration count
    log("[bench] exblas full solve to tol 1e-8")
    _, full = solve("exblas", 2000)
    spmv160 = time_spmv(rpcg, torch, Ad, n, nnz)
    log(f"[bench] rpcg_spmv {N}^3: {spmv160['ms']} ms, {spmv160['GB_s']} GB/s")
    smat160 = time_spmv(rpcg, torch, Ad, n, nnz, prepared=True)
    log(f"[bench] rpcg_smat_spmv {N}^3: {smat160['ms']} ms, {smat160['GB_s']} GB/s")
    del Ad, bd
    torch.cuda.empty_cache()

    # standalone exact dot over the length x distribution grid
    ne = 1 << args.exdot_log2
    exgrid = run_exdot_grid(args.exdot_log2, args.exdot_reps, rpcg, torch, dev, args.exdot_kinds.split(","))
    top = f"2^{args.exdot_log2}"
    exd = {f"{kind}_{mode}": exgrid["grid"][kind][top][mode] for kind in ("wide", "narrow")
           if kind in exgrid["grid"] for mode in ("exblas", "fpe", "plain")}

    cpu = None if args.no_cpu else run_cpu_baseline(A, b, N, args.cpu_iters, args.cpu_reps)

    mixed = run_mixed_precision(args.ir_grid, rpcg, torch, dev) if args.ir_grid > 0 else None
    batched = run_batched(args.batch_seed, rpcg, torch, dev) if args.batch_seed >= 0 else None
    learned_pc = run_learned(args.lp_eval, rpcg, torch, dev) if args.lp_eval > 0 else None
    stress = run_stress(args.stress_n, 100, args.stress_ill_n, 200, rpcg, torch, dev) if args.stress_n > 0 else None

    traffic = k1_traffic() if N == 160 else None
    stream_gbs = measure_stream_read(torch, dev)
    log(f"[bench] stream read (torch.sum, 2 GiB binary64) {stream_gbs:.1f} GB/s")
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": L,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"27-point Poisson {N}^3 (n={n}, nnz={nnz}), fp64 CSR, Jacobi PCG, exact dots "
                        f"(exblas mode), b = A x*, x* ~ U[-1,1) seed 2, x0 = 0",
            "mode": "exblas",
            "iterations_to_1e-8": full["iterations"],
            "timed_loops": reps,
            "it_s_spread": spread,
            "exblas_it_s_with_k1_events": round(ex["iterations"] / ex["loop_ms"] * 1e3, 2),
            "plain_it_s": round(1e3 / per_it["plain"], 2),
            "fpe_it_s": round(1e3 / per_it["fpe"], 2),
            "exblas_over_plain": round(per_it["exblas"] / per_it["plain"], 4),
            "fpe_over_plain": round(per_it["fpe"] / per_it["plain"], 4),
            "iteration_GB_s": round(it_gbs, 1),
            "kernel_ms": {"spmv_dot": round(k1_ms, 5), "update_dots": round(k2_ms, 5),
                          "direction": round(k3_ms, 5)},
            "rpcg_spmv": spmv160,
            "rpcg_smat_spmv": smat160,
            "exdot_n": ne,
            "exdot": exd,
            "exdot_grid": exgrid,
            "mixed_precision": mixed,
            "batched": batched,
            "learned_preconditioner": learned_pc,
            "stress": stress,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(k1_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(k1_gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_pcg_spmv_dot<exblas, 4, 16-bit column codes, binary64>",
            "bytes_per_launch": k1_bytes(n, nnz),
            "stream_read": {"GB_s": round(stream_gbs, 1), "frac": round(k1_gbs / stream_gbs, 4),
                            "kernel": "torch.sum over a 2 GiB binary64 vector (fastest of 10)"},
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

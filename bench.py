#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config m60_n20000] [--solve-config m21_n2000]

Headline (`value`): the kernel matrix-vector product of the largest
single-GPU workload, M = 60 atoms, N = 20000 geometries (n = 3.6M unknowns,
D = 1770 inverse distances), Matern-5/2 sigma = 10, in the precision the
solve's reduced phase uses: split BF16 (hi*hi + hi*lo + lo*hi on BF16 MFMA
with FP32 accumulation; the constant and row-sum terms in FP64).  A step is
one product y = K v on inputs already in HBM; `value` is its algorithmic
rate F / t with F = 6 N^2 D + 24 N D, timed with HIP events over K steps
after W untimed ones.  The roofline entry is the product's dominant kernel
(GEMM 2, [dA | -W][U; X_c]) from per-launch HIP-event clocks of a second
pass over the same steps, against the split-BF16 peak (the BF16 peak / 3:
three BF16 products per split product).

Beside it the run reports:
  * the product's rate in every precision at this and the other workloads;
  * the time-to-solution comparison on the M = 21, N = 2000 workload
    (n = 126000, k = 2000, lambda = 1e-9): descriptor, column selection,
    preconditioner build (L stored FP32 for the mixed arms, FP64 for the FP64
    arms) and PCG to a true FP64 relative residual of 1e-6.  The mixed
    schedule runs FP32 products until the residual is below 0.7 |F|, then
    split BF16 with an FP64 true-residual refresh every 10 iterations.  Arms:
    mixed and FP64 with the learned selection (the same columns, so their
    ratio is the precision's gain), mixed with uniform columns (what the
    network gains over the method without it), and mixed and FP64 with the
    workload's own pivoted-Cholesky columns.  The score network is trained
    before the timed region on exact ridge-leverage labels of small systems of
    the same molecule; its cost, label spread and final loss are reported as
    `learned_setup`;
  * the FP64 CPU oracle on the host's cores (`cpu_baseline`): its product at
    the headline workload on a sample of target geometries, the small
    workload's dense Cholesky solve and its textbook PCG.
The largest workload's full solve is not run: its estimated time is longer
than one benchmark job.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X dense peaks.  Split BF16 executes three BF16 products per product,
# so its peak in algorithmic flops is the BF16 peak / 3.
PEAK_TFLOPS = {"bf16": 2500.0, "bf16x3": 2500.0 / 3.0, "fp32": 157.3, "fp64": 78.6}
EXEC_FACTOR = {"bf16": 1, "bf16x3": 3, "fp32": 1, "fp64": 1}
PEAK_HBM_GBS = 8000.0
TOL = 1e-6
CLOCK_STRIDE = 16       # solves: event pairs around every 16th launch of each clocked kernel


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mvm_flops(N: int, D: int) -> float:
    """Algorithmic flops of one kernel product: 2N^2D (GEMM 1) + 4N^2D (GEMM 2) + 24ND (J v, J^T G)."""
    return 6.0 * N * N * D + 24.0 * N * D


def kernel_model(name: str, N: int, D: int, n: int, k: int, L_bytes: int):
    """(bound, algorithmic amount per launch, unit) of each clocked kernel.

    GEMMs count their algorithmic flops once, whatever the operand split;
    the GEMVs count one pass over the stored L plus their input vector."""
    return {
        "gemm1": ("mfma", 2.0 * N * N * D, "flop"),
        "gemm2": ("mfma", 4.0 * N * N * D, "flop"),
        "gemv_t": ("hbm", float(L_bytes) * n * k + 8.0 * n, "B"),
        "gemv_n": ("hbm", float(L_bytes) * n * k + 8.0 * k, "B"),
        "jv": ("hbm", 8.0 * (2 * n + N * D), "B"),
        "jtg": ("hbm", 8.0 * (N * D + 2 * n), "B"),
    }.get(name)


def iteration_roofline(cfg, n: int, k: int, rec: dict, L_bytes: int = 4) -> dict:
    """The timed mixed solve's PCG phase against a lower bound made from the peaks.

    Every iteration: two passes over the stored L and about 13 passes over
    FP64 n-vectors at the HBM peak.  Every product: the larger of its MFMA
    time (F at the peak of its precision; split BF16: its three products at
    the BF16 peak) and its HBM time (four N x N passes: dA, B, W written, W
    read; 32 B per entry in FP64, 16 B in FP32 and split BF16).  Products
    before the switch run in the first-phase precision, refreshes in FP64,
    the rest in split BF16."""
    N, D = cfg.N, cfg.D
    F = mvm_flops(N, D)
    hbm = PEAK_HBM_GBS * 1e9
    t_apply = (2.0 * L_bytes * n * k + 13 * 8.0 * n) / hbm
    t64 = max(F / (PEAK_TFLOPS["fp64"] * 1e12), 32.0 * N * N / hbm)
    t32 = max(F / (PEAK_TFLOPS["fp32"] * 1e12), 16.0 * N * N / hbm)
    tx3 = max(F / (PEAK_TFLOPS["bf16x3"] * 1e12), 16.0 * N * N / hbm)
    it, sw, nr = rec["iters"], rec["switch_iter"], rec["n_refresh"]
    t_first = t32 if rec["switch_from"] == "fp32" else t64
    ideal = it * t_apply + sw * t_first + nr * t64 + (it - sw) * tx3
    return {"ideal_pcg_s": ideal, "measured_pcg_s": rec["t_pcg_s"], "frac": ideal / rec["t_pcg_s"],
            "ideal_us_per_iteration": 1e6 * ideal / it, "measured_us_per_iteration": 1e6 * rec["t_pcg_s"] / it,
            "ideal_apply_us": 1e6 * t_apply, "ideal_product_us": {"fp64": 1e6 * t64, "fp32": 1e6 * t32,
                                                                  "bf16x3": 1e6 * tx3},
            "products": {"first_phase_" + rec["switch_from"]: sw, "fp64_refresh": nr, "bf16x3": it - sw}}


def time_mvm(ffk, ctx, S, v, prec, steps, warmup):
    """Mean ms of one product over `steps` back-to-back products (HIP events on the launch stream)."""
    import torch
    y = torch.empty_like(v)
    for _ in range(warmup):
        ffk.kernel_mvm(ctx, S, v, y, prec=prec)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(steps):
        ffk.kernel_mvm(ctx, S, v, y, prec=prec)
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def mvm_rates(ffk, ctx, cfg, S, v, steps, warmup, precs=("bf16", "bf16x3", "fp32", "fp64")):
    fl = mvm_flops(cfg.N, cfg.D)
    out = {}
    for prec in precs:
        ms = time_mvm(ffk, ctx, S, v, ffk.PRECISIONS[prec], steps, warmup)
        tf = fl / ms / 1e9
        out[prec] = {"ms": ms, "tflops": tf, "frac_peak": tf / PEAK_TFLOPS[prec],
                     "executed_tflops": tf * EXEC_FACTOR[prec]}
        log("mvm %s %-6s %9.4f ms %8.2f TFLOP/s algorithmic (%.1f%% of the %s peak of %.1f)"
            % (cfg.name, prec, ms, tf, 100 * tf / PEAK_TFLOPS[prec], prec, PEAK_TFLOPS[prec]))
    return out


def solve(ffk, ctx, R, F, cfg, arm: str, net=None):
    """One pass of the hot path from R and F in HBM; returns (alpha, record).

    arm: "<precision>_<selection>" with precision "mixed" (split BF16 after an
    FP32 first phase, L stored FP32) or "fp64" (FP64 products and L), and
    selection "learned" (the score network, pivoted-Cholesky fallback),
    "uniform" or "pivchol"."""
    import torch
    from paper_2212_12737_amd import learned
    prec_arm, sel = arm.split("_", 1)
    mixed = prec_arm == "mixed"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = ffk.descriptor_build(ctx, R, cfg.sigma)
    t_desc = time.perf_counter() - t0
    store = ffk.FP32 if mixed else ffk.FP64
    if sel == "learned":
        P, how = learned.build_with_fallback(ctx, net, S, cfg.k, cfg.lam, cfg.sel_seed, store=store)
        torch.cuda.synchronize()
        t1 = t2 = time.perf_counter()   # selection and build are one call here
    else:
        how = sel
        idx = ffk.nystrom_select(ctx, S, sel, cfg.k, lam=cfg.lam, seed=cfg.sel_seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P = ffk.precond_build(ctx, S, idx, cfg.lam, store=store)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    SWITCH_BELOW, REFRESH, FROM = ffk.MIXED_SWITCH_BELOW, ffk.MIXED_REFRESH, ffk.MIXED_SWITCH_FROM
    alpha, rep = ffk.pcg_solve(ctx, S, P, F, cfg.lam, tol=TOL, max_iter=50000,
                               prec=ffk.BF16X3 if mixed else ffk.FP64, refresh_every=REFRESH, escalate=True,
                               switch_below=SWITCH_BELOW if mixed else 0.0, switch_from=FROM)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    first = "fp64" if FROM == ffk.FP64 else "fp32"
    rec = {
        "arm": arm, "selection": how, "switch_from": first if mixed else None,
        "products": ("%s until |r| < %g |F|, then bf16x3; fp64 refresh every %d" % (first, SWITCH_BELOW, REFRESH))
        if mixed else "fp64",
        "L_storage": "fp32" if mixed else "fp64",
        "k_eff": int(P.k_eff), "iters": int(rep.iters), "switch_iter": int(rep.switch_iter),
        "status": int(rep.status), "rel_res_true": rep.rel_res_true, "n_refresh": int(rep.n_refresh),
        "n_escalations": int(rep.n_escalations), "final_prec": int(rep.final_prec),
        "t_descriptor_s": t_desc, "t_select_s": (t1 - t0 - t_desc) if sel != "learned" else None,
        "t_build_s": (t2 - t1) if sel != "learned" else None,
        "t_select_build_s": t2 - t0 - t_desc, "t_pcg_s": t3 - t2, "t_total_s": t3 - t0,
    }
    return alpha, rec


def train_network(ffk, ctx, cfg, systems: int, N: int, steps: int):
    """Score network for this molecule from exact labels of small systems
    (same molecule, displacement seeds disjoint from the workload's)."""
    import torch
    import synth
    from paper_2212_12737_amd import learned
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S_tr, y_tr = [], []
    for t in range(systems):
        st = synth.config_system(cfg, N=N, disp_seed=cfg.disp_seed + 1000 + t)
        S = ffk.descriptor_build(ctx, torch.as_tensor(st.R, device="cuda"), cfg.sigma)
        S_tr.append(S)
        y_tr.append(learned.make_labels(ctx, S, cfg.lam))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net, tl = learned.train(ctx, S_tr, y_tr, H=256, steps=steps, batch=256, lr=1e-3, seed=7, log_every=steps // 4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    y = torch.cat(y_tr)
    # the labels are log block scores centred per system: their spread is
    # what the network can tell apart
    return net, {"systems": systems, "N_each": N, "steps": steps, "t_labels_s": t1 - t0, "t_train_s": t2 - t1,
                 "loss_first": tl.losses[0][1], "loss_last": tl.losses[-1][1],
                 "label_std": float(y.std().item()), "label_min": float(y.min().item()),
                 "label_max": float(y.max().item()),
                 "label": "log of the exact per-geometry ridge-leverage score, centred per system (dense FP64 "
                          "Cholesky on the GPU)"}


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# sources whose kernels the HBM traffic figures below were taken from
KERNEL_SOURCES = {
    "gemv_t": ["paper_2212_12737_amd/csrc/precond.hip"],
    "gemv_n": ["paper_2212_12737_amd/csrc/precond.hip"],
    "gemm1": ["paper_2212_12737_amd/csrc/mvm.hip", "paper_2212_12737_amd/csrc/gemm.hpp"],
    "gemm2": ["paper_2212_12737_amd/csrc/mvm.hip", "paper_2212_12737_amd/csrc/gemm.hpp"],
}


def measured_traffic(kernel: str, workload: str, prec: str = "bf16x3"):
    """HBM bytes per launch from the committed counter summary, if its source digest still matches."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as f:
        tab = json.load(f)
    e = tab.get(workload, {}).get(kernel)
    if e and "precision" in e and e["precision"] != prec:
        e = None
    if not e or e.get("source_digest") != source_digest(KERNEL_SOURCES[kernel]):
        return None
    return e["bytes_per_launch"]


def host_info() -> dict:
    """CPU model, logical CPUs usable by this process, and RAM of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = int(line.split()[1]) * 1024
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_usable": avail,
            "ram_gb": round(ram / 2 ** 30, 1) if ram else None}


def host_cores() -> int:
    """Cores the oracle may use: the CPUs this process may run on, capped by
    the thread budget the environment sets (OMP_NUM_THREADS) if any."""
    n = host_info()["cpus_usable"] or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


# (R, v, sigma) of the oracle's product sample, set before the worker processes are forked
_ORACLE_INPUT = None


def _oracle_product_worker(targets):
    """Time the oracle's product on a sample of target geometries (one process, one BLAS thread)."""
    from threadpoolctl import threadpool_limits
    from oracle import kernel as ok
    R, v, sigma = _ORACLE_INPUT
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ok.kernel_mvm(R, R, v, sigma, targets=targets[:1], chunk=1)
        t1 = time.perf_counter()
        ok.kernel_mvm(R, R, v, sigma, targets=targets, chunk=1)
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1, len(targets)


def cpu_baseline(cfg_h, budget_s: float = 20.0) -> dict:
    """The FP64 oracle, as it stands, on the host's cores.

    Headline figure (same unit as `value`): the oracle's matrix-free product
    at the headline workload.  Each of C worker processes runs the oracle's
    kernel_mvm on its share of a sample of target geometries (one BLAS thread
    each); a call on one target and a call on all of the worker's targets give
    the time of the source-side part (J v over all sources) and the time per
    target.  The whole product on C cores is then t_sources + N t_target / C,
    and its rate F / that time.  Also: the small workload's dense Cholesky
    solve (block assembly of K plus factorisation, median of 3) and its
    textbook PCG with the workload's uniform Nystroem preconditioner, with
    BLAS on all C cores."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits, threadpool_info
    import synth
    from oracle import kernel as ok
    from oracle import select as osel
    from oracle import solve as osv

    global _ORACLE_INPUT
    info = host_info()
    C = host_cores()
    s = synth.config_system(cfg_h)
    _ORACLE_INPUT = (s.R, synth.random_vectors(s.R.size, 11), cfg_h.sigma)
    # targets per worker for about budget_s / 2 of per-target work: one target
    # costs about 0.26 s at N = 20000, D = 1770 on one core of a 2.7 GHz
    # Xeon, and scales with N D
    per_target_guess = 0.26 * cfg_h.N * cfg_h.D / (20000 * 1770)
    Tw = int(max(3, min(64, budget_s * 0.5 / per_target_guess)))
    rng = np.random.default_rng(5)
    sample = rng.choice(cfg_h.N, size=min(cfg_h.N, C * Tw), replace=False)
    chunks = [sample[i::C] for i in range(C)]
    # forked before this process touches the GPU: the workers only run numpy
    t0 = time.perf_counter()
    pool = mp.get_context("fork").Pool(C)
    try:
        res = pool.map(_oracle_product_worker, chunks)
    finally:
        pool.close()
        pool.join()
    wall = time.perf_counter() - t0
    _ORACLE_INPUT = None
    Tw = len(chunks[0])
    per_target = float(np.median([(b - a) / max(n - 1, 1) for a, b, n in res]))
    t_sources = float(np.median([a for a, b, n in res])) - per_target
    t_full = max(t_sources, 0.0) + cfg_h.N * per_target / C
    F = mvm_flops(cfg_h.N, cfg_h.D)
    head = {"value": F / t_full / 1e12, "unit": "TFLOP/s", "cores": C, "kind": "oracle",
            "sample": ("FP64 oracle kernel_mvm (per-pair numpy einsum) at %s, %d worker processes x %d target "
                       "geometries of %d (%.1f s wall): %.3f s per target geometry, %.2f s of source-side work "
                       "(J v); the whole product extrapolated to %.1f s on %d cores"
                       % (cfg_h.name, C, Tw, cfg_h.N, wall, per_target, t_sources, t_full, C)),
            "seconds_per_product": t_full, "host": info}

    # the small workload: dense Cholesky (median of 3) and textbook PCG
    c1 = synth.CONFIGS["m9_n200"]
    s1 = synth.config_system(c1)
    F1 = s1.flat_forces()
    with threadpool_limits(C):
        blas = [(d.get("internal_api"), d.get("num_threads")) for d in threadpool_info()]
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            K = ok.dense_kernel(s1.R, c1.sigma)
            a = osv.cholesky_solve(K, c1.lam, F1)
            times.append(time.perf_counter() - t0)
        idx = osel.select_uniform(K.shape[0], c1.k, c1.sel_seed)
        t0 = time.perf_counter()
        L, _, _, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), c1.k, order=idx)
        x, it, _ = osv.pcg(lambda v: K @ v + c1.lam * v, F1, osv.woodbury(L, c1.lam), tol=TOL)
        t_pcg = time.perf_counter() - t0
        res = np.linalg.norm(K @ x + c1.lam * x - F1) / np.linalg.norm(F1)
    head["small_workload"] = {
        "workload": "m9_n200: M=9, N=200, n=5400, lambda=1e-8",
        "dense_cholesky_s_median_of_3": float(np.median(times)), "dense_cholesky_s_runs": times,
        "oracle_pcg_s": t_pcg, "oracle_pcg_iterations": int(it), "oracle_pcg_true_residual": float(res),
        "oracle_pcg_note": "uniform k=100 Nystroem (incomplete Cholesky in the sampled order) + Woodbury, "
                           "dense K products, stop at recursive residual 1e-6; time includes the factor",
        "blas": blas}
    return head


def small_gpu_solve(ffk, ctx):
    """FP64 PCG of the small workload on the GPU (uniform k = 100), for the CPU baseline's context."""
    import torch
    import synth
    c1 = synth.CONFIGS["m9_n200"]
    s1 = synth.config_system(c1)
    R = torch.as_tensor(s1.R, device="cuda")
    F = torch.as_tensor(s1.flat_forces(), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = ffk.descriptor_build(ctx, R, c1.sigma)
    idx = ffk.nystrom_select(ctx, S, "uniform", c1.k, seed=c1.sel_seed)
    P = ffk.precond_build(ctx, S, idx, c1.lam)
    _, rep = ffk.pcg_solve(ctx, S, P, F, c1.lam, tol=TOL, prec=ffk.FP64)
    torch.cuda.synchronize()
    return {"t_total_s": time.perf_counter() - t0, "iters": int(rep.iters), "rel_res_true": rep.rel_res_true}


def headline_product(ffk, ctx, cfg, steps: int, warmup: int):
    """The headline: split-BF16 products at `cfg`, timed, then clocked per kernel."""
    import torch
    import synth
    s = synth.config_system(cfg)
    S = ffk.descriptor_build(ctx, torch.as_tensor(s.R, device="cuda"), cfg.sigma)
    v = torch.as_tensor(synth.random_vectors(S.n, 5), device="cuda")
    y = torch.empty_like(v)
    prec = ffk.BF16X3
    log("headline: %d split-BF16 products at %s after %d untimed" % (steps, cfg.name, warmup))
    ms = time_mvm(ffk, ctx, S, v, prec, steps, warmup)
    # second pass with an event pair around every launch of each kernel
    ffk.clock_enable(ctx, 1)
    for _ in range(steps):
        ffk.kernel_mvm(ctx, S, v, y, prec=prec)
    clocks = ffk.clock_read(ctx)
    ffk.clock_enable(ctx, 0)
    clock_ms = {k: {"total_ms": t, "launches": c, "avg_ms": (t / c if c else None)} for k, (t, c) in clocks.items()
                if c}
    log("headline clocks:", json.dumps({k: round(v["avg_ms"], 4) for k, v in clock_ms.items()}))
    N, D = cfg.N, cfg.D
    dom = max(("gemm1", "gemm2"), key=lambda k: clock_ms[k]["total_ms"])
    _, amount, _ = kernel_model(dom, N, D, S.n, 0, 4)
    avg_s = clock_ms[dom]["avg_ms"] * 1e-3
    ach = amount / avg_s / 1e12
    roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["bf16x3"], "unit": "TFLOP/s",
            "frac": ach / PEAK_TFLOPS["bf16x3"], "traffic": measured_traffic(dom, cfg.name, "bf16x3"),
            "avg_launch_ms": clock_ms[dom]["avg_ms"], "launches": clock_ms[dom]["launches"],
            "algorithmic_per_launch": amount, "algorithmic_unit": "flop",
            "executed_tflops": 3 * ach, "executed_peak": PEAK_TFLOPS["bf16"],
            "executed_frac": 3 * ach / PEAK_TFLOPS["bf16"],
            "note": "split BF16: three BF16 MFMA products per product; algorithmic flops against the BF16 peak / 3 "
                    "equal executed flops against the BF16 peak"}
    other = {}
    for k in ("gemm1", "gemm2"):
        _, amt, _ = kernel_model(k, N, D, S.n, 0, 4)
        other[k] = {"avg_ms": clock_ms[k]["avg_ms"], "tflops": amt / (clock_ms[k]["avg_ms"] * 1e-3) / 1e12,
                    "executed_tflops": 3 * amt / (clock_ms[k]["avg_ms"] * 1e-3) / 1e12}
    rates = mvm_rates(ffk, ctx, cfg, S, v, max(3, steps // 4), 1, precs=("bf16", "fp32", "fp64"))
    tf = mvm_flops(N, D) / ms / 1e9
    rates["bf16x3"] = {"ms": ms, "tflops": tf, "frac_peak": tf / PEAK_TFLOPS["bf16x3"], "executed_tflops": 3 * tf}
    rates["shape"] = {"M": cfg.M, "N": N, "D": D, "n": S.n}
    del S, v, y
    torch.cuda.synchronize()
    return ms, roof, clock_ms, other, rates


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed headline products")
    ap.add_argument("--warmup", type=int, default=3, help="untimed headline products before the timed ones")
    ap.add_argument("--config", default="m60_n20000", help="headline workload (kernel product)")
    ap.add_argument("--solve-config", default="m21_n2000", help="workload of the time-to-solution comparison")
    ap.add_argument("--solve-steps", type=int, default=3, help="timed mixed learned solves")
    ap.add_argument("--solve-warmup", type=int, default=1)
    ap.add_argument("--mvm-configs", default="m9_n200,m21_n2000,m42_n5000,m21_n10000",
                    help="comma list of further systems for kernel-product rates")
    ap.add_argument("--mvm-steps", type=int, default=20)
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-solution comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle")
    ap.add_argument("--train-systems", type=int, default=4, help="small systems labelled for the score network")
    ap.add_argument("--train-n", type=int, default=500, help="geometries per training system")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--kernels-only", type=int, default=0,
                    help="counter-collection mode: build the solve workload once, run this many preconditioner "
                         "applies and products, plus a plain copy of known size for calibration; no JSON line")
    ap.add_argument("--mvm-only", type=int, default=0,
                    help="counter-collection mode: a plain copy of known size for calibration, then this many "
                         "kernel products per precision at each --mvm-configs shape (after one untimed product "
                         "each); no JSON line")
    ap.add_argument("--mvm-precs", default="bf16,bf16x3,fp32,fp64", help="precisions of --mvm-only")
    a = ap.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only (--gpus %d requested); how the solve would shard over several GPUs "
              "is a design note, not part of this library." % max(a.gpus, world), file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2212_12737_amd import ffk

    cfg_h = synth.CONFIGS[a.config]
    cpu = None
    if not (a.no_cpu or a.mvm_only or a.kernels_only):
        # before this process initialises the GPU: the oracle runs in forked workers
        cpu = cpu_baseline(cfg_h)
        log("cpu oracle:", json.dumps(cpu))

    ctx = ffk.create(0)

    if a.mvm_only:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        y = torch.empty_like(x)
        y.copy_(x)                           # calibration: 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        del x, y
        for c in [c for c in a.mvm_configs.split(",") if c]:
            cc = synth.CONFIGS[c]
            sc = synth.config_system(cc)
            Sc = ffk.descriptor_build(ctx, torch.as_tensor(sc.R, device="cuda"), cc.sigma)
            vc = torch.as_tensor(synth.random_vectors(Sc.n, 5), device="cuda")
            for prec in a.mvm_precs.split(","):
                ffk.kernel_mvm(ctx, Sc, vc, prec=ffk.PRECISIONS[prec])
                torch.cuda.synchronize()
                log("products %s %s: %d after one untimed" % (c, prec, a.mvm_only))
                for _ in range(a.mvm_only):
                    ffk.kernel_mvm(ctx, Sc, vc, prec=ffk.PRECISIONS[prec])
                torch.cuda.synchronize()
            del Sc, vc
        log("mvm-only done")
        return 0

    if a.kernels_only:
        cfg = synth.CONFIGS[a.solve_config]
        s = synth.config_system(cfg)
        R = torch.as_tensor(s.R, device="cuda")
        n = R.numel()
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").normal_()
        y = torch.empty_like(x)
        y.copy_(x)                           # calibration: 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        S = ffk.descriptor_build(ctx, R, cfg.sigma)
        idx = ffk.nystrom_select(ctx, S, cfg.strategy, cfg.k, lam=cfg.lam, seed=cfg.sel_seed)
        P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
        v = torch.as_tensor(synth.random_vectors(n, 5), device="cuda")
        for _ in range(a.kernels_only):
            ffk.precond_apply(ctx, P, v)
            ffk.kernel_mvm(ctx, S, v, prec=ffk.BF16X3)
        torch.cuda.synchronize()
        log("kernels-only done: %d applies and products, k_eff %d" % (a.kernels_only, P.k_eff))
        return 0

    # ---- headline: the split-BF16 kernel product at the largest workload
    ms, roof, head_clocks, head_gemms, head_rates = headline_product(ffk, ctx, cfg_h, a.steps, a.warmup)
    value = mvm_flops(cfg_h.N, cfg_h.D) / ms / 1e9
    log("headline: %.3f ms per product, %.1f TFLOP/s algorithmic (%.1f%% of the split-BF16 peak)"
        % (ms, value, 100 * value / PEAK_TFLOPS["bf16x3"]))
    log("roofline:", json.dumps(roof))

    rates = {cfg_h.name: head_rates}
    for c in [c for c in a.mvm_configs.split(",") if c]:
        cc = synth.CONFIGS[c]
        sc = synth.config_system(cc)
        Sc = ffk.descriptor_build(ctx, torch.as_tensor(sc.R, device="cuda"), cc.sigma)
        vc = torch.as_tensor(synth.random_vectors(Sc.n, 5), device="cuda")
        rates[c] = mvm_rates(ffk, ctx, cc, Sc, vc, a.mvm_steps, 3)
        rates[c]["shape"] = {"M": cc.M, "N": cc.N, "D": cc.D, "n": Sc.n}
        del Sc, vc

    # ---- time to solution at the solve workload
    solve_out = None
    ok_all = True
    if not a.no_solve:
        cfg = synth.CONFIGS[a.solve_config]
        s = synth.config_system(cfg)
        R = torch.as_tensor(s.R, device="cuda")
        F = torch.as_tensor(s.flat_forces(), device="cuda")
        n = R.numel()
        log("solves %s: M=%d N=%d D=%d n=%d k=%d lambda=%g" % (cfg.name, cfg.M, cfg.N, cfg.D, n, cfg.k, cfg.lam))
        net, setup = train_network(ffk, ctx, cfg, a.train_systems, a.train_n, a.train_steps)
        log("score network:", json.dumps(setup))
        for _ in range(a.solve_warmup):
            _, rec = solve(ffk, ctx, R, F, cfg, "mixed_learned", net)
            log("warmup solve", json.dumps(rec))
        ffk.clock_enable(ctx, CLOCK_STRIDE)
        recs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.solve_steps):
            _, rec = solve(ffk, ctx, R, F, cfg, "mixed_learned", net)
            recs.append(rec)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / a.solve_steps
        clocks = ffk.clock_read(ctx)
        ffk.clock_enable(ctx, 0)
        for r in recs:
            log("timed solve", json.dumps(r))
        ok_all = all(r["status"] == 0 and r["rel_res_true"] <= TOL for r in recs)
        keff = recs[-1]["k_eff"]
        clock_ms = {k: {"total_ms": t, "launches": c, "avg_ms": (t / c if c else None)}
                    for k, (t, c) in clocks.items()}
        modelled = [k for k in clock_ms if kernel_model(k, cfg.N, cfg.D, n, keff, 4) and clock_ms[k]["launches"]]
        dom = max(modelled, key=lambda k: clock_ms[k]["total_ms"])
        bound, amount, unit = kernel_model(dom, cfg.N, cfg.D, n, keff, 4)
        avg_s = clock_ms[dom]["avg_ms"] * 1e-3
        if bound == "mfma":
            ach = amount / avg_s / 1e12
            sroof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["bf16x3"],
                     "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["bf16x3"]}
        else:
            ach = amount / avg_s / 1e9
            sroof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(dom, cfg.name)}
        sroof.update({"avg_launch_ms": clock_ms[dom]["avg_ms"], "launches": clock_ms[dom]["launches"],
                      "algorithmic_per_launch": amount, "algorithmic_unit": unit})
        arms = {"mixed_learned": recs[-1]}
        for arm in ("fp64_learned", "mixed_uniform", "mixed_pivchol", "fp64_pivchol"):
            _, arms[arm] = solve(ffk, ctx, R, F, cfg, arm, net)
            log(arm, json.dumps(arms[arm]))
            ok_all = ok_all and arms[arm]["status"] == 0
        tt = {k: v["t_total_s"] for k, v in arms.items()}
        tt["mixed_learned"] = sec
        solve_out = {
            "workload": "%s: M=%d atoms, N=%d geometries, n=%d unknowns, D=%d, lambda=%g, k=%d Nystroem; full "
                        "solve (descriptor, selection, preconditioner build, PCG to a true FP64 relative "
                        "residual of 1e-6)" % (cfg.name, cfg.M, cfg.N, n, cfg.D, cfg.lam, cfg.k),
            "s_per_solve_mixed_learned": sec, "steps": a.solve_steps, "warmup": a.solve_warmup,
            "converged": ok_all,
            "speedup": {
                "precision_at_learned_columns (fp64_learned / mixed_learned)": tt["fp64_learned"] / sec,
                "precision_at_pivchol_columns (fp64_pivchol / mixed_pivchol)": tt["fp64_pivchol"]
                / tt["mixed_pivchol"],
                "network_over_uniform (mixed_uniform / mixed_learned)": tt["mixed_uniform"] / sec,
                "learned_over_workload_selection (mixed_pivchol / mixed_learned)": tt["mixed_pivchol"] / sec,
                "mixed_learned_over_plain_fp64 (fp64_pivchol / mixed_learned)": tt["fp64_pivchol"] / sec},
            "solves": arms, "learned_setup": setup, "roofline": sroof,
            "iteration_roofline": iteration_roofline(cfg, n, keff, recs[-1]),
            "kernel_clocks_ms": clock_ms,
        }
        del net

    if cpu is not None:
        cpu["small_workload"]["gpu_fp64_solve"] = small_gpu_solve(ffk, ctx)

    out = {
        "metric": "kernel-MVM TFLOP/s; PCG time to 1e-6 residual, mixed+learned vs plain FP64",
        "value": value, "unit": "TFLOP/s (algorithmic, F = 6 N^2 D + 24 N D per product; split-BF16 products)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3 (split BF16 on MFMA, FP32 accumulation, FP64 constant and row-sum terms)",
        "data": "synthetic",
        "config": {"workload": "%s: kernel matrix-vector product y = K v, M=%d atoms, N=%d geometries, "
                               "n=%d unknowns, D=%d inverse distances, Matern-5/2 sigma=%g"
                               % (cfg_h.name, cfg_h.M, cfg_h.N, 3 * cfg_h.M * cfg_h.N, cfg_h.D, cfg_h.sigma),
                   "M": cfg_h.M, "N": cfg_h.N, "n": 3 * cfg_h.M * cfg_h.N, "D": cfg_h.D,
                   "precision": "bf16x3", "parallelism": "single GPU"},
        "roofline": roof,
        "headline_kernel_clocks_ms": head_clocks,
        "headline_gemms": head_gemms,
        "mvm_tflops": rates,
        "time_to_solution": solve_out,
        "largest_workload_solve": "not run: estimated above one benchmark job (iterations x time per iteration "
                                  "at n = 3.6M, k = 8000)",
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0 if ok_all else 1


if __name__ == "__main__":
    sys.exit(main())

"""Selection study: PCG with learned, uniform, leverage and pivoted-Cholesky
columns on one system, with the score network trained on exact ridge-leverage
labels of smaller systems of the same molecule.

    python -m paper_2212_12737_amd.study labels  --config m21_n10000 --out DIR [--first 0 --count 20]
    python -m paper_2212_12737_amd.study compare --config m21_n10000 --labels DIR [--steps 3000]
    python -m paper_2212_12737_amd.study rot --config m21_n2000 [--sweep-N 250,500,1000]
    python -m paper_2212_12737_amd.study spectrum --config m21_n2000 [--spec-N 100 --spec-ks 100,400,1600]
    python -m paper_2212_12737_amd.study sym --config m21_n2000 [--sym-N 1000 --sym-orders 1,2,4,8]
    python -m paper_2212_12737_amd.study long --config m60_n20000 --state-out DIR [--state-in PREV --deadline-s 1000]

`labels` computes the exact labels (dense FP64 Cholesky on the GPU, about a
minute per N = 2000 system) and saves one .npy per training system, so they
can be produced over several runs; `compare` trains the network from them and
prints one JSON line per selection strategy.  `rot` measures the rule of thumb
for the preconditioner size (section 4.3): a k-sweep of PCG iterations on
small systems, the power-law fit, and the workload solved at the predicted
sizes and over a grid of k.  `spectrum` compares the spectrum of the
preconditioned matrix across strategies and sizes with the optimal rank-k
preconditioner (section 4.1), on a small system.  `sym` times the kernel
symmetrized over groups of atom permutations (product and solve).  `long` runs
the workload's solve in segments of one job each, resuming PCG from the saved
alpha and search direction.  Every step of the solver
runs in libffkrr; the dense eigen-analysis of `spectrum` runs on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import ffk, learned


def _config(name):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    return synth, synth.CONFIGS[name]


def _system(ctx, synth, cfg, N, disp_seed):
    s = synth.config_system(cfg, N=N, disp_seed=disp_seed)
    return s, ffk.descriptor_build(ctx, torch.as_tensor(s.R, device=ctx.torch_device), cfg.sigma)


def labels(ctx, config, out, first, count):
    synth, cfg = _config(config)
    ex = cfg.extra
    os.makedirs(out, exist_ok=True)
    for t in range(first, first + count):
        t0 = time.perf_counter()
        _, S = _system(ctx, synth, cfg, ex["train_N"], ex["train_disp_seed0"] + t)
        y = learned.make_labels(ctx, S, cfg.lam)
        np.save(os.path.join(out, "labels_%02d.npy" % t), y.cpu().numpy())
        print(json.dumps({"train_system": t, "seconds": time.perf_counter() - t0,
                          "label_spread": float(y.max() - y.min())}), flush=True)


def compare(ctx, config, label_dir, steps, arms):
    synth, cfg = _config(config)
    ex = cfg.extra
    systems, ys = [], []
    for t in range(ex["train_systems"]):
        _, S = _system(ctx, synth, cfg, ex["train_N"], ex["train_disp_seed0"] + t)
        systems.append(S)
        ys.append(torch.as_tensor(np.load(os.path.join(label_dir, "labels_%02d.npy" % t)), device=ctx.torch_device))
    t0 = time.perf_counter()
    net, log = learned.train(ctx, systems, ys, H=256, steps=steps, batch=256, lr=1e-3, seed=7, log_every=steps // 4)
    torch.cuda.synchronize()
    print(json.dumps({"train_seconds": time.perf_counter() - t0, "losses": log.losses}), flush=True)
    del systems
    s, S = _system(ctx, synth, cfg, cfg.N, ex["test_disp_seed"])
    F = torch.as_tensor(s.flat_forces(), device=ctx.torch_device)
    for arm in arms:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if arm == "learned":
            idx = learned.select(ctx, net, S, cfg.k, seed=cfg.sel_seed)
        else:
            idx = ffk.nystrom_select(ctx, S, arm, cfg.k, lam=cfg.lam, seed=cfg.sel_seed,
                                     pilot=cfg.k if arm == "leverage" else 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, rep = ffk.pcg_solve(ctx, S, P, F, cfg.lam, tol=1e-6, max_iter=40000, prec=ffk.BF16X3,
                               refresh_every=ffk.MIXED_REFRESH, escalate=True, switch_below=ffk.MIXED_SWITCH_BELOW,
                               switch_from=ffk.MIXED_SWITCH_FROM)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(json.dumps({"selection": arm, "k_eff": P.k_eff, "iters": rep.iters, "status": rep.status,
                          "rel_res_true": rep.rel_res_true, "escalations": rep.n_escalations,
                          "t_select_s": t1 - t0, "t_build_s": t2 - t1, "t_pcg_s": t3 - t2, "t_total_s": t3 - t0}),
              flush=True)
        del P


def _solve_at_k(ctx, S, F, cfg, k, arm, seed):
    """Leverage selection (pilot of k columns), build, PCG to 1e-6; one record."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = ffk.nystrom_select(ctx, S, "leverage", k, lam=cfg.lam, seed=seed, pilot=k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mixed = arm == "mixed"
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32 if mixed else ffk.FP64)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _, rep = ffk.pcg_solve(ctx, S, P, F, cfg.lam, tol=1e-6, max_iter=3 * S.n, prec=ffk.BF16X3 if mixed else ffk.FP64,
                           refresh_every=ffk.MIXED_REFRESH, escalate=True,
                           switch_below=ffk.MIXED_SWITCH_BELOW if mixed else 0.0, switch_from=ffk.MIXED_SWITCH_FROM)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rec = {"n": S.n, "k": k, "k_eff": P.k_eff, "arm": arm, "iters": rep.iters, "iters_over_n": rep.iters / S.n,
           "status": rep.status, "rel_res_true": rep.rel_res_true, "t_select_s": t1 - t0, "t_build_s": t2 - t1,
           "t_pcg_s": t3 - t2, "t_total_s": t3 - t0}
    del P
    return rec


def _product_ms(ctx, S, reps=10):
    """Mean time of the FP64 kernel product on S, in seconds."""
    v = torch.ones(S.n, dtype=torch.float64, device=ctx.torch_device)
    ffk.kernel_mvm(ctx, S, v, prec=ffk.FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ffk.kernel_mvm(ctx, S, v, prec=ffk.FP64)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def rule_of_thumb(ctx, config, sweep_N, ks, grid, arms):
    """Section 4.3: the PCG iteration count against the preconditioner size k
    on small systems of the workload's molecule (leverage selection, as the
    paper's analysis), the power-law fit #/n = (k_min/k)^m per system size,
    the sizes it predicts for the workload (Eq. 8, with the fitted and with the
    default m = 1, k_min = 100, and with costs measured on the largest sweep
    system) and the 1%-baseline, then the full solve of the workload over a
    grid of k that contains all of them, so that each heuristic is priced
    against the best measured k."""
    synth, cfg = _config(config)
    fits, sweep_rows = [], []
    for N in sweep_N:
        s, S = _system(ctx, synth, cfg, N, cfg.disp_seed + 3000 + N)
        F = torch.as_tensor(s.flat_forces(), device=ctx.torch_device)
        rows = []
        for k in ks:
            if k > S.n // 4:
                continue
            rec = _solve_at_k(ctx, S, F, cfg, k, "fp64", cfg.sel_seed)
            rec["sweep_N"] = N
            print(json.dumps(rec), flush=True)
            if rec["status"] == 0:
                rows.append(rec)
        kmin, m = ffk.rot_fit([r["k"] for r in rows], [r["iters"] for r in rows], S.n)
        fits.append((S.n, kmin, m))
        sweep_rows = rows
        t_mvm_sweep = _product_ms(ctx, S)
        print(json.dumps({"fit_n": S.n, "k_min": kmin, "m": m, "points": len(rows)}), flush=True)
        del S
    n_fit, kmin, m = fits[-1]   # the largest sweep system
    s, S = _system(ctx, synth, cfg, cfg.N, cfg.disp_seed)
    F = torch.as_tensor(s.flat_forces(), device=ctx.torch_device)
    # costs of the calibrated form, from the largest sweep system: time per
    # iteration a + b k and build time c k^2 by least squares; b and c scale
    # with n (the apply streams n values per column, the build costs k^2 n),
    # a with the measured FP64 product time at the two sizes
    ks = np.array([r["k"] for r in sweep_rows], dtype=np.float64)
    t_it = np.array([r["t_pcg_s"] / r["iters"] for r in sweep_rows])
    t_bd = np.array([r["t_select_s"] + r["t_build_s"] for r in sweep_rows])
    b_s, a_s = np.polyfit(ks, t_it, 1)
    c_s = float(np.sum(t_bd * ks ** 2) / np.sum(ks ** 4))
    scale = S.n / n_fit
    a_w = max(a_s, 1e-9) * _product_ms(ctx, S) / t_mvm_sweep
    costs = {"a_s": a_w, "b_s_per_k": max(b_s, 0.0) * scale, "c_s_per_k2": c_s * scale}
    heur = {"rot_specific": ffk.rule_of_thumb(S.n, kmin, m), "rot_default": ffk.rule_of_thumb(S.n),
            "rot_calibrated": ffk.rule_of_thumb_calibrated(S.n, kmin, m, costs["a_s"], costs["b_s_per_k"],
                                                           costs["c_s_per_k2"]),
            "one_percent": max(1, round(S.n / 100)), "workload_k": cfg.k}
    print(json.dumps({"workload_n": S.n, "fit_from_n": n_fit, "k_min": kmin, "m": m, "costs": costs,
                      "predicted": heur}), flush=True)
    kgrid = sorted(set(list(grid) + list(heur.values())))
    for arm in arms:
        recs = []
        for k in kgrid:
            rec = _solve_at_k(ctx, S, F, cfg, k, arm, cfg.sel_seed)
            print(json.dumps(rec), flush=True)
            recs.append(rec)
        ok = [r for r in recs if r["status"] == 0]
        best = min(ok, key=lambda r: r["t_total_s"])
        rel = {h: next(r["t_total_s"] for r in recs if r["k"] == kk) / best["t_total_s"] for h, kk in heur.items()}
        print(json.dumps({"arm": arm, "best_k": best["k"], "best_total_s": best["t_total_s"],
                          "relative_time": rel}), flush=True)


def svd_preconditioned_spectrum(eigs, lam, k):
    """Eigenvalues, descending, of P^-1 K_lambda for the optimal rank-k
    preconditioner P = U_k diag(e_1..e_k) U_k^T + lam I built from the k
    dominant eigenpairs of K (section 2.2): the k dominant directions map to
    (e_i + lam)/(e_i + lam) = 1, every other one to (e_i + lam)/lam."""
    e = np.sort(np.asarray(eigs, dtype=np.float64))[::-1]
    k = min(int(k), e.size)
    return np.sort(np.concatenate([np.ones(k), (e[k:] + lam) / lam]))[::-1]


def nystrom_preconditioned_spectrum(K, L, lam):
    """Eigenvalues, descending, of P^-1 K_lambda with P = L L^T + lam I (Eq. 3),
    from the symmetric-definite pencil (K + lam I, P)."""
    import scipy.linalg as sla
    n = K.shape[0]
    Kl = K + lam * np.eye(n)
    P = L @ L.T + lam * np.eye(n)
    return sla.eigh(Kl, P, eigvals_only=True)[::-1]


def spectrum(ctx, config, N, ks, strategies, top):
    """Section 4.1: the spectrum of P^-1 K_lambda for several preconditioner
    sizes k and selection strategies on a small system of the workload's
    molecule, against the optimal rank-k (eigendecomposition, "SVD")
    preconditioner, with the FP64 PCG iteration count of each.  K comes from
    the library's column kernel, L from the library's factor; the dense
    eigen-analysis runs on the host (double precision LAPACK), which limits
    this study to small n."""
    synth, cfg = _config(config)
    s, S = _system(ctx, synth, cfg, N, cfg.disp_seed + 5000 + N)
    n, lam = S.n, cfg.lam
    F = torch.as_tensor(s.flat_forces(), device=ctx.torch_device)
    K = ffk.kernel_columns(ctx, S, torch.arange(n)).cpu().numpy()
    K = 0.5 * (K + K.T)
    eigs = np.linalg.eigvalsh(K)[::-1]
    print(json.dumps({"n": n, "lambda": lam, "kappa_K_lambda": float((eigs[0] + lam) / (max(eigs[-1], 0.0) + lam)),
                      "eig_top": [float(eigs[i]) for i in (0, 9, 99, min(999, n - 1))]}), flush=True)
    out = {"eigs_K": eigs[:top]}
    for k in ks:
        sv = svd_preconditioned_spectrum(eigs, lam, k)
        row = {"k": k, "strategy": "svd", "kappa": float(sv[0] / sv[-1]), "top": [float(sv[i]) for i in (0, 9, 49, top - 1)]}
        print(json.dumps(row), flush=True)
        out["svd_%d" % k] = sv[:top]
        for strat in strategies:
            idx = ffk.nystrom_select(ctx, S, strat, k, lam=lam, seed=cfg.sel_seed, pilot=k if strat == "leverage" else 0)
            P = ffk.precond_build(ctx, S, idx, lam, store=ffk.FP64)
            L = ffk.precond_export(ctx, P, n).cpu().numpy()
            _, rep = ffk.pcg_solve(ctx, S, P, F, lam, tol=1e-6, max_iter=4 * n, prec=ffk.FP64)
            w = nystrom_preconditioned_spectrum(K, L, lam)
            row = {"k": k, "strategy": strat, "k_eff": P.k_eff, "kappa": float(w[0] / w[-1]),
                   "kappa_over_svd": float((w[0] / w[-1]) / (sv[0] / sv[-1])),
                   "top": [float(w[i]) for i in (0, 9, 49, top - 1)], "pcg_iters": rep.iters, "status": rep.status}
            print(json.dumps(row), flush=True)
            out["%s_%d" % (strat, k)] = w[:top]
            del P
    return out


def transposition_group(M, t):
    """The group of order 2^t generated by the disjoint swaps (0 1), (2 3), ...,
    as S x M atom permutations (identity first)."""
    rows = []
    for mask in range(1 << t):
        p = list(range(M))
        for j in range(t):
            if mask >> j & 1:
                p[2 * j], p[2 * j + 1] = p[2 * j + 1], p[2 * j]
        rows.append(p)
    return np.array(rows, dtype=np.int32)


def symmetry(ctx, config, N, orders, reps):
    """The kernel symmetrized over groups of atom permutations (sGDML form):
    FP64 product time against the group order, and a PCG solve (uniform
    columns, FP64 products and factor) with the symmetrized kernel."""
    synth, cfg = _config(config)
    s, S = _system(ctx, synth, cfg, N, cfg.disp_seed)
    F = torch.as_tensor(s.flat_forces(), device=ctx.torch_device)
    v = torch.ones(S.n, dtype=torch.float64, device=ctx.torch_device)
    for order in orders:
        t = int(round(np.log2(order)))
        ffk.set_symmetries(ctx, S, transposition_group(S.M, t))
        ffk.kernel_mvm(ctx, S, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ffk.kernel_mvm(ctx, S, v)
        torch.cuda.synchronize()
        t_mvm = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        idx = ffk.nystrom_select(ctx, S, "uniform", cfg.k, seed=cfg.sel_seed)
        P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, rep = ffk.pcg_solve(ctx, S, P, F, cfg.lam, tol=1e-6, max_iter=20000, prec=ffk.FP64)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        print(json.dumps({"group_order": order, "n": S.n, "k": cfg.k, "product_ms": 1e3 * t_mvm,
                          "build_s": t1 - t0, "pcg_iters": rep.iters, "pcg_s": t2 - t1, "status": rep.status,
                          "rel_res_true": rep.rel_res_true}), flush=True)
        del P
    ffk.set_symmetries(ctx, S, transposition_group(S.M, 0))


def _train_network(ctx, synth, cfg, train):
    """The score network from exact labels of `systems` systems of N
    geometries of the workload's molecule (displacement seeds disjoint from
    the workload's), trained for `steps` steps, as the benchmark trains it."""
    systems, N, steps = train
    S_tr, y_tr = [], []
    for t in range(systems):
        _, S = _system(ctx, synth, cfg, N, cfg.disp_seed + 1000 + t)
        S_tr.append(S)
        y_tr.append(learned.make_labels(ctx, S, cfg.lam))
        print(json.dumps({"training_system": t, "N": N, "labels": "exact ridge leverage"}), flush=True)
    net, _ = learned.train(ctx, S_tr, y_tr, H=256, steps=steps, batch=256, lr=1e-3, seed=7,
                           log_every=max(1, steps // 4))
    return net


def long_solve(ctx, config, state_in, state_out, deadline_s, chunk, progress, train, max_chunks=0):
    """The workload's mixed-precision solve (learned columns, L stored FP32, the
    benchmark's schedule) run in segments that each fit one job: every
    segment rebuilds the system and the preconditioner from the saved column
    indices, resumes PCG from the saved alpha and search direction (true
    residual in FP64, direction kept), runs it in chunks of `chunk`
    iterations until `deadline_s` seconds after the start, and saves alpha,
    the direction and a log.  One JSON line per chunk and per segment."""
    t_start = time.perf_counter()
    synth, cfg = _config(config)
    os.makedirs(state_out, exist_ok=True)
    log_path = os.path.join(state_out, "log.json")
    meta = {"config": config, "segments": []}
    if state_in and os.path.exists(os.path.join(state_in, "log.json")):
        with open(os.path.join(state_in, "log.json")) as f:
            meta = json.load(f)
    seg = {"segment": len(meta["segments"])}
    s = synth.config_system(cfg)
    dev = ctx.torch_device
    S = ffk.descriptor_build(ctx, torch.as_tensor(s.R, device=dev), cfg.sigma)
    F = torch.as_tensor(s.flat_forces(), device=dev)
    torch.cuda.synchronize()
    seg["t_system_s"] = time.perf_counter() - t_start
    t0 = time.perf_counter()
    idx_in = os.path.join(state_in, "idx.npy") if state_in else None
    if idx_in and os.path.exists(idx_in):
        idx = torch.as_tensor(np.load(idx_in), device=dev)
        seg["selection"] = "saved"
    else:
        net = _train_network(ctx, synth, cfg, train) if cfg.strategy == "learned" else None
        idx = learned.select(ctx, net, S, cfg.k, cfg.sel_seed) if net is not None else \
            ffk.nystrom_select(ctx, S, cfg.strategy, cfg.k, lam=cfg.lam, seed=cfg.sel_seed)
        seg["selection"] = cfg.strategy
    torch.cuda.synchronize()
    seg["t_select_s"] = time.perf_counter() - t0
    print(json.dumps({"selected": seg["selection"], "seconds": seg["t_select_s"]}), flush=True)
    t0 = time.perf_counter()
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32, lowmem=True)
    if P.k_eff < 0.95 * cfg.k and seg["selection"] != "saved":   # the rank collapsed: pivoted Cholesky
        del P
        idx = ffk.nystrom_select(ctx, S, "pivchol", cfg.k)
        P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32, lowmem=True)
        seg["selection"] = "pivchol-fallback"
    np.save(os.path.join(state_out, "idx.npy"), idx.cpu().numpy())
    torch.cuda.synchronize()
    seg["t_build_s"] = time.perf_counter() - t0
    seg["k_eff"] = int(P.k_eff)
    resume = bool(state_in) and os.path.exists(os.path.join(state_in, "alpha.npy"))
    if resume:
        alpha = torch.as_tensor(np.load(os.path.join(state_in, "alpha.npy")), device=dev)
        direction = torch.as_tensor(np.load(os.path.join(state_in, "direction.npy")), device=dev)
    else:
        alpha = torch.zeros(S.n, dtype=torch.float64, device=dev)
        direction = torch.empty(S.n, dtype=torch.float64, device=dev)
    prec = meta.get("prec", ffk.BF16X3)
    print(json.dumps({"segment_start": seg, "resume": resume}), flush=True)
    seg.update({"iters": 0, "t_pcg_s": 0.0, "chunks": 0})
    status, t_chunk = 1, 0.0
    while time.perf_counter() - t_start + 1.3 * t_chunk + 10.0 < deadline_s and \
            (max_chunks <= 0 or seg["chunks"] < max_chunks):
        t0 = time.perf_counter()
        alpha, rep = ffk.pcg_solve(ctx, S, P, F, cfg.lam, tol=1e-6, max_iter=chunk, prec=prec,
                                   refresh_every=ffk.MIXED_REFRESH, escalate=True,
                                   switch_below=ffk.MIXED_SWITCH_BELOW, switch_from=ffk.MIXED_SWITCH_FROM,
                                   progress_every=progress, alpha=alpha, direction=direction, resume=resume)
        torch.cuda.synchronize()
        t_chunk = time.perf_counter() - t0
        resume = True
        if rep.n_escalations > 0:   # an escalation moved the products up the ladder: keep them there
            prec = int(rep.final_prec)
        status = int(rep.status)
        seg["iters"] += int(rep.iters)
        seg["t_pcg_s"] += t_chunk
        seg["chunks"] += 1
        seg["rel_res_true"] = rep.rel_res_true
        print(json.dumps({"chunk": seg["chunks"], "iters": int(rep.iters), "seconds": t_chunk,
                          "rel_res_true": rep.rel_res_true, "status": status, "final_prec": prec,
                          "n_escalations": int(rep.n_escalations)}), flush=True)
        if status != 1:   # converged, or an error: stop here
            break
    seg["status"] = status
    seg["t_segment_s"] = time.perf_counter() - t_start
    np.save(os.path.join(state_out, "alpha.npy"), alpha.cpu().numpy())
    np.save(os.path.join(state_out, "direction.npy"), direction.cpu().numpy())
    meta["segments"].append(seg)
    meta["prec"] = prec
    meta["iters_total"] = sum(g["iters"] for g in meta["segments"])
    meta["t_pcg_total_s"] = sum(g["t_pcg_s"] for g in meta["segments"])
    meta["t_total_s"] = sum(g["t_segment_s"] for g in meta["segments"])
    meta["status"] = status
    meta["rel_res_true"] = seg.get("rel_res_true")
    with open(log_path, "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps({"segment_done": seg, "iters_total": meta["iters_total"],
                      "t_pcg_total_s": meta["t_pcg_total_s"], "t_total_s": meta["t_total_s"]}), flush=True)
    return meta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["labels", "compare", "rot", "spectrum", "sym", "long"])
    ap.add_argument("--config", default="m21_n10000")
    ap.add_argument("--out", default="study_labels")
    ap.add_argument("--labels", default="study_labels")
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--count", type=int, default=20)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--arms", default=None, help="compare: selections; rot: fp64 and/or mixed")
    ap.add_argument("--sweep-N", default="250,500,1000", help="rot: geometries of the sweep systems")
    ap.add_argument("--ks", default="125,250,500,1000,2000,4000", help="rot: preconditioner sizes of the sweep")
    ap.add_argument("--grid", default="500,1000,2000,3000,4000,6000", help="rot: sizes tried on the workload")
    ap.add_argument("--spec-N", type=int, default=100, help="spectrum: geometries of the system")
    ap.add_argument("--spec-ks", default="100,400,1600", help="spectrum: preconditioner sizes")
    ap.add_argument("--spec-out", default=None, help="spectrum: .npz with the dominant eigenvalues")
    ap.add_argument("--sym-N", type=int, default=1000, help="sym: geometries of the system")
    ap.add_argument("--sym-orders", default="1,2,4,8", help="sym: group orders (powers of two)")
    ap.add_argument("--state-in", default=None, help="long: directory of the previous segment's state")
    ap.add_argument("--state-out", default="long_state", help="long: directory for this segment's state")
    ap.add_argument("--deadline-s", type=float, default=1000.0, help="long: seconds after start to stop by")
    ap.add_argument("--chunk", type=int, default=2000, help="long: PCG iterations between resumes")
    ap.add_argument("--progress", type=int, default=1000, help="long: PCG progress line every so many iterations")
    ap.add_argument("--train", default="4,500,2000", help="long: network training systems, N each, steps")
    ap.add_argument("--max-chunks", type=int, default=0, help="long: at most so many chunks (0: no limit)")
    a = ap.parse_args(argv)
    ctx = ffk.create(0)
    ints = lambda t: [int(x) for x in t.split(",")]
    if a.mode == "labels":
        labels(ctx, a.config, a.out, a.first, a.count)
    elif a.mode == "compare":
        compare(ctx, a.config, a.labels, a.steps, (a.arms or "learned,pivchol,uniform,leverage").split(","))
    elif a.mode == "rot":
        rule_of_thumb(ctx, a.config, ints(a.sweep_N), ints(a.ks), ints(a.grid), (a.arms or "fp64,mixed").split(","))
    elif a.mode == "long":
        long_solve(ctx, a.config, a.state_in, a.state_out, a.deadline_s, a.chunk, a.progress, ints(a.train),
                   a.max_chunks)
    elif a.mode == "sym":
        symmetry(ctx, a.config, a.sym_N, ints(a.sym_orders), 5)
    else:
        out = spectrum(ctx, a.config, a.spec_N, ints(a.spec_ks), (a.arms or "uniform,leverage,pivchol").split(","), 150)
        if a.spec_out:
            np.savez(a.spec_out, **out)


if __name__ == "__main__":
    main()

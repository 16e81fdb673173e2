"""Selection study: PCG with learned, uniform, leverage and pivoted-Cholesky
columns on one system, with the score network trained on exact ridge-leverage
labels of smaller systems of the same molecule.

    python -m paper_2212_12737_amd.study labels  --config m21_n10000 --out DIR [--first 0 --count 20]
    python -m paper_2212_12737_amd.study compare --config m21_n10000 --labels DIR [--steps 3000]

`labels` computes the exact labels (dense FP64 Cholesky on the GPU, about a
minute per N = 2000 system) and saves one .npy per training system, so they
can be produced over several runs; `compare` trains the network from them and
prints one JSON line per selection strategy.  Every step runs in libffkrr.
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
        _, rep = ffk.pcg_solve(ctx, S, P, F, cfg.lam, tol=1e-6, max_iter=40000, prec=ffk.BF16X3, refresh_every=10,
                               escalate=True, switch_below=0.3)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(json.dumps({"selection": arm, "k_eff": P.k_eff, "iters": rep.iters, "status": rep.status,
                          "rel_res_true": rep.rel_res_true, "escalations": rep.n_escalations,
                          "t_select_s": t1 - t0, "t_build_s": t2 - t1, "t_pcg_s": t3 - t2, "t_total_s": t3 - t0}),
              flush=True)
        del P


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["labels", "compare"])
    ap.add_argument("--config", default="m21_n10000")
    ap.add_argument("--out", default="study_labels")
    ap.add_argument("--labels", default="study_labels")
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--count", type=int, default=20)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--arms", default="learned,pivchol,uniform,leverage")
    a = ap.parse_args(argv)
    ctx = ffk.create(0)
    if a.mode == "labels":
        labels(ctx, a.config, a.out, a.first, a.count)
    else:
        compare(ctx, a.config, a.labels, a.steps, a.arms.split(","))


if __name__ == "__main__":
    main()

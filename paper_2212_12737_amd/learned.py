"""Learned inducing-column selection (orchestration over the C ABI).

Labels are exact ridge leverage scores of small training systems (dense FP64
Cholesky on the GPU), summed per geometry and log-centred; the score network
D -> H -> H -> 1 is trained with the library's FP32 forward/backward/Adam
kernels on contiguous minibatches; selection samples columns by
Efraimidis-Spirakis keys with per-geometry weights exp(network output),
computed with BF16 MFMA inference.  A preconditioner whose rank collapses
(k_eff < 0.95 k) falls back to pivoted-Cholesky selection.

Every arithmetic step runs in libffkrr; this module only sequences calls and
slices device buffers.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import ffk


@dataclass
class TrainLog:
    steps: int
    losses: list


def make_labels(ctx, sys, lam: float) -> torch.Tensor:
    """Per-geometry targets y_g = log sum_{c in g} tau_c - mean (exact tau)."""
    tau = ffk.exact_rls(ctx, sys, lam)
    return ffk.block_log_scores(ctx, tau, sys.N, sys.M)


def train(ctx, systems, labels, H: int = 256, steps: int = 2000, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, log_every: int = 100):
    """Train the score network on the descriptors of `systems` against `labels`."""
    D = systems[0].D
    net = ffk.mlp_create(ctx, D, H, seed)
    Ntot = sum(s.N for s in systems)
    X = torch.empty((Ntot, D), dtype=torch.float32, device=ctx.torch_device)
    y = torch.empty(Ntot, dtype=torch.float32, device=ctx.torch_device)
    o = 0
    for s, lab in zip(systems, labels):
        ffk.mlp_prepare_inputs(ctx, net, s, standardize=False, out=X[o:o + s.N])
        y[o:o + s.N].copy_(lab)
        o += s.N
    ffk.mlp_fit_norm(ctx, net, X)
    o = 0
    for s in systems:
        ffk.mlp_prepare_inputs(ctx, net, s, standardize=True, out=X[o:o + s.N])
        o += s.N
    batch = min(batch, Ntot)
    nb = Ntot // batch
    losses = []
    for step in range(steps):
        b0 = (step % nb) * batch
        loss, grad = ffk.mlp_grad(ctx, net, X[b0:b0 + batch], y[b0:b0 + batch])
        ffk.mlp_adam_step(ctx, net, grad, lr)
        if log_every and (step % log_every == 0 or step == steps - 1):
            losses.append((step, float(loss.item())))
    return net, TrainLog(steps, losses)


def evaluate(ctx, net, systems, labels) -> float:
    """Mean squared error of the network on standardised inputs of `systems` (FP32 inference)."""
    err, cnt = 0.0, 0
    for s, lab in zip(systems, labels):
        X = ffk.mlp_prepare_inputs(ctx, net, s, standardize=True)
        out = ffk.mlp_forward(ctx, net, X, prec=ffk.FP32)
        err += float(((out - lab) ** 2).sum().item())
        cnt += s.N
    return err / cnt


def select(ctx, net, sys, k: int, seed: int):
    """Inducing columns sampled with the network's per-geometry weights."""
    w = ffk.mlp_scores(ctx, net, sys)
    return ffk.nystrom_select(ctx, sys, "scores", k, seed=seed, weights=w)


def build_with_fallback(ctx, net, sys, k: int, lam: float, seed: int, store=ffk.FP32):
    """Learned selection, falling back to pivoted Cholesky when the kept rank collapses."""
    idx = select(ctx, net, sys, k, seed)
    P = ffk.precond_build(ctx, sys, idx, lam, store=store)
    if P.k_eff < 0.95 * k:
        idx = ffk.nystrom_select(ctx, sys, "pivchol", k)
        P = ffk.precond_build(ctx, sys, idx, lam, store=store)
        return P, "pivchol-fallback"
    return P, "learned"

"""GPU parity of the score network (forward, backward, Adam, BF16 inference) with the FP64 oracle,
and the learned-selection pipeline on small systems."""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok
from oracle import mlp as omlp
from oracle import select as osel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffk():
    from paper_2212_12737_amd import ffk as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(ffk):
    return ffk.create(0)


def f32(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def setup(D=37, H=64, B=300, seed=0):
    rng = np.random.default_rng(seed)
    theta = (rng.normal(size=omlp.n_params(D, H)) * 0.3).astype(np.float32)
    X = rng.normal(size=(B, D)).astype(np.float32)
    y = rng.normal(size=B).astype(np.float32)
    return theta, X, y


@pytest.mark.parametrize("D,H,B", [(37, 64, 300), (210, 256, 513), (5, 128, 1)])
def test_forward_and_gradient_match_oracle(ffk, ctx, D, H, B):
    theta, X, y = setup(D, H, B, seed=D + B)
    net = ffk.mlp_create(ctx, D, H, 1)
    ffk.mlp_set_params(ctx, net, f32(theta))
    out = ffk.mlp_forward(ctx, net, f32(X), prec=ffk.FP32).cpu().numpy()
    ref = omlp.forward(theta.astype(np.float64), X.astype(np.float64), D, H)
    assert np.abs(out - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    loss, grad = ffk.mlp_grad(ctx, net, f32(X), f32(y))
    L, g = omlp.backward(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64), D, H)
    assert abs(loss.item() - L) <= 1e-4 * max(1.0, L)
    g_gpu = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g_gpu - g) <= 1e-4 * np.linalg.norm(g)
    # parameters round-trip unchanged
    assert np.array_equal(ffk.mlp_get_params(ctx, net).cpu().numpy(), theta)


def test_bf16_inference_close_to_fp32(ffk, ctx):
    D, H, B = 210, 256, 1000
    theta, X, _ = setup(D, H, B, seed=5)
    net = ffk.mlp_create(ctx, D, H, 1)
    ffk.mlp_set_params(ctx, net, f32(theta))
    o32 = ffk.mlp_forward(ctx, net, f32(X), prec=ffk.FP32).cpu().numpy()
    o16 = ffk.mlp_forward(ctx, net, f32(X), prec=ffk.BF16).cpu().numpy()
    ref = omlp.forward(theta.astype(np.float64), X.astype(np.float64), D, H)
    assert np.abs(o16 - ref).max() <= 3e-2 * np.abs(ref).max()
    assert np.abs(o32 - ref).max() <= 1e-4 * np.abs(ref).max()


def test_adam_matches_oracle(ffk, ctx):
    D, H, B = 11, 64, 64
    theta, X, y = setup(D, H, B, seed=9)
    net = ffk.mlp_create(ctx, D, H, 1)
    ffk.mlp_set_params(ctx, net, f32(theta))
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, 4):
        _, grad = ffk.mlp_grad(ctx, net, f32(X), f32(y))
        g = grad.cpu().numpy().astype(np.float64)
        ffk.mlp_adam_step(ctx, net, grad, 1e-2)
        th, m, v = omlp.adam_step(th, g, m, v, t, lr=1e-2)
        got = ffk.mlp_get_params(ctx, net).cpu().numpy().astype(np.float64)
        assert np.abs(got - th).max() <= 1e-5


def test_training_reduces_loss_and_scores_follow_network(ffk, ctx):
    from paper_2212_12737_amd import learned
    s = synth.make_system(6, 60, 0.08, True, 51, 52, 53)
    S = ffk.descriptor_build(ctx, torch.as_tensor(s.R, device="cuda"), 10.0)
    lam = 1e-6
    y = learned.make_labels(ctx, S, lam)
    # labels: exact block leverage sums of the oracle, log-centred
    tau = osel.exact_ridge_leverage(ok.dense_kernel(s.R, 10.0), lam)
    blk = np.log(tau.reshape(S.N, 3 * S.M).sum(1))
    np.testing.assert_allclose(y.cpu().numpy(), blk - blk.mean(), atol=2e-5)
    net, log = learned.train(ctx, [S], [y], H=64, steps=400, batch=60, lr=3e-3, seed=2, log_every=50)
    assert log.losses[-1][1] < 0.5 * log.losses[0][1]
    sc = ffk.mlp_scores(ctx, net, S).cpu().numpy()
    Xs = ffk.mlp_prepare_inputs(ctx, net, S, standardize=True)
    o32 = ffk.mlp_forward(ctx, net, Xs, prec=ffk.FP32).cpu().numpy()
    np.testing.assert_allclose(np.log(sc), o32, atol=0.05 * max(1.0, np.abs(o32).max()))
    idx = learned.select(ctx, net, S, 50, seed=3).cpu().numpy()
    assert len(idx) == 50 and len(set(idx.tolist())) == 50 and idx.min() >= 0 and idx.max() < S.n


def test_input_standardisation(ffk, ctx):
    """The network's inputs: raw descriptor rows as floats; fit_norm sets the
    column mean and inverse (population) standard deviation of given rows;
    set_norm installs any mean and inverse standard deviation."""
    s = synth.make_system(6, 120, 0.05, True, 81, 82, 83)
    S = ffk.descriptor_build(ctx, torch.as_tensor(s.R, device="cuda"), 10.0)
    net = ffk.mlp_create(ctx, S.D, 64, 5)
    raw = ffk.mlp_prepare_inputs(ctx, net, S, standardize=False).cpu().numpy()
    np.testing.assert_allclose(raw, ok.descriptor(s.R), rtol=1e-6)
    ffk.mlp_fit_norm(ctx, net, f32(raw))
    Xs = ffk.mlp_prepare_inputs(ctx, net, S, standardize=True).cpu().numpy()
    r64 = raw.astype(np.float64)
    np.testing.assert_allclose(Xs, (r64 - r64.mean(0)) / r64.std(0), rtol=1e-4, atol=2e-4)
    rng = np.random.default_rng(4)
    mean, istd = rng.normal(size=S.D), rng.uniform(0.5, 2.0, S.D)
    ffk.mlp_set_norm(ctx, net, f32(mean), f32(istd))
    Xs2 = ffk.mlp_prepare_inputs(ctx, net, S, standardize=True).cpu().numpy()
    np.testing.assert_allclose(Xs2, (r64 - mean.astype(np.float32)) * istd.astype(np.float32), rtol=1e-5, atol=1e-5)

"""Pins of the oracle MLP (learned column selection)."""
import numpy as np

from oracle import mlp


def _setup(D=7, H=5, B=11, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(size=mlp.n_params(D, H)) * 0.5
    X = rng.normal(size=(B, D))
    y = rng.normal(size=B)
    return theta, X, y


def test_backward_matches_central_differences():
    D, H = 7, 5
    theta, X, y = _setup(D, H)
    L, g = mlp.backward(theta, X, y, D, H)
    assert np.isclose(L, mlp.loss(theta, X, y, D, H), rtol=1e-14)
    h = 1e-6
    gfd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta); e[i] = h
        gfd[i] = (mlp.loss(theta + e, X, y, D, H) - mlp.loss(theta - e, X, y, D, H)) / (2 * h)
    assert np.abs(g - gfd).max() <= 1e-7 * np.abs(g).max()


def test_gelu_limits_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert mlp.gelu(0.0) == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([8.0])), [8.0], rtol=1e-14)
    np.testing.assert_allclose(mlp.gelu(np.array([-8.0])), [0.0], atol=1e-13)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-4)

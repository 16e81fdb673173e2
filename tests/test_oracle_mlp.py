"""Pins of the oracle MLP (learned column selection)."""
import os

import numpy as np
from scipy import integrate

from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def test_gelu_is_x_times_the_normal_integral_at_table_values():
    """gelu(x) = x Phi(x) with the exact normal integral: table values of Phi
    (a tanh-approximated GELU gives 0.841192 at x = 1 and fails here)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "normal_cdf.txt")) if l.strip() and not l.startswith("#")]
    x = np.array([float(r[0]) for r in rows])
    phi = np.array([float(r[1]) for r in rows])
    np.testing.assert_allclose(mlp.gelu(x), x * phi, rtol=1e-15, atol=0)
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) <= 1e-16
    assert abs(mlp.gelu(-1.0) + 0.15865525393145707) <= 1e-16


def test_gelu_against_quadrature_of_the_normal_density():
    """An erf-free route: Phi(x) by adaptive quadrature of exp(-t^2/2)/sqrt(2 pi)."""
    dens = lambda t: np.exp(-0.5 * t * t) / np.sqrt(2.0 * np.pi)
    for x in (-3.3, -0.7, 0.25, 1.9, 4.1):
        phi, _ = integrate.quad(dens, -np.inf, x, epsabs=1e-15, epsrel=1e-14)
        assert abs(mlp.gelu(x) - x * phi) <= 1e-13 * max(1.0, abs(x))


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-4)

"""FP64 oracle: the score-predicting MLP (learned column selection).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not part of the paper: the workload adds a small network that maps a
geometry's descriptor to a predicted (log) ridge-leverage block score, used to
sample inducing columns.  Architecture D -> H -> H -> 1 with exact-erf GELU,
mean-squared-error loss and Adam (Kingma & Ba, 2015).

Parameter layout (flat, float): W1 (H x D, row-major), b1 (H), W2 (H x H),
b2 (H), w3 (H), b3 (1).

Pins (tests/test_oracle_mlp.py): backward() against central finite
differences of loss(); Adam's first step equals lr * sign(g) per coordinate;
GELU by value, x Phi(x) at tabulated points of the normal integral and
against an erf-free quadrature of the normal density.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def n_params(D: int, H: int) -> int:
    return H * D + H + H * H + H + H + 1


def unpack(theta: np.ndarray, D: int, H: int):
    o = 0
    W1 = theta[o:o + H * D].reshape(H, D); o += H * D
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(theta, X, D, H, return_cache=False):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(theta, dtype=np.float64), D, H)
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    out = H2 @ w3 + b3
    if return_cache:
        return out, (X, Z1, H1, Z2, H2)
    return out


def loss(theta, X, y, D, H):
    out = forward(theta, X, D, H)
    return np.mean((out - y) ** 2)


def backward(theta, X, y, D, H):
    """(loss, gradient) of the mean squared error."""
    theta = np.asarray(theta, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(theta, D, H)
    out, (X, Z1, H1, Z2, H2) = forward(theta, X, D, H, return_cache=True)
    B = X.shape[0]
    diff = out - y
    dout = 2.0 * diff / B
    g_w3 = H2.T @ dout
    g_b3 = dout.sum()
    dZ2 = np.outer(dout, w3) * gelu_grad(Z2)
    g_W2 = dZ2.T @ H1
    g_b2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    g_W1 = dZ1.T @ X
    g_b1 = dZ1.sum(0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return np.mean(diff ** 2), grad


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v

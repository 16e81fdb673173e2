"""Pins of the oracle's random stream, samplers, incomplete Cholesky and leverage scores."""
import os

import numpy as np
import pytest

import synth
from oracle import kernel as ok
from oracle import select as osel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    got = osel.splitmix64(0, np.arange(3))
    assert [int(g) for g in got] == vals


def test_uniform01_range_and_uniformity():
    u = osel.uniform01(12345, 0, 200000)
    assert u.min() > 0.0 and u.max() <= 1.0
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    expect = len(u) / 50
    chi2 = ((hist - expect) ** 2 / expect).sum()
    assert chi2 < 100          # 49 dof; p ~ 1e-5 tail
    # streams are distinct
    assert not np.array_equal(osel.uniform01(1, 0, 10), osel.uniform01(1, 1, 10))


def test_uniform_selection_distinct_and_unbiased():
    n, k = 40, 8
    counts = np.zeros(n)
    for seed in range(3000):
        S = osel.select_uniform(n, k, seed)
        assert len(set(S.tolist())) == k
        counts[S] += 1
    freq = counts / 3000
    assert np.abs(freq - k / n).max() < 0.035


def test_weighted_sampling_first_draw_probability():
    """Efraimidis-Spirakis: the top key is item i with probability w_i / sum(w)."""
    w = np.array([1.0, 2.0, 3.0, 4.0])
    first = np.array([osel.select_weighted(w, 1, seed, 2)[0] for seed in range(20000)])
    freq = np.bincount(first, minlength=4) / len(first)
    np.testing.assert_allclose(freq, w / w.sum(), atol=0.012)


def test_score_weights_hand_case():
    """N = 2 geometries of M = 3 atoms: columns 0-8 carry geometry 0's score,
    9-17 geometry 1's; a score below the floor is raised to 1e-12."""
    w = osel.score_weights(np.array([0.25, 3.0]), 3)
    assert w.shape == (18,)
    assert w[:9].tolist() == [0.25] * 9 and w[9:].tolist() == [3.0] * 9
    w = osel.score_weights(np.array([0.0, -1.0, 5e-13, 2.0]), 3)
    assert w[:27].tolist() == [1e-12] * 27 and w[27:].tolist() == [2.0] * 9
    # repeated per geometry (not tiled): a tile/repeat mix-up fails here
    w = osel.score_weights(np.array([1.0, 2.0, 3.0]), 4)
    assert w.tolist() == [1.0] * 12 + [2.0] * 12 + [3.0] * 12


def test_top_k_tie_break():
    keys = np.array([0.5, 0.9, 0.9, 0.1, 0.9])
    assert osel.top_k(keys, 3).tolist() == [1, 2, 4]


@pytest.fixture(scope="module")
def smallK():
    s = synth.make_system(6, 10, 0.05, True, 41, 42, 43)
    return s, ok.dense_kernel(s.R, 10.0)


def test_greedy_pivots_follow_schur_complement(smallK):
    """Each pivot is the largest diagonal entry of the current Schur complement,
    checked against the dense Schur complement formed explicitly."""
    s, K = smallK
    k = 30
    L, piv, keff, d = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), k)
    assert keff == k
    traces = []
    for m in range(k):
        Lm = L[:, :m]
        S = K - Lm @ Lm.T
        diag = np.diag(S).copy()
        diag[piv[:m]] = -np.inf
        assert piv[m] == int(np.argmax(diag))
        traces.append(np.trace(K - Lm @ Lm.T))
    assert np.all(np.diff(traces) < 0)                      # monotone improvement
    # interpolation: the factor reproduces the chosen columns exactly
    np.testing.assert_allclose((L @ L.T)[:, piv], K[:, piv], atol=1e-10 * np.abs(K).max())


def test_forced_order_drops_dependent_columns(smallK):
    s, K = smallK
    m3 = 3 * s.M
    order = np.arange(m3)              # all columns of geometry 0: rank 3M-6
    L, piv, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), m3, order=order,
                                               rel_tol=1e-10)
    assert keff == m3 - 6


def test_exact_leverage_sum_rule(smallK):
    s, K = smallK
    lam = 1e-6
    tau = osel.exact_ridge_leverage(K, lam)
    w = np.linalg.eigvalsh(K)
    assert tau.min() >= -1e-10 and tau.max() <= 1 + 1e-10
    np.testing.assert_allclose(tau.sum(), (w / (w + lam)).sum(), rtol=1e-9)


def test_leverage_estimate_bounds(smallK):
    s, K = smallK
    lam = 1e-4
    n = K.shape[0]
    tau = osel.exact_ridge_leverage(K, lam)
    # all columns as pilot: the estimate is the exact score
    allS = np.arange(n)
    raw = osel.raw_leverage_estimate(K, np.diag(K), allS, lam)
    np.testing.assert_allclose(raw, tau, atol=1e-6)
    # a pilot subset over-estimates (Nystroem residual is larger than the ridge one)
    S0 = osel.select_uniform(n, 40, 3, osel.STREAM_PILOT)
    raw = osel.raw_leverage_estimate(K[:, S0], np.diag(K), S0, lam)
    assert np.all(raw >= tau - 1e-6)
    est = osel.leverage_estimate(K[:, S0], np.diag(K), S0, lam)
    assert est.min() >= osel.WEIGHT_FLOOR and est.max() <= 1.0
    assert np.all(est[S0] == 1.0)

"""FP64 oracle: inducing-column selection (section 3, "Column selection strategies").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Random numbers.  Both this oracle and the HIP library draw their random numbers
from one counter-based generator, SplitMix64 (Steele, Lea & Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), so that sampled
index sets agree exactly.  Draw number i of stream s under seed S is
mix(S + (s * 2^40 + i + 1) * 0x9E3779B97F4A7C15) and is turned into a double
in (0, 1] as ((z >> 11) + 1) * 2^-53.  Streams: 0 uniform selection,
1 leverage pilot, 2 leverage sampling, 3 score sampling.

Readings where the paper leaves the details open:
  * uniform sampling (section 3) draws k distinct columns: the k largest draws
    u_i, ordered by decreasing u, ties to the lower index;
  * sampling proportional to weights w without replacement uses
    Efraimidis-Spirakis keys log(u_i)/w_i, again the k largest;
  * ridge leverage scores tau_i = (K (K + lambda I)^-1)_ii (section 3) are
    approximated from a uniform pilot set S0 of size s by
    tau_i ~ (K_ii - K_iS0 (K_S0S0 + lambda I)^-1 K_S0i) / lambda, clipped to
    [1e-12, 1]; pilot columns themselves get 1;
  * incomplete Cholesky (Algorithm 1 of the appendix) picks the largest
    remaining diagonal entry, ties to the lower column index, and stops once
    that entry is <= rel_tol * max(diag K).  Run with a given column order, it
    becomes the Nystroem factor of that column set (section 3: both are
    equivalent for identical columns); a column whose remaining diagonal is
    <= rel_tol * max(diag K) is then skipped (left as a zero column).

Pins (tests/test_oracle_select.py): SplitMix64 published outputs, sampler
frequencies, Nystroem == incomplete Cholesky, monotone Schur-complement trace,
exact leverage sum rule and the estimate's upper-bound property, per-column
score weights on a hand-computed case.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
STREAM_UNIFORM, STREAM_PILOT, STREAM_LEVERAGE, STREAM_SCORES = 0, 1, 2, 3
WEIGHT_FLOOR = 1e-12


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Counter-based SplitMix64: output for state seed + (counter + 1) * gamma."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(counters, dtype=np.uint64) + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    ctr = np.uint64(stream) * np.uint64(1 << 40) + np.arange(n, dtype=np.uint64)
    z = splitmix64(seed, ctr)
    return ((z >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53


def top_k(keys: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k largest keys, by decreasing key, ties to the lower index."""
    order = np.lexsort((np.arange(len(keys)), -keys))
    return order[:k].astype(np.int64)


def select_uniform(n: int, k: int, seed: int, stream: int = STREAM_UNIFORM) -> np.ndarray:
    return top_k(uniform01(seed, stream, n), k)


def weighted_keys(weights: np.ndarray, seed: int, stream: int) -> np.ndarray:
    u = uniform01(seed, stream, len(weights))
    return np.log(u) / weights


def select_weighted(weights: np.ndarray, k: int, seed: int, stream: int) -> np.ndarray:
    return top_k(weighted_keys(weights, seed, stream), k)


def incomplete_cholesky(get_col, diag: np.ndarray, k: int, order=None,
                        rel_tol: float = 1e-12):
    """Algorithm 1 (appendix "Incomplete Cholesky decomposition").

    get_col(i) returns column i of the (implicit) PSD matrix, diag its diagonal.
    Returns (L (n x k), pivots (list, in selection order), k_eff, residual diag).
    With `order` given, the pivots are taken in that order (skipping columns
    whose residual diagonal is too small); otherwise greedily.
    """
    n = diag.shape[0]
    d = diag.astype(np.float64).copy()
    L = np.zeros((n, k))
    selected = np.zeros(n, dtype=bool)
    thr = rel_tol * diag.max()
    pivots = []
    for m in range(k):
        if order is None:
            cand = np.where(selected, -np.inf, d)
            i = int(np.argmax(cand))          # first maximum = lowest index on ties
            if cand[i] <= thr:
                break
        else:
            i = int(order[m])
            if selected[i] or d[i] <= thr:
                continue
        pivot = np.sqrt(d[i])
        schur = L[:, :m] @ L[i, :m]           # Schur correction from earlier columns
        col = (get_col(i) - schur) / pivot
        col[selected] = 0.0
        col[i] = pivot
        L[:, m] = col
        selected[i] = True
        pivots.append(i)
        d -= col * col
        d[selected] = 0.0
    return L, pivots, len(pivots), d


def exact_ridge_leverage(K: np.ndarray, lam: float) -> np.ndarray:
    """tau_i = (K (K + lam I)^-1)_ii from a dense solve."""
    n = K.shape[0]
    c = sla.cho_factor(K + lam * np.eye(n), lower=True)
    return np.einsum("ij,ji->i", K, sla.cho_solve(c, np.eye(n)))


def leverage_estimate(C: np.ndarray, diag: np.ndarray, S0: np.ndarray, lam: float) -> np.ndarray:
    """Pilot estimate (K_ii - c_i^T (K_S0S0 + lam I)^-1 c_i) / lam, clipped.

    C = K[:, S0] (n x s), diag = diag(K).
    """
    KSS = C[S0, :]
    c = sla.cho_factor(KSS + lam * np.eye(len(S0)), lower=True)
    quad = np.einsum("is,is->i", C, sla.cho_solve(c, C.T).T)
    tau = (diag - quad) / lam
    tau[np.asarray(S0)] = 1.0
    return np.clip(tau, WEIGHT_FLOOR, 1.0)


def raw_leverage_estimate(C: np.ndarray, diag: np.ndarray, S0: np.ndarray, lam: float) -> np.ndarray:
    """The unclipped estimate for every column (pilot columns included)."""
    KSS = C[S0, :]
    c = sla.cho_factor(KSS + lam * np.eye(len(S0)), lower=True)
    quad = np.einsum("is,is->i", C, sla.cho_solve(c, C.T).T)
    return (diag - quad) / lam


def score_weights(geom_scores: np.ndarray, M: int) -> np.ndarray:
    """Per-column sampling weight from per-geometry scores (all 3M columns share it).

    Efraimidis-Spirakis keys are invariant to a common scale, so the weight is
    the geometry's score itself, floored at WEIGHT_FLOOR.
    """
    w = np.repeat(np.asarray(geom_scores, dtype=np.float64), 3 * M)
    return np.maximum(w, WEIGHT_FLOOR)

"""FP64 oracle: the kernel symmetrized over a group of atom permutations.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's kernels come from sGDML (section 2.1), whose kernel sums the
scalar kernel over a group S of atom permutations of the molecule:
    k_S(R, R') = sum_{q in S} k(x(R), x(P_q R')),   (P_q R)_a = R_{p_q(a)}.
The force kernel is again the mixed second derivative in raw coordinates;
by the chain rule through P_q its (i, j) block is
    K_S,ij = sum_q J(R_i)^T H(x(R_i), x(P_q R_j)) J(P_q R_j) Pi_q,
with Pi_q the 3M x 3M coordinate permutation, (Pi_q v)_(a,t) = v_(p_q(a),t).
No normalisation by |S|.  The permutations are given; finding them (sGDML
matches the molecular graph) is not part of this.

Pins (tests/test_oracle_symmetry.py): the trivial group gives the plain
kernel; a block equals the mixed finite differences of k_S in raw
coordinates; K_S is symmetric, PSD and satisfies K_S(R_i, P_g R_j) =
K_S(R_i, R_j) Pi_g^T for every g in S; the matrix-free product equals the
dense matrix; group validation rejects non-groups.
"""
from __future__ import annotations

import numpy as np

from . import kernel as ok


def check_group(perms) -> np.ndarray:
    """perms (S, M) of atom permutations; raises unless they form a group."""
    P = np.asarray(perms, dtype=np.int64)
    S, M = P.shape
    for p in P:
        if sorted(p.tolist()) != list(range(M)):
            raise ValueError("not a permutation")
    rows = {tuple(p) for p in P}
    if len(rows) != S:
        raise ValueError("repeated permutation")
    if tuple(range(M)) not in rows:
        raise ValueError("the identity is missing")
    for p in P:
        for q in P:
            if tuple(p[q]) not in rows:   # the composite a -> p(q(a))
                raise ValueError("not closed under composition")
    return P


def permute_geometries(R: np.ndarray, p) -> np.ndarray:
    """P R for one permutation: (..., M, 3) with atom a taken from atom p(a)."""
    return R[..., np.asarray(p), :]


def coordinate_permutation(p) -> np.ndarray:
    """Pi (3M x 3M) with (Pi v)_(a,t) = v_(p(a),t)."""
    p = np.asarray(p)
    M = len(p)
    Pi = np.zeros((3 * M, 3 * M))
    for a in range(M):
        for t in range(3):
            Pi[3 * a + t, 3 * p[a] + t] = 1.0
    return Pi


def sym_force_kernel_block(Ri, Rj, perms, sigma) -> np.ndarray:
    """K_S,ij = sum_q J(R_i)^T H(x(R_i), x(P_q R_j)) J(P_q R_j) Pi_q."""
    out = np.zeros((Ri.size, Rj.size))
    for p in perms:
        out += ok.force_kernel_block(Ri, permute_geometries(Rj, p), sigma) @ coordinate_permutation(p)
    return out


def dense_sym_kernel(R: np.ndarray, perms, sigma: float) -> np.ndarray:
    """Assemble K_S (n x n) block by block."""
    N, M, _ = R.shape
    m3 = 3 * M
    K = np.empty((N * m3, N * m3))
    for i in range(N):
        for j in range(N):
            K[i * m3:(i + 1) * m3, j * m3:(j + 1) * m3] = sym_force_kernel_block(R[i], R[j], perms, sigma)
    return K


def sym_kernel_mvm(R: np.ndarray, perms, v: np.ndarray, sigma: float, R_tgt=None) -> np.ndarray:
    """Matrix-free K_S(R_tgt, R) v = sum_q K(R_tgt, P_q R) (Pi_q v), with the
    plain product (R_tgt defaults to R: the training product; other targets
    give the prediction of a symmetrized model)."""
    N, M, _ = R.shape
    T = R if R_tgt is None else R_tgt
    V = v.reshape(N, M, 3)
    y = np.zeros(T.shape[0] * 3 * M)
    for p in perms:
        y += ok.kernel_mvm(T, permute_geometries(R, p), V[:, np.asarray(p), :].reshape(-1), sigma)
    return y

"""FP64 oracle: closed-form solve, textbook PCG and the Nystroem/Woodbury preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  cholesky_solve  -- the closed-form solution of K_lambda alpha = y (Eq. 1),
                     via a dense Cholesky factorisation (scipy).
  pcg             -- conjugate gradients on the preconditioned system (Eq. 2),
                     the standard Hestenes-Stiefel recurrence as in Saad,
                     "Iterative Methods for Sparse Linear Systems", Alg. 9.1.
  woodbury        -- P^{-1} for P = L L^T + lambda I (Eq. 3) by the Woodbury
                     identity (Eq. 4), with the k x k core factored by Cholesky.
  nystrom_lowrank -- K_nk K_kk^{-1} K_nk^T (Eq. 5) formed directly.

Pins (tests/test_oracle_solve.py): Woodbury against a dense inverse, PCG
against the Cholesky solve at moderate condition number, the one-step
convergence of a preconditioner that reproduces K exactly (appendix A.1).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def cholesky_solve(K: np.ndarray, lam: float, y: np.ndarray) -> np.ndarray:
    n = K.shape[0]
    c = sla.cho_factor(K + lam * np.eye(n), lower=True)
    return sla.cho_solve(c, y)


def pcg(apply_A, b: np.ndarray, apply_Minv=None, tol: float = 1e-6,
        maxiter: int | None = None, x0: np.ndarray | None = None):
    """Preconditioned CG.  Stops when |r_k| <= tol |b| (recursive residual).

    Returns (x, iterations, residual history |r_k|/|b|).
    """
    n = b.shape[0]
    maxiter = n if maxiter is None else maxiter
    x = np.zeros(n) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = apply_Minv(r) if apply_Minv is not None else r.copy()
    p = z.copy()
    rz = r @ z
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    it = 0
    while hist[-1] > tol and it < maxiter:
        q = apply_A(p)
        gamma = rz / (p @ q)
        x += gamma * p
        r -= gamma * q
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            break
        z = apply_Minv(r) if apply_Minv is not None else r.copy()
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, np.array(hist)


def woodbury(L: np.ndarray, lam: float):
    """Return r -> P^{-1} r for P = L L^T + lam I using Eq. 4."""
    k = L.shape[1]
    core = sla.cho_factor(lam * np.eye(k) + L.T @ L, lower=True)

    def apply(r: np.ndarray) -> np.ndarray:
        return (r - L @ sla.cho_solve(core, L.T @ r)) / lam

    return apply


def nystrom_lowrank(K: np.ndarray, S) -> np.ndarray:
    """K_nk K_kk^{-1} K_nk^T for the column subset S (Eq. 5)."""
    C = K[:, S]
    return C @ np.linalg.solve(K[np.ix_(S, S)], C.T)

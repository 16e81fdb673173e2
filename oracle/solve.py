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
  stored_factor   -- L as kept in a reduced storage format (FP32, or BF16 =
                     the upper 16 bits of an IEEE binary32 with round to
                     nearest even), so the Woodbury apply of the stored
                     operator can be formed here too.

Pins (tests/test_oracle_solve.py): Woodbury against a dense inverse, PCG
against the Cholesky solve at moderate condition number, the one-step
convergence of a preconditioner that reproduces K exactly (appendix A.1),
the rounding of stored_factor on hand-picked ties and its error bound.
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


def stored_factor(L: np.ndarray, fmt: str) -> np.ndarray:
    """L rounded to the storage format and returned as float64.

    fp64: unchanged.  fp32: round to nearest binary32.  bf16: round to nearest
    binary32 first, then keep the upper 16 bits of the binary32 pattern,
    rounding the dropped 16 bits to nearest with ties to an even result."""
    if fmt == "fp64":
        return L.copy()
    f = np.ascontiguousarray(L, dtype=np.float32)
    if fmt == "fp32":
        return f.astype(np.float64)
    assert fmt == "bf16"
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)

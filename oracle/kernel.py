"""FP64 oracle: descriptor, Jacobian and the Matern-5/2 force-field kernel.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (section 2.1, "Kernel machines for MLFF") encodes each geometry by a
descriptor and builds a PSD kernel matrix of size n = 3 d n_train made of
(3d x 3d) blocks, one per pair of training geometries; it does not spell the
kernel out.  The workload fixes it:
  * descriptor x = all inverse interatomic distances 1/|R_p - R_q| for p > q,
    ordered like numpy.tril_indices(M, -1)  (D = M(M-1)/2 entries);
  * scalar kernel k(x, x') = Matern-5/2 of r = |x - x'| with length scale sigma
    (Rasmussen & Williams, GPML eq. 4.17): (1 + z + z^2/3) exp(-z), z = sqrt(5) r / sigma;
  * force kernel block K_ij = J_i^T H(x_i, x_j) J_j with J the Jacobian of the
    descriptor and H = d^2 k / dx dx'^T = a(r) I + b(r) d d^T, d = x - x'.
No permutational symmetrisation (plain GDML form), no normalisation.

Pins (tests/test_oracle_kernel.py):
  descriptor_jacobian  -- central finite differences of the descriptor
  matern52             -- scipy's modified Bessel function form of the Matern family
  hessian_coeffs       -- mixed central finite differences of the scalar kernel
  force_kernel_block   -- mixed finite differences of k(x(R), x(R')) in raw coordinates
  dense_kernel         -- symmetry, PSD, null space of dimension exactly 6N
  kernel_mvm           -- equals dense_kernel @ v
"""
from __future__ import annotations

import numpy as np


def pair_indices(M: int):
    """(p, q) index arrays of all atom pairs with p > q, row-major."""
    return np.tril_indices(M, -1)


def descriptor(R: np.ndarray) -> np.ndarray:
    """Inverse distances, R (..., M, 3) -> x (..., D)."""
    p, q = pair_indices(R.shape[-2])
    diff = R[..., p, :] - R[..., q, :]
    return 1.0 / np.sqrt((diff * diff).sum(-1))


def descriptor_jacobian(R: np.ndarray) -> np.ndarray:
    """dx/dR for one geometry R (M, 3) as a dense (D, 3M) matrix.

    d(1/r_pq)/dR_p = -(R_p - R_q)/r^3 and d(1/r_pq)/dR_q = +(R_p - R_q)/r^3.
    """
    M = R.shape[0]
    p, q = pair_indices(M)
    diff = R[p] - R[q]
    r = np.sqrt((diff * diff).sum(-1))
    g = diff / r[:, None] ** 3
    D = len(p)
    J = np.zeros((D, M, 3))
    rows = np.arange(D)
    J[rows, p, :] = -g
    J[rows, q, :] = g
    return J.reshape(D, 3 * M)


def matern52(r: np.ndarray, sigma: float) -> np.ndarray:
    z = np.sqrt(5.0) * np.asarray(r, dtype=np.float64) / sigma
    return (1.0 + z + z * z / 3.0) * np.exp(-z)


def hessian_coeffs(r: np.ndarray, sigma: float):
    """(a, b) with d^2 k(x,x')/dx dx'^T = a I + b d d^T for the Matern-5/2 kernel.

    With f(r) the scalar kernel: a = -f'(r)/r and b = -(f''(r) - f'(r)/r)/r^2,
    which for Matern-5/2 gives a = 5/(3 sigma^2) (1+z) e^-z and
    b = -25/(3 sigma^4) e^-z.
    """
    z = np.sqrt(5.0) * np.asarray(r, dtype=np.float64) / sigma
    e = np.exp(-z)
    a = 5.0 / (3.0 * sigma ** 2) * (1.0 + z) * e
    b = -25.0 / (3.0 * sigma ** 4) * e
    return a, b


def hessian_block(x: np.ndarray, xp: np.ndarray, sigma: float) -> np.ndarray:
    d = x - xp
    a, b = hessian_coeffs(np.linalg.norm(d), sigma)
    return a * np.eye(len(d)) + b * np.outer(d, d)


def force_kernel_block(Ri: np.ndarray, Rj: np.ndarray, sigma: float) -> np.ndarray:
    """K_ij = J_i^T H(x_i, x_j) J_j, a (3M, 3M) block."""
    Ji, Jj = descriptor_jacobian(Ri), descriptor_jacobian(Rj)
    H = hessian_block(descriptor(Ri), descriptor(Rj), sigma)
    return Ji.T @ H @ Jj


def jacobians(R: np.ndarray) -> np.ndarray:
    """Stacked dense Jacobians (N, D, 3M)."""
    return np.stack([descriptor_jacobian(Ri) for Ri in R])


def dense_kernel(R: np.ndarray, sigma: float) -> np.ndarray:
    """Assemble the full n x n kernel matrix block by block (n = 3 M N)."""
    N, M, _ = R.shape
    X = descriptor(R)
    J = jacobians(R)
    D = X.shape[1]
    m3 = 3 * M
    K = np.empty((N * m3, N * m3))
    eye = np.eye(D)
    for i in range(N):
        d = X[i][None, :] - X                                  # (N, D)
        a, b = hessian_coeffs(np.linalg.norm(d, axis=1), sigma)
        H = a[:, None, None] * eye + b[:, None, None] * d[:, :, None] * d[:, None, :]
        blocks = np.einsum("da,jde,jeb->jab", J[i], H, J, optimize=True)
        K[i * m3:(i + 1) * m3, :] = blocks.transpose(1, 0, 2).reshape(m3, N * m3)
    return K


def kernel_diag(R: np.ndarray, sigma: float) -> np.ndarray:
    """diag(K): H(x, x) = a(0) I, so K_cc = a(0) |J e_c|^2."""
    a0, _ = hessian_coeffs(0.0, sigma)
    J = jacobians(R)                                           # (N, D, 3M)
    return (a0 * (J * J).sum(1)).reshape(-1)


def _apply_jacobian(R: np.ndarray, V: np.ndarray) -> np.ndarray:
    """u_i = J_i v_i for every geometry, written per pair: (N, D)."""
    p, q = pair_indices(R.shape[1])
    diff = R[:, p, :] - R[:, q, :]
    r = np.sqrt((diff * diff).sum(-1))
    g = diff / r[..., None] ** 3
    return -(g * (V[:, p, :] - V[:, q, :])).sum(-1)


def _apply_jacobian_t(R: np.ndarray, G: np.ndarray) -> np.ndarray:
    """J_i^T g_i for every geometry, written per pair: (N, M, 3)."""
    N, M, _ = R.shape
    p, q = pair_indices(M)
    diff = R[:, p, :] - R[:, q, :]
    r = np.sqrt((diff * diff).sum(-1))
    contrib = (G / r ** 3)[..., None] * diff                    # (N, D, 3)
    out = np.zeros((N, M, 3))
    for ax in range(3):
        np.add.at(out[:, :, ax].T, p, -contrib[:, :, ax].T)
        np.add.at(out[:, :, ax].T, q, contrib[:, :, ax].T)
    return out


def kernel_mvm(R_tgt: np.ndarray, R_src: np.ndarray, v: np.ndarray, sigma: float,
               targets=None, chunk: int = 16) -> np.ndarray:
    """Matrix-free y = K(tgt, src) v, one target geometry block at a time.

    y_i = sum_j J_i^T (a_ij u_j + b_ij d_ij (d_ij . u_j)),  u_j = J_j v_j,
    d_ij = x_i - x_j.  `targets` restricts the output to some target
    geometries (returned as (len(targets), 3M)); otherwise the full flat vector.
    """
    Ns, M, _ = R_src.shape
    Xs = descriptor(R_src)
    U = _apply_jacobian(R_src, v.reshape(Ns, M, 3))
    idx = np.arange(R_tgt.shape[0]) if targets is None else np.asarray(targets)
    Xt = descriptor(R_tgt[idx])
    G = np.empty((len(idx), Xs.shape[1]))
    for s in range(0, len(idx), chunk):
        d = Xt[s:s + chunk, None, :] - Xs[None, :, :]           # (c, Ns, D)
        a, b = hessian_coeffs(np.sqrt((d * d).sum(-1)), sigma)
        du = np.einsum("cjd,jd->cj", d, U)
        G[s:s + chunk] = np.einsum("cj,jd->cd", a, U) + np.einsum("cj,cjd->cd", b * du, d)
    y = _apply_jacobian_t(R_tgt[idx], G)
    return y.reshape(-1) if targets is None else y.reshape(len(idx), -1)


def kernel_columns(R: np.ndarray, cols: np.ndarray, sigma: float) -> np.ndarray:
    """K[:, cols] by block evaluation of the source geometries (n x k)."""
    N, M, _ = R.shape
    m3 = 3 * M
    X = descriptor(R)
    J = jacobians(R)
    cols = np.asarray(cols)
    out = np.empty((N * m3, len(cols)))
    for c, col in enumerate(cols):
        g, loc = divmod(int(col), m3)
        u = J[g][:, loc]                                        # J_g e_c  (D,)
        d = X - X[g][None, :]
        a, b = hessian_coeffs(np.linalg.norm(d, axis=1), sigma)
        h = a[:, None] * u[None, :] + (b * (d @ u))[:, None] * d     # (N, D)
        out[:, c] = np.einsum("nda,nd->na", J, h).reshape(-1)
    return out

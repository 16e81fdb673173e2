"""Host helpers of the spectrum study (section 4.1) against brute force:
the eigenvalues of P^-1 K_lambda formed explicitly and diagonalised."""
import numpy as np


def _psd(n, rank, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, rank)) * np.logspace(0, -4, rank)
    return A @ A.T


def test_svd_preconditioned_spectrum_closed_form():
    from paper_2212_12737_amd.study import svd_preconditioned_spectrum
    n, lam = 40, 1e-3
    K = _psd(n, 30, 1)
    e, U = np.linalg.eigh(K)
    e, U = e[::-1], U[:, ::-1]
    for k in (0, 1, 7, 30, 40):
        P = (U[:, :k] * e[:k]) @ U[:, :k].T + lam * np.eye(n)
        brute = np.sort(np.linalg.eigvals(np.linalg.solve(P, K + lam * np.eye(n))).real)[::-1]
        got = svd_preconditioned_spectrum(e, lam, k)
        np.testing.assert_allclose(got, brute, rtol=1e-8)


def test_nystrom_preconditioned_spectrum_pencil():
    from paper_2212_12737_amd.study import nystrom_preconditioned_spectrum
    n, lam = 40, 1e-3
    K = _psd(n, 30, 2)
    cols = [3, 11, 17, 25, 31]
    C = K[:, cols]
    L = C @ np.linalg.cholesky(np.linalg.inv(K[np.ix_(cols, cols)]))   # L L^T = C K_SS^-1 C^T (Eq. 5)
    P = L @ L.T + lam * np.eye(n)
    brute = np.sort(np.linalg.eigvals(np.linalg.solve(P, K + lam * np.eye(n))).real)[::-1]
    got = nystrom_preconditioned_spectrum(K, L, lam)
    np.testing.assert_allclose(got, brute, rtol=1e-7)
    # a Nystroem approximation never exceeds K, so P^-1 K_lambda >= 1
    assert got[-1] >= 1 - 1e-9

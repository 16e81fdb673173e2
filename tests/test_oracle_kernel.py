"""Pins of the oracle's descriptor, Jacobian and force kernel against the mathematics."""
import numpy as np
import pytest
from scipy.special import gamma as gamma_fn
from scipy.special import kv
from scipy.spatial.transform import Rotation

import synth
from oracle import kernel as ok


def small_system(M=6, N=8, seed=7, sd=0.05):
    return synth.make_system(M, N, sd, True, seed, seed + 1, seed + 2)


def test_descriptor_rigid_invariance():
    s = small_system()
    Rot = Rotation.from_rotvec([0.3, -1.1, 0.7]).as_matrix()
    R2 = s.R @ Rot.T + np.array([1.5, -2.0, 0.25])
    np.testing.assert_allclose(ok.descriptor(R2), ok.descriptor(s.R), rtol=1e-13)


def test_descriptor_pair_order_is_tril():
    R = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 2.0, 0], [0, 0, 4.0]])
    x = ok.descriptor(R)
    # pairs (1,0), (2,0), (2,1), (3,0), (3,1), (3,2)
    expect = 1.0 / np.array([1.0, 2.0, np.sqrt(5.0), 4.0, np.sqrt(17.0), np.sqrt(20.0)])
    np.testing.assert_allclose(x, expect, rtol=1e-15)


def test_jacobian_central_differences():
    R = small_system().R[0]
    J = ok.descriptor_jacobian(R)
    h = 1e-6
    Jfd = np.empty_like(J)
    flat = R.reshape(-1)
    for c in range(flat.size):
        e = np.zeros_like(flat)
        e[c] = h
        Jfd[:, c] = (ok.descriptor((flat + e).reshape(R.shape)) -
                     ok.descriptor((flat - e).reshape(R.shape))) / (2 * h)
    assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(J).max()


@pytest.mark.parametrize("sigma", [1.0, 10.0])
def test_matern_against_bessel_form(sigma):
    # Matern family: 2^(1-nu)/Gamma(nu) (sqrt(2nu) r/s)^nu K_nu(sqrt(2nu) r/s), nu = 5/2
    nu = 2.5
    r = np.linspace(1e-3, 5 * sigma, 57)
    t = np.sqrt(2 * nu) * r / sigma
    ref = 2 ** (1 - nu) / gamma_fn(nu) * t ** nu * kv(nu, t)
    np.testing.assert_allclose(ok.matern52(r, sigma), ref, rtol=1e-12)
    assert ok.matern52(0.0, sigma) == 1.0


def _scalar_k(x, xp, sigma):
    return ok.matern52(np.linalg.norm(x - xp), sigma)


def test_hessian_mixed_finite_differences():
    rng = np.random.default_rng(3)
    D = 5
    x = rng.normal(size=D)
    xp = x + 0.7 * rng.normal(size=D)
    sigma = 2.0
    H = ok.hessian_block(x, xp, sigma)
    h = 1e-4
    Hfd = np.empty((D, D))
    for a in range(D):
        for b in range(D):
            ea = np.zeros(D); ea[a] = h
            eb = np.zeros(D); eb[b] = h
            Hfd[a, b] = (_scalar_k(x + ea, xp + eb, sigma) - _scalar_k(x + ea, xp - eb, sigma)
                         - _scalar_k(x - ea, xp + eb, sigma) + _scalar_k(x - ea, xp - eb, sigma)) / (4 * h * h)
    assert np.abs(H - Hfd).max() <= 1e-6 * np.abs(H).max()
    # r -> 0 limit: H = 5/(3 sigma^2) I
    np.testing.assert_allclose(ok.hessian_block(x, x, sigma), 5 / (3 * sigma ** 2) * np.eye(D), rtol=1e-15)


def test_force_block_is_mixed_second_derivative_in_coordinates():
    """K_ij = d^2 k(x(R_i), x(R_j)) / dR_i dR_j^T, by finite differences in raw coordinates."""
    s = small_system(M=4, N=2, sd=0.1)
    Ri, Rj = s.R[0], s.R[1]
    sigma = 1.5   # short length scale so the block is far from the r->0 limit
    Kij = ok.force_kernel_block(Ri, Rj, sigma)

    def k_of(Ra, Rb):
        return _scalar_k(ok.descriptor(Ra), ok.descriptor(Rb), sigma)

    h = 1e-4
    m3 = Ri.size
    Kfd = np.empty((m3, m3))
    fi, fj = Ri.reshape(-1), Rj.reshape(-1)
    for a in range(m3):
        ea = np.zeros(m3); ea[a] = h
        for b in range(m3):
            eb = np.zeros(m3); eb[b] = h
            sh = Ri.shape
            Kfd[a, b] = (k_of((fi + ea).reshape(sh), (fj + eb).reshape(sh))
                         - k_of((fi + ea).reshape(sh), (fj - eb).reshape(sh))
                         - k_of((fi - ea).reshape(sh), (fj + eb).reshape(sh))
                         + k_of((fi - ea).reshape(sh), (fj - eb).reshape(sh))) / (4 * h * h)
    assert np.abs(Kij - Kfd).max() <= 1e-5 * np.abs(Kij).max()


@pytest.fixture(scope="module")
def dense_small():
    s = small_system(M=6, N=10, seed=11)
    return s, ok.dense_kernel(s.R, 10.0)


def test_dense_symmetric_psd_and_null_space(dense_small):
    s, K = dense_small
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    w = np.linalg.eigvalsh(K)
    assert w.min() >= -1e-12 * w.max()
    null = int((w < 1e-11 * w.max()).sum())
    assert null == 6 * s.N          # rigid motions of every geometry (section 2.1)
    assert w[6 * s.N] > 1e3 * 1e-11 * w.max()   # clear gap above the null space


def test_rigid_motions_are_annihilated(dense_small):
    s, K = dense_small
    N, M, _ = s.R.shape
    for g in (0, N - 1):
        for mode in range(6):
            v = np.zeros((N, M, 3))
            if mode < 3:
                v[g, :, mode] = 1.0                           # translation
            else:
                axis = np.zeros(3); axis[mode - 3] = 1.0
                v[g] = np.cross(axis, s.R[g])                  # infinitesimal rotation
            assert np.linalg.norm(K @ v.reshape(-1)) <= 1e-12 * np.abs(K).max()


def test_matrix_free_mvm_matches_dense(dense_small):
    s, K = dense_small
    v = synth.random_vectors(K.shape[0], 5)
    np.testing.assert_allclose(ok.kernel_mvm(s.R, s.R, v, 10.0), K @ v, rtol=0, atol=1e-12 * np.abs(K @ v).max())
    tg = [3, 7]
    y = ok.kernel_mvm(s.R, s.R, v, 10.0, targets=tg)
    m3 = 3 * s.M
    for a, t in enumerate(tg):
        np.testing.assert_allclose(y[a], (K @ v)[t * m3:(t + 1) * m3], atol=1e-12 * np.abs(K @ v).max())


def test_columns_and_diag_match_dense(dense_small):
    s, K = dense_small
    cols = np.array([0, 5, 17, 18, K.shape[0] - 1])
    np.testing.assert_allclose(ok.kernel_columns(s.R, cols, 10.0), K[:, cols], atol=1e-14 * np.abs(K).max())
    np.testing.assert_allclose(ok.kernel_diag(s.R, 10.0), np.diag(K), rtol=1e-13)


def test_cross_mvm_uses_blocks():
    a = small_system(M=5, N=3, seed=21)
    b = small_system(M=5, N=4, seed=21)   # same molecule, other draws? different seed triple -> same R0
    v = synth.random_vectors(b.R.size, 9)
    y = ok.kernel_mvm(a.R, b.R, v, 10.0)
    m3 = 15
    ref = np.zeros(a.R.size)
    for i in range(a.N):
        for j in range(b.N):
            ref[i * m3:(i + 1) * m3] += ok.force_kernel_block(a.R[i], b.R[j], 10.0) @ v[j * m3:(j + 1) * m3]
    np.testing.assert_allclose(y, ref, atol=1e-13 * np.abs(ref).max())


def test_parallel_oracle_product_equals_the_serial_one():
    """The test helper that spreads the oracle's product over processes
    returns the oracle's own rows, in order (rectangular and square)."""
    import oracle_parallel
    tr = synth.make_system(6, 37, 0.05, True, 61, 62, 63)
    te = synth.make_system(6, 11, 0.05, True, 61, 64, 63)
    v = synth.random_vectors(tr.R.size, 5)
    np.testing.assert_allclose(oracle_parallel.kernel_mvm(tr.R, tr.R, v, 10.0, workers=3),
                               ok.kernel_mvm(tr.R, tr.R, v, 10.0), rtol=1e-13, atol=0)
    np.testing.assert_allclose(oracle_parallel.kernel_mvm(te.R, tr.R, v, 10.0, workers=4),
                               ok.kernel_mvm(te.R, tr.R, v, 10.0), rtol=1e-13, atol=0)

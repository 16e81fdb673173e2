"""Pins of the permutation-symmetrized kernel oracle (sGDML form, section 2.1)."""
import numpy as np
import pytest

import synth
from oracle import kernel as ok
from oracle import symmetry as osym


def small(M=5, N=4, seed=3, sd=0.1):
    return synth.make_system(M, N, sd, False, seed, seed + 1, seed + 2)


# a group of order 4 on 5 atoms: the identity, two swaps and their product
GROUP = [[0, 1, 2, 3, 4], [1, 0, 2, 3, 4], [0, 1, 2, 4, 3], [1, 0, 2, 4, 3]]


def test_trivial_group_is_the_plain_kernel():
    s = small()
    K = ok.dense_kernel(s.R, 10.0)
    Ks = osym.dense_sym_kernel(s.R, [list(range(5))], 10.0)
    np.testing.assert_allclose(Ks, K, rtol=0, atol=1e-13 * np.abs(K).max())   # same blocks, other summation order


def test_block_is_mixed_second_derivative_of_the_symmetrized_kernel():
    s = small(M=4, N=2, sd=0.1)
    Ri, Rj = s.R[0], s.R[1]
    sigma = 1.5
    perms = [[0, 1, 2, 3], [1, 0, 2, 3]]
    K = osym.sym_force_kernel_block(Ri, Rj, perms, sigma)

    def k_of(Ra, Rb):   # k_S(R, R') = sum_q Matern52(|x(R) - x(P_q R')|)
        xa = ok.descriptor(Ra)
        return sum(ok.matern52(np.linalg.norm(xa - ok.descriptor(Rb[p])), sigma) for p in perms)

    h, m3, sh = 1e-4, Ri.size, Ri.shape
    fi, fj = Ri.reshape(-1), Rj.reshape(-1)
    Kfd = np.empty((m3, m3))
    for a in range(m3):
        ea = np.zeros(m3); ea[a] = h
        for b in range(m3):
            eb = np.zeros(m3); eb[b] = h
            Kfd[a, b] = (k_of((fi + ea).reshape(sh), (fj + eb).reshape(sh))
                         - k_of((fi + ea).reshape(sh), (fj - eb).reshape(sh))
                         - k_of((fi - ea).reshape(sh), (fj + eb).reshape(sh))
                         + k_of((fi - ea).reshape(sh), (fj - eb).reshape(sh))) / (4 * h * h)
    assert np.abs(K - Kfd).max() <= 1e-5 * np.abs(K).max()


def test_symmetric_psd_and_group_covariant():
    s = small()
    Ks = osym.dense_sym_kernel(s.R, GROUP, 10.0)
    np.testing.assert_allclose(Ks, Ks.T, rtol=0, atol=1e-13 * np.abs(Ks).max())
    assert np.linalg.eigvalsh(Ks).min() >= -1e-12 * np.abs(Ks).max()
    for g in GROUP:
        left = osym.sym_force_kernel_block(s.R[0], osym.permute_geometries(s.R[1], g), GROUP, 10.0)
        right = osym.sym_force_kernel_block(s.R[0], s.R[1], GROUP, 10.0) @ osym.coordinate_permutation(g).T
        np.testing.assert_allclose(left, right, rtol=0, atol=1e-12 * np.abs(right).max())


def test_matrix_free_product_equals_dense():
    s = small()
    v = synth.random_vectors(s.R.shape[0] * 15, 4)
    Ks = osym.dense_sym_kernel(s.R, GROUP, 10.0)
    y = osym.sym_kernel_mvm(s.R, GROUP, v, 10.0)
    np.testing.assert_allclose(y, Ks @ v, rtol=0, atol=1e-12 * np.abs(Ks @ v).max())


@pytest.mark.parametrize("perms", [
    [[1, 0, 2]],                                  # no identity
    [[0, 1, 2], [1, 2, 0]],                       # not closed (needs its square)
    [[0, 1, 2], [0, 0, 2]],                       # not a permutation
    [[0, 1, 2], [1, 0, 2], [1, 0, 2]],            # repeated
])
def test_group_validation(perms):
    with pytest.raises(ValueError):
        osym.check_group(perms)
    assert osym.check_group([[0, 1, 2], [1, 2, 0], [2, 0, 1]]).shape == (3, 3)

"""GPU: the kernel symmetrized over a group of atom permutations (sGDML form,
section 2.1) against the FP64 oracle: product, columns and diagonal, a PCG
solve with a preconditioner built from the symmetrized columns, prediction,
argument checks, and the trivial group restoring the plain kernel."""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok
from oracle import solve as osv
from oracle import symmetry as osym

pytestmark = pytest.mark.gpu

SIGMA = 10.0
GROUP = [[0, 1, 2, 3, 4], [1, 0, 2, 3, 4], [0, 1, 2, 4, 3], [1, 0, 2, 4, 3]]   # order 4 on 5 atoms


@pytest.fixture(scope="module")
def ffk():
    from paper_2212_12737_amd import ffk as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(ffk):
    return ffk.create(0)


def system(N=12, seed=31):
    return synth.make_system(5, N, 0.1, False, seed, seed + 1, seed + 2)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def sym_case(ffk, ctx):
    s = system()
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    ffk.set_symmetries(ctx, S, GROUP)
    return s, S, osym.dense_sym_kernel(s.R, GROUP, SIGMA)


def test_product_columns_and_diagonal(ffk, ctx, sym_case):
    s, S, K = sym_case
    print("symmetrized kernel, n =", S.n, flush=True)
    v = synth.random_vectors(S.n, 3)
    y = ffk.kernel_mvm(ctx, S, dev(v), shift=0.5).cpu().numpy()
    assert relerr(y, K @ v + 0.5 * v) <= 1e-10
    cols = np.array([0, 1, 2, 5, 17, 44, 101, S.n - 1])   # atoms inside and outside the permuted pairs
    C = ffk.kernel_columns(ctx, S, dev(cols, torch.int64)).cpu().numpy()
    np.testing.assert_allclose(C, K[:, cols], rtol=0, atol=1e-10 * np.abs(K).max())   # n x k
    d = ffk.kernel_diag(ctx, S).cpu().numpy()
    np.testing.assert_allclose(d, np.diag(K), rtol=0, atol=1e-10 * np.abs(K).max())


def test_solve_and_prediction(ffk, ctx, sym_case):
    s, S, K = sym_case
    lam = 1e-4 * np.abs(K).max()
    F = s.flat_forces()
    idx = ffk.nystrom_select(ctx, S, "pivchol", 60)
    P = ffk.precond_build(ctx, S, idx, lam, store=ffk.FP64)
    alpha, rep = ffk.pcg_solve(ctx, S, P, dev(F), lam, tol=1e-10, max_iter=2000, prec=ffk.FP64)
    assert rep.status == 0
    a = alpha.cpu().numpy()
    ref = osv.cholesky_solve(K, lam, F)
    print("symmetrized solve: %d iterations, relative error of alpha %.2e" % (rep.iters, relerr(a, ref)), flush=True)
    assert relerr(a, ref) <= 1e-7
    te = system(N=5, seed=77)
    T = ffk.descriptor_build(ctx, dev(te.R), SIGMA)
    Fp = ffk.kernel_predict(ctx, S, T, alpha).cpu().numpy()
    assert relerr(Fp, osym.sym_kernel_mvm(s.R, GROUP, a, SIGMA, R_tgt=te.R)) <= 1e-10


def test_argument_checks_and_trivial_group(ffk, ctx):
    s = system(N=6, seed=55)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    for bad in ([[1, 0, 2, 3, 4]], [[0, 1, 2, 3, 4], [1, 2, 0, 3, 4]], [[0, 1, 2, 3, 4], [0, 0, 2, 3, 4]]):
        with pytest.raises(ffk.FfkError):
            ffk.set_symmetries(ctx, S, bad)
    ffk.set_symmetries(ctx, S, GROUP)
    v = dev(synth.random_vectors(S.n, 8))
    with pytest.raises(ffk.FfkError):
        ffk.kernel_mvm(ctx, S, v, prec=ffk.BF16X3)
    ffk.set_symmetries(ctx, S, [list(range(5))])   # back to the plain kernel
    y = ffk.kernel_mvm(ctx, S, v).cpu().numpy()
    assert relerr(y, ok.kernel_mvm(s.R, s.R, v.cpu().numpy(), SIGMA)) <= 1e-10
    ffk.kernel_mvm(ctx, S, v, prec=ffk.BF16X3)      # reduced precisions are available again

"""Pins of the oracle's solvers and preconditioner against the mathematics."""
import numpy as np
import pytest

import synth
from oracle import kernel as ok
from oracle import select as osel
from oracle import solve as osv


def test_woodbury_against_dense_inverse():
    rng = np.random.default_rng(0)
    n, k, lam = 60, 9, 1e-2
    L = rng.normal(size=(n, k))
    r = rng.normal(size=n)
    z = osv.woodbury(L, lam)(r)
    ref = np.linalg.solve(L @ L.T + lam * np.eye(n), r)
    np.testing.assert_allclose(z, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.fixture(scope="module")
def tiny():
    s = synth.make_system(5, 12, 0.05, True, 31, 32, 33)
    K = ok.dense_kernel(s.R, 10.0)
    return s, K


def test_pcg_matches_cholesky_at_moderate_condition(tiny):
    s, K = tiny
    w = np.linalg.eigvalsh(K)
    lam = w.max() / 1e3                  # kappa(K + lam I) <= ~1e3
    y = s.flat_forces()
    ref = osv.cholesky_solve(K, lam, y)
    A = K + lam * np.eye(K.shape[0])
    x, it, hist = osv.pcg(lambda v: A @ v, y, tol=1e-14, maxiter=2000)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    # and with a preconditioner
    L, piv, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), 20)
    x2, it2, _ = osv.pcg(lambda v: A @ v, y, osv.woodbury(L[:, :keff], lam), tol=1e-14, maxiter=2000)
    assert np.linalg.norm(x2 - ref) <= 1e-10 * np.linalg.norm(ref)
    assert it2 < it


def test_cholesky_residual(tiny):
    s, K = tiny
    lam = 1e-6
    y = s.flat_forces()
    a = osv.cholesky_solve(K, lam, y)
    assert np.linalg.norm(K @ a + lam * a - y) <= 1e-8 * np.linalg.norm(y)


def test_full_rank_preconditioner_converges_in_one_step(tiny):
    """Appendix A.1: a preconditioner that removes the whole spectrum leaves a flat
    spectrum and CG needs a single search direction."""
    s, K = tiny
    lam = 1e-6
    n = K.shape[0]
    L, piv, keff, d = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), n, rel_tol=1e-13)
    assert keff == n - 6 * s.N            # numerical rank: all but the rigid motions
    L = L[:, :keff]
    assert np.abs(L @ L.T - K).max() <= 1e-10 * np.abs(K).max()
    y = s.flat_forces()
    ref = osv.cholesky_solve(K, lam, y)
    x, it, _ = osv.pcg(lambda v: K @ v + lam * v, y, osv.woodbury(L, lam), tol=1e-8, maxiter=10)
    assert it <= 2
    assert np.linalg.norm(x - ref) <= 1e-6 * np.linalg.norm(ref)


def test_nystrom_equals_incomplete_cholesky_with_same_columns(tiny):
    """Section 3: Nystroem and incomplete Cholesky coincide for identical columns."""
    s, K = tiny
    S = osel.select_uniform(K.shape[0], 25, seed=5)
    L, piv, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), len(S), order=S)
    assert keff == len(S)
    ref = osv.nystrom_lowrank(K, S)
    assert np.abs(L @ L.T - ref).max() <= 1e-9 * np.abs(K).max()


@pytest.mark.slow
def test_m9_n200_uniform_pcg_reaches_cholesky_solution():
    """The small plain-FP64 workload: PCG with uniform Nystroem k=100 to 1e-6
    against the dense Cholesky solve (Table II compares the two solvers)."""
    cfg = synth.CONFIGS["m9_n200"]
    s = synth.config_system(cfg)
    K = ok.dense_kernel(s.R, cfg.sigma)
    y = s.flat_forces()
    ref = osv.cholesky_solve(K, cfg.lam, y)
    S = osel.select_uniform(K.shape[0], cfg.k, cfg.sel_seed)
    L, piv, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), cfg.k, order=S)
    A = lambda v: K @ v + cfg.lam * v
    x, it, _ = osv.pcg(A, y, osv.woodbury(L, cfg.lam), tol=1e-6)
    relres = np.linalg.norm(A(x) - y) / np.linalg.norm(y)
    assert relres <= 1.01e-6
    # fitted forces agree to the residual level; alpha to the conditioning bound
    assert np.linalg.norm(K @ x - K @ ref) <= 2e-6 * np.linalg.norm(y)
    _, it_plain, _ = osv.pcg(A, y, None, tol=1e-6, maxiter=3 * it)
    assert it < it_plain


def test_stored_factor_rounding():
    one = 1.0
    cases = {
        1.0: 1.0,                               # representable values stay
        -2.5: -2.5,
        one + 2.0 ** -8: 1.0,                   # tie between 1 and 1 + 2^-7: to the even 1
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,   # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,   # just above the tie
        -(one + 2.0 ** -8 + 2.0 ** -20): -(one + 2.0 ** -7),
    }
    x = np.array(list(cases))
    np.testing.assert_array_equal(osv.stored_factor(x, "bf16"), np.array(list(cases.values())))
    rng = np.random.default_rng(3)
    y = rng.standard_normal(10000) * 10.0 ** rng.uniform(-20, 20, 10000)
    for fmt, eps in (("bf16", 2.0 ** -8), ("fp32", 2.0 ** -24)):
        r = osv.stored_factor(y, fmt)
        assert np.all(np.abs(r - y) <= eps * np.abs(y) * (1 + 1e-12))
    np.testing.assert_array_equal(osv.stored_factor(y, "fp64"), y)

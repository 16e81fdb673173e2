"""GPU parity of the HIP path against the FP64 oracle, called through the C ABI.

Tolerances: 1e-10 relative (norm-wise) for the FP64 operators; reduced
precision MVMs as stated per test; solves judged on the oracle-computed true
residual (several alpha satisfy |r| <= tol |F|, see the conditioning bound).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok
from oracle import select as osel
from oracle import solve as osv

pytestmark = pytest.mark.gpu

SIGMA = 10.0


@pytest.fixture(scope="module")
def ffk():
    from paper_2212_12737_amd import ffk as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(ffk):
    return ffk.create(0)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def system(M, N, seed, sd=0.05, coulomb=True):
    return synth.make_system(M, N, sd, coulomb, seed, seed + 1, seed + 2)


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ------------------------------------------------------------------ descriptor
def test_descriptor_matches_oracle(ffk, ctx):
    s = system(7, 300, 10)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    assert (S.N, S.M, S.D, S.n) == (300, 7, 21, 6300)
    X = host(ffk.descriptor_export(ctx, S))
    np.testing.assert_allclose(X, ok.descriptor(s.R), rtol=1e-14)


def test_descriptor_rejects_coincident_atoms(ffk, ctx):
    s = system(5, 4, 11)
    R = s.R.copy()
    R[2, 3] = R[2, 1]
    with pytest.raises(ffk.FfkError):
        ffk.descriptor_build(ctx, dev(R), SIGMA)


# ------------------------------------------------------------ columns / diag
def test_diag_and_columns_match_oracle(ffk, ctx):
    s = system(6, 45, 12)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    d = host(ffk.kernel_diag(ctx, S))
    np.testing.assert_allclose(d, ok.kernel_diag(s.R, SIGMA), rtol=1e-13)
    cols = np.concatenate([[0, 1, 17, S.n - 1], np.random.default_rng(0).choice(S.n, 67, replace=False)])
    C = host(ffk.kernel_columns(ctx, S, dev(cols, torch.int64)))
    ref = ok.kernel_columns(s.R, cols, SIGMA)
    assert np.abs(C - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------------------ MVM
@pytest.mark.parametrize("M,N", [(7, 300), (21, 150), (9, 200), (4, 1), (3, 129), (12, 257)])
def test_mvm_fp64_matches_oracle(ffk, ctx, M, N):
    print("mvm fp64", M, N, flush=True)
    s = system(M, N, 100 + M + N)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = synth.random_vectors(S.n, 7)
    y = host(ffk.kernel_mvm(ctx, S, dev(v), shift=0.0, prec=ffk.FP64))
    ref = ok.kernel_mvm(s.R, s.R, v, SIGMA)
    assert relerr(y, ref) <= 1e-10
    lam = 0.37
    y2 = host(ffk.kernel_mvm(ctx, S, dev(v), shift=lam, prec=ffk.FP64))
    assert relerr(y2, ref + lam * v) <= 1e-10


def test_mvm_fp64_forces_label_vector(ffk, ctx):
    """The product with the label vector (F is orthogonal to the rigid-motion null space)."""
    s = synth.config_system(synth.CONFIGS["m9_n200"])
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    F = s.flat_forces()
    y = host(ffk.kernel_mvm(ctx, S, dev(F)))
    assert relerr(y, ok.kernel_mvm(s.R, s.R, F, SIGMA)) <= 1e-10


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x3", 1e-6), ("bf16", 3e-3)])
@pytest.mark.parametrize("M,N", [(7, 300), (21, 150), (4, 1), (3, 2), (3, 129), (5, 65)])
def test_mvm_reduced_precision(ffk, ctx, prec, tol, M, N):
    """Reduced-precision products against the FP64 oracle, down to the
    degenerate shapes: one geometry (one kernel block, d = 0 so only the
    a(0) term), three atoms (D = 3), and source counts one past a tile."""
    print("mvm", prec, M, N, flush=True)
    s = system(M, N, 200 + M + N, sd=0.08)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = synth.random_vectors(S.n, 8)
    y = host(ffk.kernel_mvm(ctx, S, dev(v), prec=ffk.PRECISIONS[prec]))
    ref = ok.kernel_mvm(s.R, s.R, v, SIGMA)
    err = relerr(y, ref)
    print("relerr", prec, err, flush=True)
    assert err <= tol


@pytest.mark.parametrize("M,N", [(25, 1100), (42, 600)])
def test_mvm_long_descriptor_rows(ffk, ctx, M, N):
    """Descriptor rows longer than one block's 256 lanes (D = 300, and the
    odd D = 861), where the J^T G reduction takes two columns per thread and
    the last pair runs past the row's end; several GEMM tiles with a ragged
    tail.  The whole output, every precision, against the FP64 oracle."""
    s = system(M, N, 500 + M + N, sd=0.08)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = synth.random_vectors(S.n, 9)
    ref = ok.kernel_mvm(s.R, s.R, v, SIGMA)
    for prec, tol in [("fp64", 1e-10), ("fp32", 1e-6), ("bf16x3", 1e-6), ("bf16", 3e-3)]:
        print("mvm", prec, M, N, flush=True)
        y = host(ffk.kernel_mvm(ctx, S, dev(v), prec=ffk.PRECISIONS[prec]))
        err = relerr(y, ref)
        print("relerr", prec, err, flush=True)
        assert err <= tol


@pytest.mark.parametrize("M,N", [(21, 2000), (25, 1100), (42, 600), (42, 5000)])
def test_mvm_repeats_bit_for_bit(ffk, ctx, M, N):
    """Every reduction of the two-GEMM product has a fixed order (no
    floating-point atomics), so repeated products agree bit for bit in every
    precision.  The shapes reach 16 and 8 K splits of GEMM 2 at small N, the
    two-column J^T G reduction (D = 300, 861), and the large tiles."""
    s = system(M, N, 700 + M + N, sd=0.08)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = dev(synth.random_vectors(S.n, 11))
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        print("repeat", prec, M, N, flush=True)
        y1 = host(ffk.kernel_mvm(ctx, S, v, prec=ffk.PRECISIONS[prec]))
        y2 = host(ffk.kernel_mvm(ctx, S, v, prec=ffk.PRECISIONS[prec]))
        assert np.array_equal(y1, y2), prec


def test_predict_matches_oracle(ffk, ctx):
    tr = synth.make_system(8, 170, 0.05, True, 31, 32, 33)
    te = synth.make_system(8, 37, 0.05, True, 31, 34, 33)
    Str = ffk.descriptor_build(ctx, dev(tr.R), SIGMA)
    Ste = ffk.descriptor_build(ctx, dev(te.R), SIGMA)
    alpha = synth.random_vectors(Str.n, 3)
    Fp = host(ffk.kernel_predict(ctx, Str, Ste, dev(alpha)))
    ref = ok.kernel_mvm(te.R, tr.R, alpha, SIGMA)
    assert relerr(Fp, ref) <= 1e-10


# ------------------------------------------------------------------ selection
@pytest.mark.parametrize("M,N,k", [(9, 200, 100), (7, 300, 700), (5, 3, 45)])
def test_uniform_selection_bit_exact(ffk, ctx, M, N, k):
    s = system(M, N, 300 + N)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    for seed in (0, 3003, 2 ** 63 + 5):
        idx = host(ffk.nystrom_select(ctx, S, "uniform", k, seed=seed))
        assert idx.tolist() == osel.select_uniform(S.n, k, seed).tolist()


def test_score_sampling_bit_exact(ffk, ctx):
    s = system(6, 400, 301)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    g = synth.random_weights(S.N, 17, 0.05, 3.0)
    k = 333
    idx = host(ffk.nystrom_select(ctx, S, "scores", k, seed=99, weights=dev(g)))
    ref = osel.select_weighted(osel.score_weights(g, S.M), k, 99, osel.STREAM_SCORES)
    if idx.tolist() != ref.tolist():
        # only a near-tie of two keys (one ulp of log) may reorder them
        keys = osel.weighted_keys(osel.score_weights(g, S.M), 99, osel.STREAM_SCORES)
        diff = set(idx.tolist()) ^ set(ref.tolist())
        thr = np.sort(keys)[::-1][k - 1]
        assert all(abs(keys[i] - thr) <= 1e-13 * abs(thr) for i in diff)


def test_pivoted_cholesky_sequence(ffk, ctx):
    s = system(6, 20, 302)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    K = ok.dense_kernel(s.R, SIGMA)
    k = 90
    gp = host(ffk.nystrom_select(ctx, S, "pivchol", k))
    L, piv, keff, d = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), k)
    assert len(gp) == keff
    # identical until the first near-tie (top-2 remaining diagonals within 1e-9)
    dd = np.diag(K).copy()
    Lm = np.zeros((K.shape[0], 0))
    for m in range(keff):
        if gp[m] != piv[m]:
            res = np.diag(K) - (Lm ** 2).sum(1)
            res[piv[:m]] = -np.inf
            top = np.sort(res)[::-1]
            assert top[0] - top[1] <= 1e-9 * top[0], (m, gp[m], piv[m])
            break
        Lm = L[:, :m + 1]


def test_pivoted_cholesky_stops_at_numerical_rank(ffk, ctx):
    s = system(5, 6, 303)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    gp = host(ffk.nystrom_select(ctx, S, "pivchol", S.n))
    assert len(gp) <= S.n - 6 * S.N
    assert len(set(gp.tolist())) == len(gp)


# ------------------------------------------------------------- preconditioner
def test_precond_factor_and_apply_match_oracle(ffk, ctx):
    s = system(6, 30, 304)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    K = ok.dense_kernel(s.R, SIGMA)
    idx = osel.select_uniform(S.n, 150, 7)            # > 2 panels, ragged
    P = ffk.precond_build(ctx, S, dev(idx, torch.int64), 1e-4, store=ffk.FP64)
    L = host(ffk.precond_export(ctx, P, S.n))
    Lo, piv, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), len(idx), order=idx)
    assert P.k_eff == keff
    Lo = Lo[:, [j for j in range(len(idx)) if np.any(Lo[:, j] != 0)]]
    assert np.abs(L @ L.T - Lo @ Lo.T).max() <= 1e-10 * np.abs(K).max()
    r = synth.random_vectors(S.n, 5)
    z = host(ffk.precond_apply(ctx, P, dev(r)))
    zo = osv.woodbury(Lo, 1e-4)(r)
    assert relerr(z, zo) <= 1e-9
    # FP32 storage: still an SPD operator; close to the FP64 one
    P32 = ffk.precond_build(ctx, S, dev(idx, torch.int64), 1e-4, store=ffk.FP32)
    z32 = host(ffk.precond_apply(ctx, P32, dev(r)))
    assert relerr(z32, zo) <= 1e-3
    assert float(r @ z32) > 0


@pytest.fixture(scope="module")
def apply_case():
    s = system(7, 300, 330)                            # n = 6300: several row blocks and ragged tails
    K = ok.dense_kernel(s.R, SIGMA)
    idx = osel.select_uniform(K.shape[0], 200, 9)       # 200 columns: ragged column tiles
    Lo, _, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), len(idx), order=idx)
    lam = 1e-3 * np.diag(K).max()
    r = synth.random_vectors(K.shape[0], 5)
    return s, idx, Lo[:, :keff], lam, r


@pytest.mark.parametrize("store", ["fp64", "fp32", "bf16"])
def test_precond_apply_storage_formats(ffk, ctx, apply_case, store):
    s, idx, Lo, lam, r = apply_case
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    P = ffk.precond_build(ctx, S, dev(idx, torch.int64), lam, store=ffk.PRECISIONS[store])
    assert P.k_eff == Lo.shape[1]
    z = host(ffk.precond_apply(ctx, P, dev(r)))
    Ls = host(ffk.precond_export(ctx, P, S.n))
    Lst = osv.stored_factor(Lo, store)
    if store == "fp64":
        np.testing.assert_allclose(Ls, Lst, rtol=0, atol=1e-10 * np.abs(Lst).max())
        assert relerr(z, osv.woodbury(Lst, lam)(r)) <= 1e-9
    else:
        # the stored factor is the oracle's factor rounded to the format; an
        # element whose FP64 value sits within rounding noise of a tie may land
        # one unit of the format away (rare)
        ulp = {"fp32": 2.0 ** -23, "bf16": 2.0 ** -7}[store]
        diff = np.abs(Ls - Lst)
        assert np.all(diff <= ulp * np.abs(Lst) + 1e-10 * np.abs(Lst).max())
        assert np.count_nonzero(diff > 1e-10 * np.abs(Lst).max()) <= 1e-4 * Lst.size
    # z inverts the operator built from the stored factor, to the accuracy of
    # the FP64 Woodbury apply at this condition number
    a, b = Ls @ (Ls.T @ z), lam * z
    scale = (np.linalg.norm(a) + np.linalg.norm(b)) / np.linalg.norm(r)
    assert relerr(a + b, r) <= 1e-9 * max(scale, 1.0)
    assert float(r @ z) > 0


def test_precond_low_memory_build(ffk, ctx, apply_case):
    """FP32-storage build (panels in FP64, earlier columns read in FP32).

    The first panel has no earlier columns, so it is the oracle's factor
    rounded to FP32.  Later columns carry the FP32 rounding of the earlier
    ones through the Schur-complement updates, amplified where the remaining
    pivots are small, so they are compared through L L^T; the apply must
    still invert the operator built from the stored factor exactly."""
    s, idx, Lo, lam, r = apply_case
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    P = ffk.precond_build(ctx, S, dev(idx, torch.int64), lam, store=ffk.FP32, lowmem=True)
    assert P.k_eff == Lo.shape[1]
    Ls = host(ffk.precond_export(ctx, P, S.n))
    d0 = np.abs(Ls[:, :64] - Lo[:, :64])
    assert np.all(d0 <= 2.0 ** -23 * np.abs(Lo[:, :64]) + 1e-10 * np.abs(Lo).max())
    LLo = Lo @ Lo.T
    dev_LL = np.abs(Ls @ Ls.T - LLo).max() / np.abs(LLo).max()
    z = host(ffk.precond_apply(ctx, P, dev(r)))
    dev_z = relerr(z, osv.woodbury(Lo, lam)(r))
    print("low-memory build: L L^T deviation %.2e, apply deviation %.2e" % (dev_LL, dev_z), flush=True)
    assert dev_LL <= 1e-5
    a, b = Ls @ (Ls.T @ z), lam * z
    scale = (np.linalg.norm(a) + np.linalg.norm(b)) / np.linalg.norm(r)
    assert relerr(a + b, r) <= 1e-9 * max(scale, 1.0)
    assert float(r @ z) > 0


def test_precond_matrix_free_equals_the_stored_factor(ffk, ctx, apply_case):
    """The matrix-free form (no n x k factor kept; L = K[:, S] L_SS^-T applied
    through two FP64 kernel products) is the same operator as the stored FP64
    factor: the same apply, the same exported L, and a solve that meets the
    oracle's bound."""
    s, idx, Lo, lam, r = apply_case
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    P = ffk.precond_build(ctx, S, dev(idx, torch.int64), lam, store=ffk.FP64)
    Pm = ffk.precond_build(ctx, S, dev(idx, torch.int64), lam, store=ffk.FP64, matrix_free=True)
    assert Pm.k_eff == P.k_eff == Lo.shape[1]
    assert Pm.bytes < P.bytes
    z = host(ffk.precond_apply(ctx, P, dev(r)))
    zm = host(ffk.precond_apply(ctx, Pm, dev(r)))
    print("matrix-free apply: |z_mf - z| / |z| = %.2e, %d vs %d bytes" % (relerr(zm, z), Pm.bytes, P.bytes),
          flush=True)
    assert relerr(zm, z) <= 1e-9
    assert relerr(zm, osv.woodbury(Lo, lam)(r)) <= 1e-9
    Lm = host(ffk.precond_export(ctx, Pm, S.n))
    assert np.abs(Lm @ Lm.T - Lo @ Lo.T).max() <= 1e-10 * np.abs(Lo @ Lo.T).max()
    K = ok.dense_kernel(s.R, SIGMA)
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, Pm, dev(F), lam, tol=1e-8, prec=ffk.FP64, max_iter=5000)
    _, rep_s = ffk.pcg_solve(ctx, S, P, dev(F), lam, tol=1e-8, prec=ffk.FP64, max_iter=5000)
    print("  PCG to 1e-8: matrix-free %d iterations, stored %d" % (rep.iters, rep_s.iters), flush=True)
    assert rep.status == 0 and abs(rep.iters - rep_s.iters) <= 1
    assert oracle_relres(K, lam, host(a), F) <= 1.01e-8
    with pytest.raises(ffk.FfkError):      # built from an FP64 factor only
        ffk.precond_build(ctx, S, dev(idx, torch.int64), lam, store=ffk.FP32, matrix_free=True)


def test_precond_drops_dependent_columns(ffk, ctx):
    s = system(5, 8, 305)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    m3 = 3 * S.M
    idx = np.concatenate([np.arange(m3), [3, m3 + 2]])     # a whole geometry (rank 3M-6) + a duplicate
    P = ffk.precond_build(ctx, S, dev(idx, torch.int64), 1e-6)
    assert P.dropped and P.k_eff == m3 - 6 + 1


def test_leverage_estimate_matches_oracle(ffk, ctx):
    s = system(6, 30, 306)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    lam, k, pilot, seed = 1e-5, 60, 80, 4
    idx, tau = ffk.nystrom_select(ctx, S, "leverage", k, lam=lam, seed=seed, pilot=pilot, return_tau=True)
    S0 = osel.select_uniform(S.n, pilot, seed, osel.STREAM_PILOT)
    C = ok.kernel_columns(s.R, S0, SIGMA)
    tau_o = osel.leverage_estimate(C, ok.kernel_diag(s.R, SIGMA), S0, lam)
    assert np.abs(host(tau) - tau_o).max() <= 1e-6
    ref = osel.select_weighted(tau_o, k, seed, osel.STREAM_LEVERAGE)
    assert len(set(host(idx).tolist()) & set(ref.tolist())) >= k - 2


def test_exact_rls_matches_oracle(ffk, ctx):
    s = system(6, 20, 307)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    lam = 1e-6
    tau = host(ffk.exact_rls(ctx, S, lam))
    K = ok.dense_kernel(s.R, SIGMA)
    ref = osel.exact_ridge_leverage(K, lam)
    assert np.abs(tau - ref).max() <= 1e-7


# ------------------------------------------------------------------------ PCG
def test_plain_cg_matches_cholesky(ffk, ctx):
    s = system(5, 12, 308)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    K = ok.dense_kernel(s.R, SIGMA)
    lam = np.linalg.eigvalsh(K).max() / 1e3
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, None, dev(F), lam, tol=1e-13, max_iter=2000)
    ref = osv.cholesky_solve(K, lam, F)
    assert rep.status == 0
    assert relerr(host(a), ref) <= 1e-10


@pytest.fixture(scope="module")
def small(ffk, ctx):
    cfg = synth.CONFIGS["m9_n200"]
    s = synth.config_system(cfg)
    S = ffk.descriptor_build(ctx, dev(s.R), cfg.sigma)
    K = ok.dense_kernel(s.R, cfg.sigma)
    idx = ffk.nystrom_select(ctx, S, "uniform", cfg.k, seed=cfg.sel_seed)
    return cfg, s, S, K, idx


def oracle_relres(K, lam, a, F):
    return np.linalg.norm(K @ a + lam * a - F) / np.linalg.norm(F)


def test_pcg_m9_n200_fp64_uniform(ffk, ctx, small):
    cfg, s, S, K, idx = small
    assert host(idx).tolist() == osel.select_uniform(S.n, cfg.k, cfg.sel_seed).tolist()
    P = ffk.precond_build(ctx, S, idx, cfg.lam)
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, tol=1e-6, prec=ffk.FP64)
    print("m9_n200 fp64 iters", rep.iters, rep.rel_res_true, flush=True)
    assert rep.status == 0
    assert oracle_relres(K, cfg.lam, host(a), F) <= 1.01e-6
    ref = osv.cholesky_solve(K, cfg.lam, F)
    print("m9_n200 fp64 forces %.3e alpha %.3e" % (np.linalg.norm(K @ host(a) - K @ ref) / np.linalg.norm(K @ ref),
                                                   np.linalg.norm(host(a) - ref) / np.linalg.norm(ref)), flush=True)
    assert np.linalg.norm(K @ host(a) - K @ ref) <= 2.1e-6 * np.linalg.norm(F)
    # same iteration count as the oracle's textbook PCG up to rounding effects
    L, _, _, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), cfg.k, order=host(idx))
    _, it_o, _ = osv.pcg(lambda v: K @ v + cfg.lam * v, F, osv.woodbury(L, cfg.lam), tol=1e-6)
    assert abs(rep.iters - it_o) <= 0.05 * it_o


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "bf16"])
def test_pcg_m9_n200_mixed_precision_reaches_fp64_residual(ffk, ctx, small, prec):
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, tol=1e-6, prec=ffk.PRECISIONS[prec], refresh_every=10,
                           escalate=True, max_iter=20000)
    assert rep.status == 0
    res = oracle_relres(K, cfg.lam, host(a), F)
    assert res <= 1.01e-6
    # against the oracle's Cholesky solution: the fitted forces to the same
    # bound as the FP64 solve, and alpha within what the residual allows,
    # |alpha - alpha*| <= |r| / lambda_min(K + lambda I) <= |r| / lambda
    ref = osv.cholesky_solve(K, cfg.lam, F)
    f_err = np.linalg.norm(K @ host(a) - K @ ref) / np.linalg.norm(K @ ref)
    a_err = np.linalg.norm(host(a) - ref) / np.linalg.norm(ref)
    print("m9_n200", prec, "iters", rep.iters, "esc", rep.n_escalations, "final", rep.final_prec,
          "residual %.3e forces %.3e alpha %.3e" % (res, f_err, a_err), flush=True)
    assert np.linalg.norm(K @ host(a) - K @ ref) <= 2.1e-6 * np.linalg.norm(F)
    # alpha: what separates it from alpha* is the stopping tolerance (FP64 PCG
    # to 1e-6 lands 1.7e-6 away); the bound |r| / lambda is far looser
    assert a_err <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_pcg_m9_n200_alpha_within_1e6_at_tighter_tolerance(ffk, ctx, small, prec):
    """Solved to a true residual of 1e-7, FP64 PCG and the refined split-BF16
    path both give alpha within 1e-6 (relative) of the oracle's Cholesky
    solution, and the fitted forces within 1e-6 too."""
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    mixed = prec == "bf16x3"
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, tol=1e-7, prec=ffk.PRECISIONS[prec], refresh_every=10,
                           escalate=True, switch_below=0.7 if mixed else 0.0, switch_from=ffk.FP32 if mixed else ffk.FP64,
                           max_iter=20000)
    assert rep.status == 0
    ref = osv.cholesky_solve(K, cfg.lam, F)
    f_err = np.linalg.norm(K @ host(a) - K @ ref) / np.linalg.norm(K @ ref)
    a_err = np.linalg.norm(host(a) - ref) / np.linalg.norm(ref)
    print("m9_n200 tol 1e-7", prec, "iters", rep.iters, "esc", rep.n_escalations,
          "residual %.3e forces %.3e alpha %.3e" % (oracle_relres(K, cfg.lam, host(a), F), f_err, a_err), flush=True)
    assert oracle_relres(K, cfg.lam, host(a), F) <= 1.01e-7
    assert f_err <= 1e-6 and a_err <= 1e-6


@pytest.mark.parametrize("first", ["fp64", "fp32"])
def test_pcg_m9_n200_switch_schedule(ffk, ctx, small, first):
    """First-phase products in FP64 or FP32 until the recursive residual is
    below 0.7 |F|, split BF16 after: the switch happens, and the oracle's
    residual of the result meets the bound."""
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, tol=1e-6, prec=ffk.BF16X3, refresh_every=20, escalate=True,
                           switch_below=0.7, switch_from=ffk.PRECISIONS[first], max_iter=20000)
    print("m9_n200 switch from", first, "at", rep.switch_iter, "iters", rep.iters, "esc", rep.n_escalations,
          rep.rel_res_true, flush=True)
    assert rep.status == 0
    assert 0 < rep.switch_iter < rep.iters
    assert rep.final_prec == ffk.BF16X3
    assert oracle_relres(K, cfg.lam, host(a), F) <= 1.01e-6


def test_pcg_escalation_in_the_first_phase_moves_it_to_fp64(ffk, ctx, small):
    """An escalation before the switch escalates the first phase's products:
    with a gap threshold so small that the first refresh (FP32 products)
    escalates, the solve leaves FP32 there for FP64, not for the reduced
    precision it would have switched to, and still meets the oracle's bound."""
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, tol=1e-6, prec=ffk.BF16X3, refresh_every=10, escalate=True,
                           switch_below=1e-12, switch_from=ffk.FP32, gap_escalate=1e-300, max_iter=20000)
    print("first-phase escalation: iters", rep.iters, "esc", rep.n_escalations, tuple(rep.esc_iter), "switch",
          rep.switch_iter, "final", rep.final_prec, flush=True)
    assert rep.status == 0
    assert rep.n_escalations == 1 and rep.esc_iter[0] == 10
    assert rep.switch_iter == 10
    assert rep.final_prec == ffk.FP64
    assert oracle_relres(K, cfg.lam, host(a), F) <= 1.01e-6


def test_pcg_escalation_after_the_switch_climbs_the_ladder(ffk, ctx, small):
    """After the switch the same threshold escalates split BF16 to FP32 at the
    first refresh and FP32 to FP64 at the next one."""
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, tol=1e-6, prec=ffk.BF16X3, refresh_every=10, escalate=True,
                           gap_escalate=1e-300, max_iter=20000)
    print("ladder: iters", rep.iters, "esc", rep.n_escalations, tuple(rep.esc_iter), "final", rep.final_prec,
          flush=True)
    assert rep.status == 0
    assert rep.n_escalations == 2 and tuple(rep.esc_iter)[:2] == (10, 20)
    assert rep.final_prec == ffk.FP64
    assert oracle_relres(K, cfg.lam, host(a), F) <= 1.01e-6


def test_pcg_restarts_after_a_gap_escalation(ffk, ctx):
    """A nearly exact preconditioner (60 pivoted-Cholesky columns of n = 180)
    and a tolerance below what split-BF16 products can hold: the recursive
    residual falls to 1e-9 in a few iterations while the true one stays near
    1e-5.  The refresh escalates and CG restarts from the true residual (p =
    z); the solve then reaches 1e-8 within a few iterations (keeping the
    stale direction, it stagnated for thousands)."""
    s = synth.make_system(5, 12, 0.1, False, 31, 32, 33)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    K = ok.dense_kernel(s.R, SIGMA)
    lam = 1e-4 * np.abs(K).max()
    F = s.flat_forces()
    idx = ffk.nystrom_select(ctx, S, "pivchol", 60)
    P = ffk.precond_build(ctx, S, idx, lam, store=ffk.FP32)
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), lam, tol=1e-8, max_iter=3000, prec=ffk.BF16X3, refresh_every=10,
                           escalate=True, switch_below=0.7, switch_from=ffk.FP32)
    res = oracle_relres(K, lam, host(a), F)
    print("gap escalation with restart: %d iterations, %d escalations %s, oracle residual %.3e"
          % (rep.iters, rep.n_escalations, tuple(rep.esc_iter), res), flush=True)
    assert rep.status == 0 and res <= 1.01e-8
    assert rep.iters <= 200 and rep.n_escalations >= 1


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_pcg_resume_continues_the_solve(ffk, ctx, small, prec):
    """A solve stopped halfway and resumed from (alpha, direction) continues
    the same CG: the resume replaces r by the true residual, as a refresh does,
    and keeps the direction, so the two parts together take about the
    iterations of the uninterrupted solve.  A resume without the direction
    (a restart from p = P^-1 r) converges too.  Checked against the oracle's
    dense residual."""
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    Fd = dev(F)
    kw = dict(tol=1e-8, prec=ffk.PRECISIONS[prec], refresh_every=10, escalate=True,
              switch_below=0.7 if prec != "fp64" else 0.0, switch_from=ffk.FP32 if prec != "fp64" else ffk.FP64)
    _, full = ffk.pcg_solve(ctx, S, P, Fd, cfg.lam, max_iter=20000, **kw)
    assert full.status == 0
    half = max(2, full.iters // 2)
    a = torch.empty_like(Fd)
    d = torch.empty_like(Fd)
    a, r1 = ffk.pcg_solve(ctx, S, P, Fd, cfg.lam, max_iter=half, alpha=a, direction=d, **kw)
    assert r1.status != 0 and r1.iters == half
    a2, r2 = ffk.pcg_solve(ctx, S, P, Fd, cfg.lam, max_iter=20000, alpha=a.clone(), direction=d.clone(),
                           resume=True, **kw)
    a3, r3 = ffk.pcg_solve(ctx, S, P, Fd, cfg.lam, max_iter=20000, alpha=a.clone(), resume=True, **kw)
    print("%s: uninterrupted %d iterations; %d + %d resumed with the direction; %d + %d restarted"
          % (prec, full.iters, r1.iters, r2.iters, r1.iters, r3.iters), flush=True)
    assert r2.status == 0 and r3.status == 0
    assert r1.iters + r2.iters <= full.iters + max(3, full.iters // 20)
    for x in (a2, a3):
        assert oracle_relres(K, cfg.lam, host(x), F) <= 1.01e-8
    # a converged alpha resumes to an immediate stop
    _, r4 = ffk.pcg_solve(ctx, S, P, Fd, cfg.lam, alpha=a2.clone(), resume=True, **kw)
    assert r4.status == 0 and r4.iters == 0


def test_pcg_rejects_reduced_first_phase(ffk, ctx, small):
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = dev(s.flat_forces())
    with pytest.raises(ffk.FfkError):
        ffk.pcg_solve(ctx, S, P, F, cfg.lam, prec=ffk.BF16X3, switch_below=0.7, switch_from=ffk.BF16)


def test_pcg_options_flexible_timing_history_progress(ffk, ctx, small, capfd):
    """The solve's optional outputs: Polak-Ribiere beta (flexible) reaches the
    oracle's bound; phase timing changes nothing but the clocks (it only adds
    events and waits); the residual history has one entry per iteration and
    reaches the tolerance; progress lines go to stderr."""
    cfg, s, S, K, idx = small
    P = ffk.precond_build(ctx, S, idx, cfg.lam, store=ffk.FP32)
    F = s.flat_forces()
    kw = dict(tol=1e-6, prec=ffk.BF16X3, refresh_every=10, escalate=True, max_iter=20000)
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, flexible=True, **kw)
    print("m9_n200 flexible iters", rep.iters, rep.rel_res_true, flush=True)
    assert rep.status == 0
    assert oracle_relres(K, cfg.lam, host(a), F) <= 1.01e-6
    a0, r0 = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, hist_cap=50000, progress_every=100, **kw)
    a1, r1 = ffk.pcg_solve(ctx, S, P, dev(F), cfg.lam, timing=True, **kw)
    assert (r1.iters, r1.rel_res_true) == (r0.iters, r0.rel_res_true)
    assert torch.equal(a0, a1)
    assert min(r1.t_mvm_ms, r1.t_prec_ms, r1.t_vec_ms) > 0.0 and r1.t_total_ms > 0.0
    h = np.array(r0.hist)
    assert len(h) == r0.iters and np.all(h > 0) and h.min() <= 1e-6
    err = capfd.readouterr().err
    assert err.count("pcg it ") == r0.iters // 100


def test_product_phase_clocks(ffk, ctx):
    """kernel_mvm_phases: five phase times per product (J v, column sums,
    GEMM 1 with its epilogue, GEMM 2, J^T G) in every precision.  The BF16
    products at this width (D = 21) run both GEMMs as one fused kernel: its
    time is the GEMM 1 phase and the GEMM 2 phase is empty."""
    s = system(7, 300, 500)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = dev(synth.random_vectors(S.n, 9))
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        ph = ffk.kernel_mvm_phases(ctx, S, v, prec=ffk.PRECISIONS[prec], iters=3)
        print("phases", prec, {k: round(t, 4) for k, t in ph.items()}, flush=True)
        t = list(ph.values())
        assert len(t) == 5 and all(np.isfinite(x) and x >= 0.0 for x in t)
        fused = prec in ("bf16x3", "bf16")
        assert all(x > 0.0 for i, x in enumerate(t) if not (fused and i == 3))


def test_full_rank_nystrom_preconditioner_solves_at_once(ffk, ctx):
    """Every numerically independent column (pivoted Cholesky asked for k = n
    stops at the rank, n - 6N): the factor reproduces K, so P = K + lambda I
    and PCG converges in a couple of iterations to the exact (Cholesky)
    solution."""
    s = system(5, 20, 305)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    K = ok.dense_kernel(s.R, SIGMA)
    lam = 1e-3 * np.abs(np.diag(K)).max()
    idx = ffk.nystrom_select(ctx, S, "pivchol", S.n)
    P = ffk.precond_build(ctx, S, idx, lam, store=ffk.FP64)
    L = host(ffk.precond_export(ctx, P, S.n))
    err = np.abs(L @ L.T - K).max() / np.abs(K).max()
    print("full-rank Nystrom: k_eff", P.k_eff, "of n", S.n, "|LL^T - K| / |K|", err, flush=True)
    assert P.k_eff == S.n - 6 * S.N
    assert err <= 1e-9
    F = s.flat_forces()
    a, rep = ffk.pcg_solve(ctx, S, P, dev(F), lam, tol=1e-10, prec=ffk.FP64, max_iter=50)
    print("  iterations", rep.iters, "residual", rep.rel_res_true, flush=True)
    assert rep.status == 0 and rep.iters <= 3
    ref = osv.cholesky_solve(K, lam, F)
    assert np.linalg.norm(host(a) - ref) <= 1e-8 * np.linalg.norm(ref)

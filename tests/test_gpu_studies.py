"""The studies built on the solver, checked on the GPU against the oracle:
the rule of thumb for the preconditioner size (section 4.3, Eq. 7-8) and the
spectrum of the Nystroem-preconditioned system (section 4.1).

Rule of thumb: a k-sweep of PCG iteration counts on the small workload (M = 9,
N = 200, n = 5400, lambda = 1e-8, uniform columns from the seeded stream, so
oracle and library use the same columns).  The library's FP64 PCG counts must
be within 5% of the oracle's textbook PCG on the dense K, and the power law
fitted by ffk_rot_fit to the library's counts must equal the oracle's fit of
the same counts and agree with the oracle's fit of its own counts.

Spectrum: at n = 1008 the generalized eigenvalues of (K + lambda I, L L^T +
lambda I) from the library's K (its column kernel) and factor L must match
those from the oracle's dense K and its incomplete Cholesky in the same column
order: the 50 largest to 1e-6 relative, for uniform and pivoted-Cholesky
columns.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import synth
from oracle import kernel as ok
from oracle import rot
from oracle import select as osel
from oracle import solve as osv

pytestmark = pytest.mark.gpu


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


@pytest.mark.timeout(600)
def test_rule_of_thumb_sweep_against_oracle_pcg(ffk, ctx):
    cfg = synth.CONFIGS["m9_n200"]
    s = synth.config_system(cfg)
    S = ffk.descriptor_build(ctx, dev(s.R), cfg.sigma)
    K = ok.dense_kernel(s.R, cfg.sigma)
    n, lam = S.n, cfg.lam
    F = s.flat_forces()
    Fd = dev(F)
    ks = [50, 100, 200, 400, 800]
    it_gpu, it_or = [], []
    for k in ks:
        idx = osel.select_uniform(n, k, cfg.sel_seed)
        P = ffk.precond_build(ctx, S, dev(idx, torch.int64), lam, store=ffk.FP64)
        _, rep = ffk.pcg_solve(ctx, S, P, Fd, lam, tol=1e-6, prec=ffk.FP64, max_iter=4 * n)
        assert rep.status == 0
        L, _, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), k, order=idx)
        L = L[:, np.any(L != 0, axis=0)]             # columns the forced order skipped stay zero
        assert L.shape[1] == keff
        _, it, _ = osv.pcg(lambda v: K @ v + lam * v, F, osv.woodbury(L, lam), tol=1e-6)
        print("k %4d: library %5d iterations, oracle %5d" % (k, rep.iters, it), flush=True)
        assert abs(rep.iters - it) <= 0.05 * it
        it_gpu.append(rep.iters)
        it_or.append(it)
    kmin_g, m_g = ffk.rot_fit(ks, it_gpu, n)
    kmin_same, m_same = rot.fit_power_law(ks, it_gpu, n)
    kmin_o, m_o = rot.fit_power_law(ks, it_or, n)
    print("fit: library k_min %.2f m %.4f; oracle fit of the library counts %.2f %.4f; of its own %.2f %.4f"
          % (kmin_g, m_g, kmin_same, m_same, kmin_o, m_o), flush=True)
    assert kmin_g == pytest.approx(kmin_same, rel=1e-12) and m_g == pytest.approx(m_same, rel=1e-12)
    assert m_g == pytest.approx(m_o, rel=0.05)
    assert kmin_g == pytest.approx(kmin_o, rel=0.15)
    # the rule of thumb (Eq. 8) from either fit picks nearly the same k
    k_g = ffk.rule_of_thumb(n, kmin_g, m_g)
    k_o = rot.k_rule_of_thumb(n, kmin_o, m_o)
    print("k_RoT: library %d, oracle %.1f" % (k_g, k_o), flush=True)
    assert abs(k_g - k_o) <= 0.05 * k_o


@pytest.mark.parametrize("strategy", ["uniform", "pivchol"])
def test_preconditioned_spectrum_against_oracle(ffk, ctx, strategy):
    from paper_2212_12737_amd.study import nystrom_preconditioned_spectrum
    s = synth.make_system(6, 56, 0.08, True, 810, 811, 812)
    S = ffk.descriptor_build(ctx, dev(s.R), 10.0)
    n, lam, k, top = S.n, 1e-6, 100, 50
    assert n == 1008
    idx = ffk.nystrom_select(ctx, S, strategy, k, lam=lam, seed=813)
    P = ffk.precond_build(ctx, S, idx, lam, store=ffk.FP64)
    K_lib = ffk.kernel_columns(ctx, S, torch.arange(n, device="cuda")).cpu().numpy()
    K_lib = 0.5 * (K_lib + K_lib.T)
    L_lib = ffk.precond_export(ctx, P, n).cpu().numpy()
    w_lib_all = nystrom_preconditioned_spectrum(K_lib, L_lib, lam)
    w_lib = w_lib_all[:top]
    # the oracle: dense K and the incomplete Cholesky in the library's column order
    K = ok.dense_kernel(s.R, 10.0)
    Lo, _, keff, _ = osel.incomplete_cholesky(lambda i: K[:, i], np.diag(K), k, order=idx.cpu().numpy())
    Lo = Lo[:, np.any(Lo != 0, axis=0)]
    assert Lo.shape[1] == keff
    w_or = sla.eigh(K + lam * np.eye(n), Lo @ Lo.T + lam * np.eye(n), eigvals_only=True)[::-1][:top]
    err = np.abs(w_lib - w_or) / np.abs(w_or)
    print("%s k=%d: largest %.6e (oracle %.6e), 50th %.6e (oracle %.6e), max rel. deviation %.2e, smallest %.6f"
          % (strategy, P.k_eff, w_lib[0], w_or[0], w_lib[-1], w_or[-1], err.max(), w_lib_all[-1]), flush=True)
    assert P.k_eff == keff
    assert err.max() <= 1e-6
    # P^-1 K_lambda >= 1: a Nystroem approximation never exceeds K
    assert w_lib_all[-1] >= 1.0 - 1e-6

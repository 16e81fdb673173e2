"""Argument checks at the C ABI and the method's degenerate cases.

Every rejected call must raise (a negative status) before any kernel runs,
and leave the context usable: each test ends with a valid call on the same
context.  Degenerate inputs with a defined answer must return it: F = 0
gives alpha = 0 at once.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok

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


@pytest.fixture(scope="module")
def small(ffk, ctx):
    s = synth.make_system(5, 40, 0.05, True, 71, 72, 73)
    S = ffk.descriptor_build(ctx, torch.as_tensor(s.R, device="cuda"), SIGMA)
    return s, S


def still_works(ffk, ctx, s, S):
    v = synth.random_vectors(S.n, 3)
    y = ffk.kernel_mvm(ctx, S, torch.as_tensor(v, device="cuda")).cpu().numpy()
    ref = ok.kernel_mvm(s.R, s.R, v, SIGMA)
    assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref)


def test_descriptor_arguments(ffk, ctx, small):
    s, S = small
    R = torch.as_tensor(s.R, device="cuda")
    print("descriptor argument checks", flush=True)
    for bad in (R[:0], R[:, :2]):                       # no geometries; fewer than 3 atoms
        with pytest.raises(ffk.FfkError):
            ffk.descriptor_build(ctx, bad, SIGMA)
    for sigma in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(ffk.FfkError):
            ffk.descriptor_build(ctx, R, sigma)
    still_works(ffk, ctx, s, S)


def test_selection_and_build_arguments(ffk, ctx, small):
    s, S = small
    print("selection and build argument checks", flush=True)
    for k in (0, S.n + 1):
        with pytest.raises(ffk.FfkError):
            ffk.nystrom_select(ctx, S, "uniform", k, seed=1)
    with pytest.raises(ffk.FfkError):                   # leverage scores need lambda > 0
        ffk.nystrom_select(ctx, S, "leverage", 10, lam=0.0, seed=1)
    # one column from each of 10 geometries (the 3M columns of one geometry
    # have rank 3M - 6: rigid motions are in the kernel's null space)
    good = torch.arange(0, 10 * 3 * 5, 3 * 5, dtype=torch.int64, device="cuda")
    for idx in (torch.tensor([0, 5, -1], device="cuda"), torch.tensor([0, S.n], device="cuda"),
                torch.empty(0, dtype=torch.int64, device="cuda")):
        with pytest.raises(ffk.FfkError):
            ffk.precond_build(ctx, S, idx, 1e-6)
    for lam in (0.0, -1e-6, float("nan")):
        with pytest.raises(ffk.FfkError):
            ffk.precond_build(ctx, S, good, lam)
    with pytest.raises(ffk.FfkError):
        ffk.kernel_columns(ctx, S, torch.tensor([3, S.n], device="cuda"))
    P = ffk.precond_build(ctx, S, good, 1e-6)
    assert P.k_eff == 10
    still_works(ffk, ctx, s, S)


def test_solve_arguments_and_zero_forces(ffk, ctx, small):
    s, S = small
    print("solve argument checks", flush=True)
    idx = ffk.nystrom_select(ctx, S, "uniform", 60, seed=2)
    P = ffk.precond_build(ctx, S, idx, 1e-6)
    F = torch.as_tensor(s.flat_forces(), device="cuda")
    for kw in (dict(lam=0.0), dict(lam=-1.0), dict(tol=0.0), dict(prec=7)):
        args = dict(lam=1e-6, tol=1e-6, prec=ffk.FP64)
        args.update(kw)
        lam = args.pop("lam")
        with pytest.raises(ffk.FfkError):
            ffk.pcg_solve(ctx, S, P, F, lam, **args)
    Fn = F.clone()
    Fn[7] = float("nan")
    with pytest.raises(ffk.FfkError):
        ffk.pcg_solve(ctx, S, P, Fn, 1e-6)
    # a preconditioner built for another system
    other = synth.make_system(5, 41, 0.05, True, 71, 74, 73)
    S2 = ffk.descriptor_build(ctx, torch.as_tensor(other.R, device="cuda"), SIGMA)
    P2 = ffk.precond_build(ctx, S2, torch.arange(20, device="cuda"), 1e-6)
    with pytest.raises(ffk.FfkError):
        ffk.pcg_solve(ctx, S, P2, F, 1e-6)
    # the product refuses to overwrite its input
    with pytest.raises(ffk.FfkError):
        ffk.kernel_mvm(ctx, S, F, y=F)
    # F = 0: alpha = 0 at once, whatever the schedule
    Z = torch.zeros_like(F)
    for prec, sw in ((ffk.FP64, 0.0), (ffk.BF16X3, 0.7)):
        a, rep = ffk.pcg_solve(ctx, S, P, Z, 1e-6, prec=prec, switch_below=sw)
        assert rep.status == 0 and rep.iters == 0
        assert torch.count_nonzero(a).item() == 0
    # resuming a solve of F = 0 from a nonzero alpha returns alpha = 0 as well
    a0 = torch.ones_like(F)
    a, rep = ffk.pcg_solve(ctx, S, P, Z, 1e-6, alpha=a0, direction=torch.ones_like(F), resume=True)
    assert rep.status == 0 and rep.iters == 0 and torch.count_nonzero(a).item() == 0
    # resume needs the starting alpha; the direction may not alias F or alpha
    with pytest.raises(ValueError):
        ffk.pcg_solve(ctx, S, P, F, 1e-6, resume=True)
    with pytest.raises(ffk.FfkError):
        ffk.pcg_solve(ctx, S, P, F, 1e-6, alpha=torch.zeros_like(F), direction=F, resume=True)
    still_works(ffk, ctx, s, S)

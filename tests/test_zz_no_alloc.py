"""The caller-free product (ffk_kernel_mvm_noalloc) against ffk_kernel_mvm.

Both run the same kernels on the same inputs; only the workspace differs
(the library's fixed scratch array instead of the system's own buffers), so
their outputs agree bit for bit, and both meet the oracle's bound.  Two calls
in a row, the second on a smaller system, show that what the first call left
in the shared scratch does not leak into the second.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok

pytestmark = pytest.mark.gpu

SIGMA = 10.0
TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6, "bf16": 3e-3}


@pytest.fixture(scope="module")
def ffk():
    from paper_2212_12737_amd import ffk as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(ffk):
    return ffk.create(0)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "fp32", "bf16"])
def test_noalloc_product_equals_the_allocating_one(ffk, ctx, prec):
    p = ffk.PRECISIONS[prec]
    # first a larger system, then a smaller one: the second call runs on
    # scratch that the first one filled
    for M, N, seed, shift in ((21, 1100, 700, 0.0), (7, 300, 710, 0.37)):
        print("noalloc", prec, "M", M, "N", N, flush=True)
        s = synth.make_system(M, N, 0.08, True, seed, seed + 1, seed + 2)
        S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
        vh = synth.random_vectors(S.n, seed)
        v = dev(vh)
        y_ref = ffk.kernel_mvm(ctx, S, v, shift=shift, prec=p)      # builds the coefficients
        y = torch.full_like(v, float("nan"))
        ffk.kernel_mvm_noalloc(ctx, S, v, y, shift=shift, prec=p)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        ref = ok.kernel_mvm(s.R, s.R, vh, SIGMA) + shift * vh
        err = relerr(y.cpu().numpy(), ref)
        print("  relerr against the oracle %.3e" % err, flush=True)
        assert err <= TOL[prec]


def test_noalloc_repeated_calls_alternate_precisions(ffk, ctx):
    """Alternating precisions and systems on the shared scratch: each result
    still equals the allocating product's."""
    systems = []
    for M, N, seed in ((9, 700, 720), (12, 257, 730)):
        s = synth.make_system(M, N, 0.08, True, seed, seed + 1, seed + 2)
        S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
        v = dev(synth.random_vectors(S.n, seed))
        refs = {p: ffk.kernel_mvm(ctx, S, v, prec=ffk.PRECISIONS[p]) for p in ("fp64", "bf16x3")}
        systems.append((S, v, refs))
    for rep in range(2):
        for S, v, refs in systems:
            for p in ("bf16x3", "fp64"):
                y = torch.empty_like(v)
                ffk.kernel_mvm_noalloc(ctx, S, v, y, prec=ffk.PRECISIONS[p])
                assert torch.equal(y, refs[p]), (rep, S.N, p)


def test_noalloc_rejects_unprepared_and_oversized_systems(ffk, ctx):
    s = synth.make_system(6, 50, 0.05, True, 740, 741, 742)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = dev(synth.random_vectors(S.n, 3))
    y = torch.empty_like(v)
    with pytest.raises(ffk.FfkError):       # no FP32 product yet on this system
        ffk.kernel_mvm_noalloc(ctx, S, v, y, prec=ffk.FP32)
    big = synth.make_system(4, 4200, 0.05, True, 743, 744, 745)
    B = ffk.descriptor_build(ctx, dev(big.R), SIGMA)
    vb = dev(synth.random_vectors(B.n, 4))
    ffk.kernel_mvm(ctx, B, vb, prec=ffk.FP64)
    with pytest.raises(ffk.FfkError):       # FP64 -W alone is 4352^2 x 8 B > 128 MiB
        ffk.kernel_mvm_noalloc(ctx, B, vb, torch.empty_like(vb), prec=ffk.FP64)
    # the context stays usable
    ffk.kernel_mvm(ctx, S, v, prec=ffk.FP32)
    ffk.kernel_mvm_noalloc(ctx, S, v, y, prec=ffk.FP32)
    assert torch.equal(y, ffk.kernel_mvm(ctx, S, v, prec=ffk.FP32))

"""The fused kernel product (both dense steps of the product in one kernel, W
kept on chip; BF16 and split-BF16 products at descriptor widths D <= 96, and
96 < D <= 128 up to N_t N_s = 4096^2, where it was measured faster than the
two-GEMM form) against the FP64 oracle.

Every K-tile count of the descriptor (KD = ceil(D / 32) = 1 .. 4) is covered,
with ragged sizes: target counts that leave a partial block of 64 targets,
source counts that leave a partial chunk of 16.  Widths above the limit
(M = 17, D = 136; M = 21, D = 210) run the two-GEMM form and must agree as
well.  The
fused product is deterministic (fixed split ranges and reduction order), so
two calls agree bit for bit; the kernel clocks show which form ran.  The full
workload sizes (M = 21 at N = 2000 and 10000, several source splits) are
checked on sampled rows in test_gpu_fullsize.py (two-GEMM form there).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok

pytestmark = pytest.mark.gpu

SIGMA = 10.0
TOL = {"bf16x3": 1e-6, "bf16": 3e-3}
# (M, N): D = M (M - 1) / 2 = 10, 36, 66, 120 -> KD = 1 .. 4 (fused); 136, 210 (two GEMMs)
CASES = [(5, 37), (9, 123), (12, 257), (16, 70), (17, 90), (21, 301)]


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


def expect_fused(D, N):
    """The library's choice of form for a square product of N geometries."""
    return D <= 96 or (D <= 128 and N * N <= 4096 * 4096)


@pytest.mark.parametrize("M,N", CASES)
def test_fused_product_every_descriptor_width(ffk, ctx, M, N):
    D = M * (M - 1) // 2
    print("fused product M %d (D %d, KD %d) N %d" % (M, D, -(-D // 32), N), flush=True)
    s = synth.make_system(M, N, 0.08, True, 800 + M, 801 + M, 802 + M)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = synth.random_vectors(S.n, 810 + M)
    ref = ok.kernel_mvm(s.R, s.R, v, SIGMA) + 0.5 * v
    for prec in ("bf16x3", "bf16"):
        ffk.clock_enable(ctx, 1)
        y = ffk.kernel_mvm(ctx, S, dev(v), shift=0.5, prec=ffk.PRECISIONS[prec])
        clk = ffk.clock_read(ctx)
        ffk.clock_enable(ctx, 0)
        err = relerr(y.cpu().numpy(), ref)
        print("  %s: relerr %.3e, fused launches %d, GEMM 1 launches %d"
              % (prec, err, clk["fused"][1], clk["gemm1"][1]), flush=True)
        assert err <= TOL[prec]
        if expect_fused(D, N):
            assert clk["fused"][1] == 1 and clk["gemm1"][1] == 0 and clk["gemm2"][1] == 0
        else:
            assert clk["fused"][1] == 0 and clk["gemm1"][1] == 1


def test_fused_product_repeats_bit_for_bit(ffk, ctx):
    s = synth.make_system(12, 1700, 0.08, True, 830, 831, 832)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    v = dev(synth.random_vectors(S.n, 833))
    for prec in (ffk.BF16X3, ffk.BF16):
        y1 = ffk.kernel_mvm(ctx, S, v, prec=prec)
        y2 = ffk.kernel_mvm(ctx, S, v, prec=prec)
        assert torch.equal(y1, y2)


def test_fused_product_is_symmetric_and_agrees_with_fp64(ffk, ctx):
    """u^T K v = v^T K u to split-BF16 rounding, and the product agrees with
    the library's own FP64 product (M = 12, N = 5000: several source splits,
    several rounds of workgroups)."""
    s = synth.make_system(12, 5000, 0.08, True, 840, 841, 842)
    S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
    u = dev(synth.random_vectors(S.n, 843))
    v = dev(synth.random_vectors(S.n, 844))
    Kv = ffk.kernel_mvm(ctx, S, v, prec=ffk.BF16X3)
    Ku = ffk.kernel_mvm(ctx, S, u, prec=ffk.BF16X3)
    Kv64 = ffk.kernel_mvm(ctx, S, v, prec=ffk.FP64)
    err = (torch.linalg.norm(Kv - Kv64) / torch.linalg.norm(Kv64)).item()
    a, b = torch.dot(u, Kv).item(), torch.dot(v, Ku).item()
    scale = (torch.linalg.norm(u) * torch.linalg.norm(Kv)).item()
    print("fused vs FP64 product %.3e; |u^T K v - v^T K u| / scale %.3e" % (err, abs(a - b) / scale), flush=True)
    assert err <= 1e-6
    assert abs(a - b) <= 1e-6 * scale


def test_form_switches_at_the_size_limit(ffk, ctx):
    """D = 120: fused up to N = 4096, two GEMMs above (the clocks tell), and
    both agree with the library's FP64 product to the split-BF16 bound."""
    for N in (4096, 4200):
        s = synth.make_system(16, N, 0.08, True, 850, 851, 852)
        S = ffk.descriptor_build(ctx, dev(s.R), SIGMA)
        v = dev(synth.random_vectors(S.n, 853))
        ffk.clock_enable(ctx, 1)
        y = ffk.kernel_mvm(ctx, S, v, prec=ffk.BF16X3)
        clk = ffk.clock_read(ctx)
        ffk.clock_enable(ctx, 0)
        y64 = ffk.kernel_mvm(ctx, S, v, prec=ffk.FP64)
        err = (torch.linalg.norm(y - y64) / torch.linalg.norm(y64)).item()
        print("D 120 N %d: fused launches %d, GEMM 1 launches %d, vs FP64 %.2e"
              % (N, clk["fused"][1], clk["gemm1"][1], err), flush=True)
        assert err <= 1e-6
        assert (clk["fused"][1] == 1) == expect_fused(120, N)
        assert (clk["gemm1"][1] == 1) == (not expect_fused(120, N))

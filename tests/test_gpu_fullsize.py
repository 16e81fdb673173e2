"""GPU kernel products at the full workload sizes (large-tile GEMM path),
checked against the FP64 oracle on sampled target geometries.

The oracle evaluates the product one target geometry at a time
(y_i = sum_j J_i^T H_ij J_j v_j), so a handful of rows of the
n = 630000 and n = 3.6M products is cheap; the first, last and middle
geometries and a seeded random set are compared.  Tolerances are norm-wise
relative errors over the sampled rows: FP64 products agree to rounding, the
FP32 and split-BF16 products (FP32 accumulation over K = 2N terms) to a few
units of 1e-6, single BF16 to its 8-bit mantissa.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import kernel as ok

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 2e-5, "bf16x3": 2e-5, "bf16": 5e-3}


@pytest.fixture(scope="module")
def ffk():
    from paper_2212_12737_amd import ffk as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(ffk):
    return ffk.create(0)


def sample_targets(N, seed=0, extra=4):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, 1, N // 2, N - 1], rng.integers(0, N, extra)]))


@pytest.mark.parametrize("name", ["m42_n5000", "m60_n20000"])
def test_full_size_products_match_oracle_rows(ffk, ctx, name):
    cfg = synth.CONFIGS[name]
    s = synth.config_system(cfg)
    print("full-size products", name, flush=True)
    S = ffk.descriptor_build(ctx, torch.as_tensor(s.R, device="cuda"), cfg.sigma)
    v = synth.random_vectors(S.n, 21)
    vd = torch.as_tensor(v, device="cuda")
    tg = sample_targets(cfg.N)
    ref = ok.kernel_mvm(s.R, s.R, v, cfg.sigma, targets=tg, chunk=1)
    m3 = 3 * cfg.M
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        print("  precision", prec, flush=True)
        y = ffk.kernel_mvm(ctx, S, vd, prec=ffk.PRECISIONS[prec]).cpu().numpy().reshape(cfg.N, m3)[tg]
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        print("  relerr", prec, err, flush=True)
        assert err <= TOL[prec]

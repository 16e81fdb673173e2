"""Host-side models of bench.py: algorithmic work per kernel launch and the
per-iteration bound of the timed solve, checked against hand counts."""
import pytest

import bench
import synth


def test_product_flops_match_the_gemm_shapes():
    # GEMM 1 (N x D)(D x N): 2 N^2 D; GEMM 2 (N x 2N)(2N x D): 4 N^2 D;
    # J v and J^T G: 12 N D each (3 coordinates, two atoms, multiply-add)
    N, D = 2000, 210
    assert bench.mvm_flops(N, D) == 2 * N * N * D + 4 * N * N * D + 24 * N * D
    assert bench.kernel_model("gemm1", N, D, 3 * 21 * N, 2000, 4)[1] == 2.0 * N * N * D
    assert bench.kernel_model("gemm2", N, D, 3 * 21 * N, 2000, 4)[1] == 4.0 * N * N * D


def test_gemv_bytes_are_one_pass_over_l_plus_the_vector():
    n, k = 126000, 2000
    bound, b_t, unit = bench.kernel_model("gemv_t", 2000, 210, n, k, 4)
    assert (bound, unit) == ("hbm", "B")
    assert b_t == 4 * n * k + 8 * n
    assert bench.kernel_model("gemv_n", 2000, 210, n, k, 4)[1] == 4 * n * k + 8 * k
    assert bench.kernel_model("nonexistent", 1, 1, 1, 1, 4) is None


@pytest.mark.parametrize("first", ["fp32", "fp64"])
def test_iteration_roofline_by_hand(first):
    cfg = synth.CONFIGS["m21_n2000"]
    n, k = 3 * cfg.M * cfg.N, 2000
    rec = {"iters": 1000, "switch_iter": 200, "n_refresh": 100, "t_pcg_s": 1.0, "switch_from": first}
    out = bench.iteration_roofline(cfg, n, k, rec)
    hbm = 8000e9
    F = bench.mvm_flops(cfg.N, cfg.D)
    apply = (2 * 4 * n * k + 13 * 8 * n) / hbm
    t64 = max(F / 78.6e12, 32 * cfg.N ** 2 / hbm)
    t32 = max(F / 157.3e12, 16 * cfg.N ** 2 / hbm)
    tx3 = max(3 * F / 2500e12, 16 * cfg.N ** 2 / hbm)
    want = 1000 * apply + 200 * (t32 if first == "fp32" else t64) + 100 * t64 + 800 * tx3
    assert out["ideal_pcg_s"] == pytest.approx(want, rel=1e-12)
    assert out["frac"] == pytest.approx(want / 1.0, rel=1e-12)
    assert out["products"] == {"first_phase_" + first: 200, "fp64_refresh": 100, "bf16x3": 800}
    # at this size the products are MFMA-bound in FP64, N x N-traffic-bound in split BF16
    assert t64 == F / 78.6e12 and tx3 == 16 * cfg.N ** 2 / hbm


def test_more_than_one_gpu_is_refused_before_any_gpu_work(capsys):
    # one GPU only: the bench exits with status 2 and says why, before it
    # imports torch or touches a device
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err

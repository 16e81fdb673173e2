"""The C ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffkrr.h")
LIB = os.path.join(ROOT, "paper_2212_12737_amd", "libffkrr.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffk_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_header_and_host_only_calls():
    from paper_2212_12737_amd import ffk
    assert set(declared()) == set(ffk.exported_symbols())
    assert ffk.version().startswith("ffkrr")
    from oracle import rot
    for n, kmin, m in [(63000, 100, 1.0), (500000, 236, 1.14), (5400, 10, 0.87)]:
        assert ffk.rule_of_thumb(n, kmin, m) == round(rot.k_rule_of_thumb(n, kmin, m))
    assert ffk.mlp_num_params(210, 256) == 210 * 256 + 256 + 256 * 256 + 256 + 256 + 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_power_law_fit_matches_oracle():
    """ffk_rot_fit (host computation) against the oracle's least-squares fit,
    on noisy counts, and its argument checks."""
    import numpy as np
    from paper_2212_12737_amd import ffk
    from oracle import rot
    rng = np.random.default_rng(3)
    n = 31500
    for kmin, m in [(236.0, 1.14), (10.0, 0.87), (400.0, 0.6)]:
        k = np.array([125, 250, 500, 1000, 2000, 4000])
        iters = np.maximum(1, np.round(n * (kmin / k) ** m * np.exp(rng.normal(0, 0.05, k.size)))).astype(np.int64)
        got = ffk.rot_fit(k, iters, n)
        want = rot.fit_power_law(k, iters, n)
        assert abs(got[0] / want[0] - 1) < 1e-12 and abs(got[1] / want[1] - 1) < 1e-12
    for k, it in [([100], [50]), ([100, 100], [50, 40]), ([100, 200], [40, 50]), ([0, 200], [40, 50])]:
        with pytest.raises(ffk.FfkError):
            ffk.rot_fit(k, it, n)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_calibrated_rule_of_thumb_matches_brute_force():
    from paper_2212_12737_amd import ffk
    from oracle import rot
    cases = [(15750, 100.0, 1.0, 15750.0 ** 2, 0.0, 15750.0), (126000, 65.0, 0.92, 2e-4, 1.65e-7, 2.2e-8),
             (126000, 65.0, 0.92, 2e-4, 0.0, 2.2e-8), (31500, 236.0, 1.14, 1e-4, 3e-8, 1e-9),
             (5400, 10.0, 0.87, 0.0, 1e-6, 1e-6), (5400, 10.0, 1.3, 1.0, 1.0, 0.0)]
    for n, kmin, m, a, b, c in cases:
        got = ffk.rule_of_thumb_calibrated(n, kmin, m, a, b, c)
        want = rot.k_calibrated(n, kmin, m, a, b, c)
        f = lambda k: float(rot.runtime_calibrated(k, n, kmin, m, a, b, c))
        assert got == want or abs(f(got) / f(want) - 1) < 1e-12, (n, kmin, m, a, b, c, got, want)
    assert ffk.rule_of_thumb_calibrated(100, 10.0, 1.0, 0.0, 0.0, 1.0) == -1
    assert ffk.rule_of_thumb_calibrated(0, 10.0, 1.0, 1.0, 0.0, 1.0) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built library every call raises."""
    from paper_2212_12737_amd import ffk
    monkeypatch.setattr(ffk, "_lib", None)
    monkeypatch.setattr(ffk, "LIB_PATH", str(tmp_path / "libffkrr.so"))
    with pytest.raises(RuntimeError, match="not built"):
        ffk.lib()
    with pytest.raises(RuntimeError, match="not built"):
        ffk.rule_of_thumb(1000)

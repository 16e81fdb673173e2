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

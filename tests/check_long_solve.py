"""Independent FP64 check of a solve's result at full size (test infrastructure).

    python tests/check_long_solve.py --config m60_n20000 --alpha DIR/alpha.npy [--workers 8]

Regenerates the workload's system from its seeds and computes the true
relative residual |F - (K + lambda I) alpha| / |F| of the given alpha with
the oracle's matrix-free FP64 product over every geometry, split over host
processes (tests/oracle_parallel.py).  Nothing of the library runs here; one
JSON line is printed.  At M = 60, N = 20000 this takes about 0.26 s of one
core per target geometry.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import oracle_parallel  # noqa: E402
import synth  # noqa: E402


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="m60_n20000")
    ap.add_argument("--alpha", required=True)
    ap.add_argument("--workers", type=int, default=0)
    a = ap.parse_args(argv)
    cfg = synth.CONFIGS[a.config]
    s = synth.config_system(cfg)
    F = s.flat_forces()
    alpha = np.load(a.alpha, allow_pickle=False)
    assert alpha.shape == F.shape, (alpha.shape, F.shape)
    t0 = time.perf_counter()
    Ka = oracle_parallel.kernel_mvm(s.R, s.R, alpha, cfg.sigma, workers=a.workers or None)
    res = F - Ka - cfg.lam * alpha
    rel = float(np.linalg.norm(res) / np.linalg.norm(F))
    print(json.dumps({"config": a.config, "alpha": a.alpha, "oracle_true_rel_residual": rel,
                      "seconds": time.perf_counter() - t0,
                      "workers": a.workers or oracle_parallel.cores()}), flush=True)


if __name__ == "__main__":
    main()

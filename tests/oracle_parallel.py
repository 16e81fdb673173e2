"""The oracle's matrix-free product over all host cores (test helper).

The oracle evaluates y = K(tgt, src) v one target geometry at a time, so the
target geometries split over worker processes without changing any
arithmetic: each worker runs oracle.kernel.kernel_mvm on its share of the
targets (one BLAS thread each) and the rows are put back in order.  Workers
are forked; they run numpy only.  The inputs travel to them by the fork
itself (module globals set just before the pool starts).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_INPUT = None


def cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, min(n, 16))


def _rows(targets):
    from threadpoolctl import threadpool_limits
    from oracle import kernel as ok
    R_tgt, R_src, v, sigma = _INPUT
    with threadpool_limits(1):
        return ok.kernel_mvm(R_tgt, R_src, v, sigma, targets=targets)


def kernel_mvm(R_tgt: np.ndarray, R_src: np.ndarray, v: np.ndarray, sigma: float, workers: int | None = None):
    """Flat y = K(R_tgt, R_src) v, as oracle.kernel.kernel_mvm returns it."""
    global _INPUT
    Nt = R_tgt.shape[0]
    w = min(workers or cores(), Nt)
    parts = [p for p in np.array_split(np.arange(Nt), w) if len(p)]
    _INPUT = (R_tgt, R_src, np.asarray(v, dtype=np.float64), sigma)
    try:
        pool = mp.get_context("fork").Pool(len(parts))
        try:
            rows = pool.map(_rows, parts)
        finally:
            pool.close()
            pool.join()
    finally:
        _INPUT = None
    return np.concatenate(rows, axis=0).reshape(-1)

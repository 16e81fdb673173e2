"""Pins of the rule of thumb for the preconditioner size (section 4.3, Eq. 7-8)."""
import numpy as np

from oracle import rot


def test_rule_of_thumb_is_the_minimiser():
    for n, kmin, m in [(63000, 100, 1.0), (500000, 236, 1.14), (31400, 10, 0.87)]:
        ks = np.exp(np.linspace(np.log(1), np.log(n), 200001))
        kbest = ks[np.argmin(rot.runtime_model(ks, n, kmin, m))]
        assert abs(rot.k_rule_of_thumb(n, kmin, m) / kbest - 1) < 1e-3


def test_power_law_fit_recovers_parameters():
    n = 30000
    k = np.array([100, 200, 400, 800, 1600])
    iters = n * (150.0 / k) ** 1.1
    kmin, m = rot.fit_power_law(k, iters, n)
    assert abs(kmin - 150) < 1e-6 and abs(m - 1.1) < 1e-9

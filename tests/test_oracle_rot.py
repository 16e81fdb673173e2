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


def test_calibrated_form_reduces_to_eq8():
    """With the costs of Eq. 7 (a = n^2, b = 0, c = n) the calibrated model is
    n^3 [(k_min/k)^m + (k/n)^2], whose integer minimiser is k_RoT rounded."""
    for n, kmin, m in [(15750, 100, 1.0), (63000, 236, 1.14), (31400, 10, 0.87)]:
        kc = rot.k_calibrated(n, kmin, m, float(n) ** 2, 0.0, float(n))
        assert abs(kc - rot.k_rule_of_thumb(n, kmin, m)) <= 1.0


def test_calibrated_form_moves_with_the_per_column_cost():
    """A per-iteration cost that grows with k moves the optimum to smaller k;
    stationarity of the continuous model at the integer minimiser."""
    n, kmin, m, a, c = 126000, 65.0, 0.92, 2e-4, 2.2e-8
    k0 = rot.k_calibrated(n, kmin, m, a, 0.0, c)
    k1 = rot.k_calibrated(n, kmin, m, a, 1.65e-7, c)
    assert k1 < k0
    for kk, b in [(k0, 0.0), (k1, 1.65e-7)]:
        f = lambda x: rot.runtime_calibrated(x, n, kmin, m, a, b, c)
        assert f(kk) <= f(kk - 1) and f(kk) <= f(kk + 1)

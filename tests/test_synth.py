"""The synthetic input generator: geometry constraints and force labels."""
import numpy as np

import synth


def test_equilibrium_geometry_constraints():
    R0 = synth.equilibrium_geometry(21, 2000)
    dist = np.linalg.norm(R0[:, None] - R0[None], axis=-1)
    np.fill_diagonal(dist, np.inf)
    assert dist.min() >= 1.0 - 1e-12
    # every atom after the first has a neighbour at a bond length in [1.0, 1.5]
    for p in range(1, 21):
        assert np.any((dist[p, :p] >= 1.0) & (dist[p, :p] <= 1.5))


def test_forces_are_negative_energy_gradient():
    s = synth.make_system(7, 3, 0.08, True, 5, 6, 7)
    ff = synth.draw_force_field(s.R0, 7, True)
    h = 1e-6
    R = s.R[:1].copy()
    fd = np.empty(R.size)
    flat = R.reshape(-1)
    for c in range(flat.size):
        e = np.zeros_like(flat); e[c] = h
        Ep, _ = synth.energy_and_forces((flat + e).reshape(R.shape), ff)
        Em, _ = synth.energy_and_forces((flat - e).reshape(R.shape), ff)
        fd[c] = -(Ep[0] - Em[0]) / (2 * h)
    np.testing.assert_allclose(s.F[0].reshape(-1), fd, atol=1e-7 * np.abs(fd).max())


def test_zero_net_force_and_torque():
    s = synth.config_system(synth.CONFIGS["m9_n200"])
    assert np.abs(s.F.sum(1)).max() < 1e-12
    assert np.abs(np.cross(s.R, s.F).sum(1)).max() < 1e-12


def test_mixture_of_displacement_scales():
    """Each scale contributes its share of geometries (the first takes the
    rounding remainder), in a permuted order; labels stay central pair forces."""
    s = synth.mixture_system(6, 101, (0.01, 0.3), (0.7, 0.3), True, 5, 6, 7)
    assert s.R.shape == (101, 6, 3)
    spread = np.abs(s.R - s.R0).reshape(101, -1).max(1)
    small = spread < 0.06          # 0.01 x 6 sigma
    assert small.sum() == 71 and (~small).sum() == 30
    assert not np.all(small[:71])  # shuffled, not in blocks
    assert np.abs(s.F.sum(1)).max() < 1e-12
    again = synth.mixture_system(6, 101, (0.01, 0.3), (0.7, 0.3), True, 5, 6, 7)
    assert np.array_equal(s.R, again.R)

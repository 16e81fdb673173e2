"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds input generation only: molecules, displaced geometries and
pair-potential force labels.  It contains none of the kernel-regression
arithmetic (descriptor, kernel, preconditioner, solver); both the CPU oracle and
the HIP library consume its outputs as plain arrays.
"""
from .molecules import (  # noqa: F401
    CONFIGS,
    Config,
    System,
    make_system,
    mixture_system,
    config_system,
    equilibrium_geometry,
    displaced_geometries,
    draw_force_field,
    energy_and_forces,
    random_vectors,
    random_weights,
)

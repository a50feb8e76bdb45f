"""Seeded synthetic particle sets for the SPH solid-body right-hand side.

This package only *builds inputs*: lattice positions with jitter, velocities,
densities, deviatoric stresses, masses, and the constants of each workload.
It holds none of the method's arithmetic (no kernel, no sums, no equation of
state), so both the CPU oracle and the GPU library can consume it without
sharing any of the computation.
"""
from .generate import (  # noqa: F401
    Workload,
    MATERIAL,
    PARAM_ORDER,
    config,
    cube,
    two_particles,
    lattice_cube,
    random_state,
    subsample,
    flaws,
    CONFIG_NAMES,
)

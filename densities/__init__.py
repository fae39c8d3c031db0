"""Seeded synthetic charge densities shared by the tests, the smoke check and
the benchmark.

This module holds no Poisson-solver arithmetic: it only draws and evaluates
Gaussian charge clouds on a grid.  Both the HIP path and the FP64 oracle take
its output as their input, so neither depends on the other.
"""

from .gaussian_mixture import (  # noqa: F401
    BATCH_BCS,
    BATCH_EDGES,
    BC_FREE,
    BC_PERIODIC,
    BC_SURFACE_Y,
    BC_WIRE_Z,
    SPACING,
    WORKLOADS,
    GaussianSpec,
    batch_density,
    batch_workload,
    draw_gaussians,
    gaussian_mixture,
    workload_density,
)

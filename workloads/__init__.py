"""Seeded synthetic inputs shaped like the paper's workloads.

This package is shared by the tests, the benchmark and the smoke check.  It
holds none of the method's arithmetic (no neighbour test, no pair force, no
prediction): it only draws star clusters -- positions, velocities, masses,
stored force derivatives, times, neighbour radii and regular time-steps --
from seeded NumPy generators.
"""
from .clusters import (  # noqa: F401
    Cluster,
    plummer,
    salpeter_masses,
    add_binaries,
    plummer_mean_field,
    neighbour_radii,
    regular_steps,
    make_cluster,
    config,
    serving_trace,
    CONFIG_SEED_BASE,
)

"""Seeded synthetic particle sets used by the tests, the benchmark and the smoke check.

This module only draws inputs (positions, velocities, masses). It holds none of the
tree-code arithmetic: no keys, no tree, no moments, no forces. Both the CPU oracle and
the HIP path consume the arrays it returns, so they always see identical inputs.

All arrays are float64 NumPy arrays: positions and velocities of shape (n, 3), masses
of shape (n,).
"""

from .batches import cluster_batch, cluster_sizes, hernquist, request_trace
from .galaxy import galaxy
from .merger import black_holes, merger, parabolic_orbit
from .plummer import plummer, plummer_radii
from .shapes import (
    two_body,
    coincident,
    on_a_line,
    lattice,
    clustered,
    uniform_cube,
)

__all__ = [
    "black_holes",
    "merger",
    "parabolic_orbit",
    "cluster_batch",
    "cluster_sizes",
    "hernquist",
    "request_trace",
    "galaxy",
    "plummer",
    "plummer_radii",
    "two_body",
    "coincident",
    "on_a_line",
    "lattice",
    "clustered",
    "uniform_cube",
]

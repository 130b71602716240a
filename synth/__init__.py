"""Seeded synthetic power-grid workloads.

This package only draws random numbers and builds graphs: branch lists,
branch parameters, bus types, planted voltages and per-case scaling factors.
It contains none of the power-flow arithmetic (no admittance matrix, no
mismatch, no gradient): both the CPU oracle and the GPU library receive its
outputs and compute everything else on their own.
"""

from .grids import (  # noqa: F401
    Grid,
    PQ,
    PV,
    SLACK,
    config0,
    config1,
    config2,
    config3,
    config4,
    flat_start,
    geometric_grid,
    non_bridge_branches,
    tree_chord_grid,
)

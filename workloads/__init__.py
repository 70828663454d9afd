"""Seeded synthetic inputs for the layered 3D-IC thermal systems.

This package only *describes* problems: layer stacks (materials, thicknesses,
conductivities, heat capacities), per-cell lateral conductivity multipliers and
power maps in watts per cell.  It holds none of the solver's arithmetic (no face
conductances, no assembly, no iteration), so that both the CPU oracle and the
GPU path can draw identical inputs from it without sharing any computation.
"""

from .stacks import (  # noqa: F401
    MATERIALS,
    CELL,
    H_TOP,
    T_AMB,
    Stack,
    config0,
    config1,
    config2_stack,
    config2_power,
    config2_floorplan_index,
    config3,
    config4,
    config4_small,
    fd_cells_config4,
    uniform_stack,
    lanczos_start,
)

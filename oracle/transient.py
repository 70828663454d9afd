"""Backward-Euler steps by direct solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper Section 3.2, eq. "transient": for the rise theta = T - T_amb,
(A + diag(C V / dt)) theta_{n+1} = p_{n+1} V + (C V / dt) theta_n.
"""

from __future__ import annotations

from typing import Callable, Optional

import numpy as np

from . import assembly, direct


def step(stack, P_next: np.ndarray, theta_n: np.ndarray, dt: float,
         solve: Optional[Callable] = None, A=None) -> np.ndarray:
    """theta_{n+1} for one step; `A` may pass a pre-assembled transient matrix."""
    if A is None:
        A = assembly.assemble(stack, dt=dt)
    b = assembly.rhs_transient(stack, P_next, theta_n, dt)
    if solve is None:
        if stack.k_lat_mult is None:
            return direct.solve_separable(stack, b, dt=dt)
        solve = direct.solve_splu
    return solve(A, b)

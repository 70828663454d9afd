"""Backward-Euler steps by direct solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper Section 3.2, eq. "transient": for the rise theta = T - T_amb,
(A + diag(C V / dt)) theta_{n+1} = p_{n+1} V + (C V / dt) theta_n.

``step`` solves one step directly; ``SeparableSteps`` runs many steps of a
per-layer-uniform stack with the operator eliminated once (pinned against
``step`` and SuperLU).
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


class SeparableSteps:
    """Backward-Euler steps of a per-layer-uniform stack by the separable solve
    (``direct.SeparableFactors``), the operator A + diag(C V / dt) eliminated
    once for every step.

    The right-hand side P_{n+1} + (C V / dt) theta_n is formed in the DCT basis
    (the capacity term is constant within each layer, so it commutes with the
    lateral transform): ``step_hat`` maps DCT coefficients to DCT coefficients,
    so a whole trajectory can stay in that basis; ``step`` takes and returns
    flat fields like ``step``."""

    def __init__(self, stack, dt: float):
        if stack.k_lat_mult is not None:
            raise ValueError("separable steps need per-layer uniform conductivity")
        self.shape = stack.shape
        self.factors = direct.SeparableFactors(stack, dt)
        cap = np.asarray(stack.heat_cap, float)
        self.cv = (cap * float(stack.dx) * float(stack.dy) * np.asarray(stack.dz, float) /
                   float(dt))[:, None, None]

    def to_hat(self, v: np.ndarray) -> np.ndarray:
        return direct.dct_layers(v, self.shape)

    def from_hat(self, vh: np.ndarray) -> np.ndarray:
        return direct.idct_layers(vh)

    def step_hat(self, P_hat: np.ndarray, theta_hat: np.ndarray) -> np.ndarray:
        return self.factors.solve_hat(P_hat + self.cv * theta_hat)

    def step(self, P_next: np.ndarray, theta_n: np.ndarray) -> np.ndarray:
        return self.from_hat(self.step_hat(self.to_hat(P_next), self.to_hat(theta_n)))

"""Smoothed-peak loss, its temperature gradient, and the adjoint gradient.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The loss is L = (1/beta) log sum_{i in Si} exp(beta T_i) (a smoothed maximum of
the silicon temperatures).  For the steady system A theta = P, T = T_amb + theta:

* dL/dT_i = softmax(beta T)_i on silicon cells, 0 elsewhere;
* dL/dP = lambda with A^T lambda = dL/dT (A = A^T), since dtheta/dP = A^{-1};
* for any conductance parameter k, dL/dk = -lambda^T (dA/dk) theta, and
  A = sum_faces g_f (e_a - e_b)(e_a - e_b)^T + diag(sink), so
  dL/dk = -sum_f (dg_f/dk) (lambda_a - lambda_b)(theta_a - theta_b).

Derivatives of the series half-cell conductances (oracle.assembly):
* a lateral face of layer l is homogeneous of degree one in k_lat[l], so
  dg/dk_lat[l] = g / k_lat[l];
* a vertical face g = dx dy / (dz_l/(2 k_l) + dz_m/(2 k_m)) between layers l and
  m = l + 1 has dg/dk_l = g^2 dz_l / (2 k_l^2 dx dy).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Callable

import numpy as np

from . import assembly


def lse_loss(T: np.ndarray, mask: np.ndarray, beta: float) -> float:
    t = beta * np.asarray(T, float).ravel()[np.asarray(mask).ravel()]
    m = t.max()
    return float((m + np.log(np.exp(t - m).sum())) / beta)


def lse_grad(T: np.ndarray, mask: np.ndarray, beta: float) -> np.ndarray:
    Tf = np.asarray(T, float).ravel()
    msk = np.asarray(mask).ravel()
    t = beta * Tf[msk]
    w = np.exp(t - t.max())
    g = np.zeros_like(Tf)
    g[msk] = w / w.sum()
    return g


@dataclass
class Gradient:
    dP: np.ndarray        # dL/dP per cell (flat)
    dk_lat: np.ndarray    # dL/dk_lat[l]
    dk_vert: np.ndarray   # dL/dk_vert[l]

    @property
    def dk_layer(self) -> np.ndarray:
        """Gradient w.r.t. one conductivity per layer scaling both directions."""
        return self.dk_lat + self.dk_vert


def gradient(stack, theta: np.ndarray, dL_dT: np.ndarray,
             solve: Callable[[object, np.ndarray], np.ndarray]) -> Gradient:
    """Adjoint gradient of L given theta = A^{-1} P and dL/dT."""
    A = assembly.assemble(stack)
    lam = solve(A, np.asarray(dL_dT, float))
    c = assembly.conductances(stack)
    th = np.asarray(theta, float).reshape(stack.shape)
    la = lam.reshape(stack.shape)
    nz = stack.nz
    kl = np.asarray(stack.k_lat, float)
    kv = np.asarray(stack.k_vert, float)
    dz = np.asarray(stack.dz, float)
    dxdy = float(stack.dx) * float(stack.dy)

    # per-layer sums of g_f (dlam)(dtheta) over lateral faces
    s_lat = (c.gx * (la[:, :, :-1] - la[:, :, 1:]) * (th[:, :, :-1] - th[:, :, 1:])).sum(axis=(1, 2))
    s_lat += (c.gy * (la[:, :-1, :] - la[:, 1:, :]) * (th[:, :-1, :] - th[:, 1:, :])).sum(axis=(1, 2))
    dk_lat = -s_lat / kl

    dk_vert = np.zeros(nz)
    for l in range(nz - 1):
        g = c.gz[l, 0, 0]
        s = ((la[l] - la[l + 1]) * (th[l] - th[l + 1])).sum()
        dk_vert[l] -= g * g * dz[l] / (2.0 * kv[l] ** 2 * dxdy) * s
        dk_vert[l + 1] -= g * g * dz[l + 1] / (2.0 * kv[l + 1] ** 2 * dxdy) * s
    return Gradient(lam, dk_lat, dk_vert)

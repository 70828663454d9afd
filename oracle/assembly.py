"""FP64 CSR assembly of the layered 7-point finite-volume system.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the paper's discretization (Section 3.2, eq. "steady-state" and eq.
"transient"): for each cell 0 with neighbours i,

    sum_i g_{0,i} (T_0 - T_i) + h S_0 T_0 = p_0 V_0 + h S_0 T_amb            (steady)
    C_0 V_0 T_{0,n+1}/dt + sum_i g_{0,i}(T_{0,n+1} - T_{i,n+1}) + h S_0 T_{0,n+1}
        = p_0 V_0 + h S_0 T_amb + C_0 V_0 T_{0,n}/dt                          (transient)

Written for the temperature rise theta = T - T_amb, the h S_0 T_amb terms cancel
and the system is A theta = b with A symmetric positive definite and 7-diagonal
(Section 3.2, last paragraph).

Readings where the paper is silent (listed in the design doc):
* g_{0,i} is the series (harmonic) conductance of the two half cells:
  lateral g = (face area) / (d/(2 k_a) + d/(2 k_b)), vertical likewise with the
  two layers' thicknesses and vertical conductivities;
* the convective term h S_0 is h * dx * dy added to the diagonal of the top
  (and, if h_bottom > 0, bottom) cells with no half-cell resistance in series;
* each face is computed once and used for both rows, so A == A^T exactly;
* power is given in watts per cell (the p_0 V_0 product).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class Conductances:
    gx: np.ndarray     # (nz, ny, nx-1) between (i, j, l) and (i+1, j, l)
    gy: np.ndarray     # (nz, ny-1, nx) between (i, j, l) and (i, j+1, l)
    gz: np.ndarray     # (nz-1, ny, nx) between (i, j, l) and (i, j, l+1)
    sink: np.ndarray   # (nz, ny, nx) diagonal-only terms: h S (+ C V / dt)


def conductances(stack, dt: Optional[float] = None,
                 k_lat: Optional[np.ndarray] = None,
                 k_vert: Optional[np.ndarray] = None) -> Conductances:
    """Face conductances (W/K) and diagonal sink terms of one stack.

    ``k_lat``/``k_vert`` override the stack's per-layer values (the multiplier
    field is still applied to the lateral one); used for perturbation checks.
    """
    nz, ny, nx = stack.shape
    dx, dy = float(stack.dx), float(stack.dy)
    dz = np.asarray(stack.dz, float)
    kl = np.asarray(stack.k_lat if k_lat is None else k_lat, float)
    kv = np.asarray(stack.k_vert if k_vert is None else k_vert, float)
    kc = np.broadcast_to(kl[:, None, None], stack.shape).copy()
    if stack.k_lat_mult is not None:
        kc = kc * np.asarray(stack.k_lat_mult, float).reshape(stack.shape)

    # lateral x faces: area dy*dz_l, two half-cell lengths dx/2
    area_x = (dy * dz)[:, None, None]
    gx = area_x / (dx / (2.0 * kc[:, :, :-1]) + dx / (2.0 * kc[:, :, 1:]))
    # lateral y faces: area dx*dz_l, half lengths dy/2
    area_y = (dx * dz)[:, None, None]
    gy = area_y / (dy / (2.0 * kc[:, :-1, :]) + dy / (2.0 * kc[:, 1:, :]))
    # vertical faces: area dx*dy, half thicknesses dz_l/2 and dz_{l+1}/2
    gz_l = (dx * dy) / (dz[:-1] / (2.0 * kv[:-1]) + dz[1:] / (2.0 * kv[1:]))
    gz = np.broadcast_to(gz_l[:, None, None], (nz - 1, ny, nx)).copy()

    sink = np.zeros(stack.shape)
    sink[nz - 1] += float(stack.h_top) * dx * dy
    sink[0] += float(stack.h_bottom) * dx * dy
    if dt is not None:
        cap = np.asarray(stack.heat_cap, float)
        sink += (cap * dx * dy * dz / float(dt))[:, None, None]
    return Conductances(gx, gy, gz, sink)


def assemble(stack, dt: Optional[float] = None, cond: Optional[Conductances] = None) -> sp.csr_matrix:
    """A (N x N, FP64 CSR) with A theta = b for the rise theta = T - T_amb."""
    c = conductances(stack, dt) if cond is None else cond
    nz, ny, nx = stack.shape
    N = nx * ny * nz
    idx = np.arange(N).reshape(stack.shape)

    rows, cols, vals = [], [], []
    diag = c.sink.copy()
    for g, a, b in (
        (c.gx, idx[:, :, :-1], idx[:, :, 1:]),
        (c.gy, idx[:, :-1, :], idx[:, 1:, :]),
        (c.gz, idx[:-1, :, :], idx[1:, :, :]),
    ):
        g = g.ravel()
        a = a.ravel()
        b = b.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-g, -g]
        np.add.at(diag.reshape(-1), a, g)
        np.add.at(diag.reshape(-1), b, g)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def rhs_steady(P: np.ndarray) -> np.ndarray:
    """b = p V (watts per cell) for the steady rise system."""
    return np.asarray(P, float).ravel().copy()


def rhs_transient(stack, P_next: np.ndarray, theta_n: np.ndarray, dt: float) -> np.ndarray:
    """b = p_{n+1} V + C V theta_n / dt (eq. transient, rise form)."""
    cap = np.asarray(stack.heat_cap, float)
    cv = (cap * float(stack.dx) * float(stack.dy) * np.asarray(stack.dz, float) / float(dt))
    cvf = np.broadcast_to(cv[:, None, None], stack.shape).ravel()
    return np.asarray(P_next, float).ravel() + cvf * np.asarray(theta_n, float).ravel()


def capacity_per_cell(stack, dt: float) -> np.ndarray:
    """C V / dt per cell, flat."""
    cap = np.asarray(stack.heat_cap, float)
    cv = cap * float(stack.dx) * float(stack.dy) * np.asarray(stack.dz, float) / float(dt)
    return np.broadcast_to(cv[:, None, None], stack.shape).ravel().copy()


def convective_per_cell(stack) -> np.ndarray:
    """h S per cell (flat): the only path from the grid to ambient."""
    s = np.zeros(stack.shape)
    s[stack.nz - 1] += float(stack.h_top) * float(stack.dx) * float(stack.dy)
    s[0] += float(stack.h_bottom) * float(stack.dx) * float(stack.dy)
    return s.ravel()


# ---------------------------------------------------------------------------
# FP16 storage of the lateral conductances (Section 4.2, the third copy of the
# Quad-Diag diagonals kept in half precision; Algorithm "Physics-Aware FP32/16
# SpMV with AD", where each loaded value is promoted before it is used).
#
# Reading (listed in the design doc): FP16's normal range starts at 2^-14, below
# which small conductances would lose bits, so each layer's lateral values are
# stored scaled by a power of two, 2^e_l with e_l = 14 - ceil(log2(max g in the
# layer)), which puts the largest at or below 2^14 (FP16's largest finite value
# is about 2^16).  The stored value is the FP16 rounding of the FP32 rounding of
# g * 2^e_l (round to nearest even at each step); the operator uses
# stored * 2^-e_l.  Only the in-plane (lateral) conductances are stored this
# way: the out-of-plane ones and the sink are per layer here and are not stored
# per cell at all.

def fp16_exponents(cond: Conductances) -> np.ndarray:
    """Per-layer exponent e_l of the FP16 storage scale (0 for a layer with no
    lateral face)."""
    nz = cond.sink.shape[0]
    e = np.zeros(nz, dtype=np.int64)
    for l in range(nz):
        m = 0.0
        if cond.gx[l].size:
            m = max(m, float(cond.gx[l].max()))
        if cond.gy[l].size:
            m = max(m, float(cond.gy[l].max()))
        if m > 0.0:
            e[l] = 14 - int(np.ceil(np.log2(m)))
    return e


def fp16_lateral(cond: Conductances) -> Conductances:
    """The conductances the FP16-stored operator uses: lateral values rounded
    through FP32 then FP16 at scale 2^e_l and scaled back (exact in FP64);
    vertical faces and sinks unchanged."""
    e = fp16_exponents(cond)
    s = np.ldexp(1.0, e)[:, None, None]

    def rounded(g):
        return np.asarray(g * s, np.float64).astype(np.float32).astype(np.float16).astype(np.float64) / s

    return Conductances(rounded(cond.gx), rounded(cond.gy), cond.gz.copy(), cond.sink.copy())

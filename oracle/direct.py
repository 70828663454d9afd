"""Direct reference solves and exact spectra.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The method of the paper (Chebyshev-preconditioned CG, Section 4.3) converges to
the unique solution of the SPD system of Section 3.2, so the oracle computes that
solution by definition:

* ``solve_dense``     - dense Cholesky (N <= 4096);
* ``solve_splu``      - sparse LU (SuperLU) of the assembled CSR matrix;
* ``solve_separable`` - exact solve for stacks whose conductivity is uniform
  within each layer: a 2-D orthonormal DCT-II diagonalises the lateral Neumann
  Laplacian (eigenvalues 4 sin^2(pi m / 2n)), leaving one nz x nz tridiagonal
  system per lateral mode, solved by the Thomas algorithm.  It never forms the
  CSR matrix, so it checks the assembly as well as the solve.
* ``exact_extremes``  - smallest and largest eigenvalue of A for such stacks,
  from the same separable structure.
"""

from __future__ import annotations

from typing import Optional, Tuple

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def solve_dense(A, b: np.ndarray) -> np.ndarray:
    """Cholesky solve; raises numpy.linalg.LinAlgError if A is not SPD."""
    M = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    if M.shape[0] > 4096:
        raise ValueError("dense oracle is for N <= 4096")
    c = sla.cho_factor(M, lower=True, check_finite=True)
    return sla.cho_solve(c, np.asarray(b, float))


def solve_splu(A, b: np.ndarray) -> np.ndarray:
    return spla.splu(A.tocsc()).solve(np.asarray(b, float))


def _uniform_layer_terms(stack, dt: Optional[float]):
    """Per-layer lateral conductances, vertical couplings and sink (uniform k).

    For a layer of uniform conductivity the two half cells of a lateral face are
    equal, so the series conductance reduces to k * (face area) / (cell pitch).
    """
    if stack.k_lat_mult is not None:
        raise ValueError("separable oracle needs per-layer uniform conductivity")
    dx, dy = float(stack.dx), float(stack.dy)
    dz = np.asarray(stack.dz, float)
    kl = np.asarray(stack.k_lat, float)
    kv = np.asarray(stack.k_vert, float)
    gxl = kl * dy * dz / dx
    gyl = kl * dx * dz / dy
    # vertical coupling: half layer l in series with half layer l+1
    rz = dz[:-1] / (2.0 * kv[:-1]) + dz[1:] / (2.0 * kv[1:])
    gzl = dx * dy / rz
    sink = np.zeros(stack.nz)
    sink[-1] += float(stack.h_top) * dx * dy
    sink[0] += float(stack.h_bottom) * dx * dy
    if dt is not None:
        sink += np.asarray(stack.heat_cap, float) * dx * dy * dz / float(dt)
    return gxl, gyl, gzl, sink


def _neumann_eigs(n: int) -> np.ndarray:
    m = np.arange(n)
    return 4.0 * np.sin(np.pi * m / (2.0 * n)) ** 2


class SeparableFactors:
    """The separable solve of one per-layer-uniform operator (steady, or
    transient with step dt), its per-mode tridiagonal systems eliminated once.

    ``solve_hat`` solves in the DCT basis (the right-hand side and the result as
    DCT-II coefficients over x, y per layer), so a sequence of solves with the
    same operator (backward-Euler steps) can stay in that basis."""

    def __init__(self, stack, dt: Optional[float] = None):
        nz, ny, nx = stack.shape
        self.shape = stack.shape
        gxl, gyl, gzl, sink = _uniform_layer_terms(stack, dt)
        mux = _neumann_eigs(nx)[None, :]
        muy = _neumann_eigs(ny)[:, None]
        # tridiagonal per lateral mode: diag d_l, off-diagonal -gz_l between l, l+1
        d = np.empty((nz, ny, nx))
        for l in range(nz):
            dl = mux * gxl[l] + muy * gyl[l] + sink[l]
            if l > 0:
                dl = dl + gzl[l - 1]
            if l < nz - 1:
                dl = dl + gzl[l]
            d[l] = dl
        # forward elimination of the Thomas algorithm along l (vectorised over
        # modes): multipliers cp and pivots denom
        cp = np.zeros((nz, ny, nx))
        den = np.empty((nz, ny, nx))
        den[0] = d[0]
        if nz > 1:
            cp[0] = -gzl[0] / den[0]
        for l in range(1, nz):
            a = -gzl[l - 1]
            den[l] = d[l] - a * cp[l - 1]
            if l < nz - 1:
                cp[l] = -gzl[l] / den[l]
        self.gzl, self.cp, self.den = gzl, cp, den

    def solve_hat(self, bh: np.ndarray) -> np.ndarray:
        nz = self.shape[0]
        gzl, cp, den = self.gzl, self.cp, self.den
        dp = np.zeros(self.shape)
        dp[0] = bh[0] / den[0]
        for l in range(1, nz):
            a = -gzl[l - 1]
            dp[l] = (bh[l] - a * dp[l - 1]) / den[l]
        x = np.empty(self.shape)
        x[nz - 1] = dp[nz - 1]
        for l in range(nz - 2, -1, -1):
            x[l] = dp[l] - cp[l] * x[l + 1]
        return x


def dct_layers(v: np.ndarray, shape) -> np.ndarray:
    """Orthonormal 2-D DCT-II of every layer of a flat field."""
    return sfft.dctn(np.asarray(v, float).reshape(shape), type=2, axes=(1, 2), norm="ortho")


def idct_layers(vh: np.ndarray) -> np.ndarray:
    """Inverse of ``dct_layers``, flattened."""
    return sfft.idctn(vh, type=2, axes=(1, 2), norm="ortho").ravel()


def solve_separable(stack, b: np.ndarray, dt: Optional[float] = None) -> np.ndarray:
    """Exact solve of A theta = b for a per-layer-uniform stack."""
    f = SeparableFactors(stack, dt)
    return idct_layers(f.solve_hat(dct_layers(b, stack.shape)))


def _z_matrix(gxl, gyl, gzl, sink, mux: float, muy: float) -> np.ndarray:
    nz = len(sink)
    M = np.diag(mux * gxl + muy * gyl + sink)
    for l in range(nz - 1):
        M[l, l] += gzl[l]
        M[l + 1, l + 1] += gzl[l]
        M[l, l + 1] -= gzl[l]
        M[l + 1, l] -= gzl[l]
    return M


def exact_extremes(stack, dt: Optional[float] = None) -> Tuple[float, float]:
    """(lambda_min, lambda_max) of A for a per-layer-uniform stack.

    The lateral terms enter as mu * diag(g) with diag(g) >= 0, so by Weyl's
    inequality the extreme eigenvalues come from the extreme lateral modes.
    """
    gxl, gyl, gzl, sink = _uniform_layer_terms(stack, dt)
    lo = np.linalg.eigvalsh(_z_matrix(gxl, gyl, gzl, sink, 0.0, 0.0))[0]
    mx = _neumann_eigs(stack.nx)[-1]
    my = _neumann_eigs(stack.ny)[-1]
    hi = np.linalg.eigvalsh(_z_matrix(gxl, gyl, gzl, sink, mx, my))[-1]
    return float(lo), float(hi)


def all_eigenvalues(stack, dt: Optional[float] = None) -> np.ndarray:
    """Full spectrum of A for a per-layer-uniform stack (small grids only)."""
    gxl, gyl, gzl, sink = _uniform_layer_terms(stack, dt)
    out = []
    for mx in _neumann_eigs(stack.nx):
        for my in _neumann_eigs(stack.ny):
            out.append(np.linalg.eigvalsh(_z_matrix(gxl, gyl, gzl, sink, mx, my)))
    return np.sort(np.concatenate(out))

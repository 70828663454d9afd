"""Shared helpers of the GPU parity tests (seeded inputs + oracle references)."""

from __future__ import annotations

import numpy as np
import torch

import workloads as w


def dev():
    return torch.device("cuda", 0)


def t64(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device=dev())


def t32(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32).ravel(), device=dev())


def grid_of(stack):
    import paper_2606_17850_amd as cuth
    return cuth.Grid.from_stack(stack, device=dev())


def ragged_stack(nx=70, ny=9, layers=("Si", "BEOL", "bond", "TIM", "Cu"), mult=True, seed=11):
    """A grid that spans several 64x4 tiles with ragged tails in x and y."""
    st = w.Stack(nx, ny, list(layers))
    st.dies = [[l] for l, n in enumerate(layers) if n == "Si"]
    if mult:
        st.k_lat_mult = np.exp(0.3 * np.random.default_rng(seed).standard_normal(st.shape))
    return st


def rise_err(T, ref, t_amb):
    """Rise-relative inf-norm error ||T - T*||_inf / ||T* - T_amb||_inf."""
    T = np.asarray(T, float).ravel()
    ref = np.asarray(ref, float).ravel()
    return float(np.abs(T - ref).max() / np.abs(ref - t_amb).max())


def say(msg: str):
    print(msg, flush=True)


def fp32_cheb_bar(A, r, lmin, lmax, k, ref, jacobi=False):
    """Error bar of an FP32 Chebyshev application against the FP64 oracle's
    ``ref`` (inf-norm).  The scale is the oracle's own spread: the paper's
    listing run with FP32 vectors and the FP32-rounded matrix, against the same
    listing in FP64.  The solver evaluates the polynomial in the two-term form,
    whose rounding errors propagate through a three-term recurrence; on the
    interval its amplification is bounded by Chebyshev polynomials of the
    second kind, which grow at most linearly in the degree.  Hence the bar
    4 max(k, 4) times the spread (floored at one FP32 unit roundoff of the
    scale)."""
    from oracle import krylov
    if jacobi:
        ref32 = krylov.jacobi_chebyshev_precondition(A, r, lmin, lmax, k, dtype=np.float32)
    else:
        A32 = A.astype(np.float32)
        ref32 = krylov.chebyshev_precondition(lambda v: A32 @ v, np.asarray(r, np.float32),
                                              lmin, lmax, k, dtype=np.float32)
    scale = float(np.abs(ref).max())
    spread = max(float(np.abs(ref32.astype(np.float64) - ref).max()), 2.0 ** -24 * scale)
    return 4.0 * max(k, 4) * spread

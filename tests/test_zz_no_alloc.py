"""The allocation-free preconditioner entry point (cuth_precond_apply_noalloc),
called through the C ABI, against cuth_precond_apply on the same inputs.

Both run the same single-sweep kernels on the same operator and constants, so
the results must agree bit for bit.  Calls follow each other on one device (the
scratch array keeps the previous call's contents): a larger grid, then a
smaller one, then the larger one again, in every precision and preconditioner.
A grid whose buffers exceed the scratch is rejected with CUTH_E_INVALID."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import dev, grid_of, ragged_stack, say

pytestmark = pytest.mark.gpu

PRECS = {"fp64": 0, "mixed": 1, "mixed16": 2}
PCS = {"chebyshev": 0, "jacobi": 1, "none": 2, "chebyshev_jacobi": 3}


def _lib():
    from paper_2606_17850_amd import _lib as L
    return L.load()


def _run(lib, fn, g, prec, pc, r, lmin, lmax, k, dt=0.0):
    z = torch.full_like(r, float("nan"))
    torch.cuda.synchronize()
    code = getattr(lib, fn)(g.handle, ctypes.c_double(dt), PRECS[prec], PCS[pc],
                            ctypes.c_double(lmin), ctypes.c_double(lmax), k,
                            ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()))
    assert code == 0, (fn, code, lib.cuth_last_error())
    return z


def _bounds(g, pc, dt):
    if pc in ("chebyshev", "chebyshev_jacobi"):
        b = g.spectral_bounds(dt=dt, preconditioner=pc)
        return b["lmin"], b["lmax"]
    return 1.0, 2.0   # validated, then unused


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("pc", list(PCS))
def test_noalloc_matches_precond_apply(prec, pc):
    lib = _lib()
    big = ragged_stack(nx=200, ny=70, layers=("Si", "BEOL", "bond", "Si", "BEOL", "bond", "TIM", "Cu"),
                       seed=3)
    small = ragged_stack(nx=36, ny=5, layers=("Si", "BEOL", "TIM"), mult=False)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    grids = {"big": grid_of(big), "small": grid_of(small)}
    for name, k, dt in (("big", 30, 0.0), ("small", 7, 0.0), ("big", 12, 1e-4)):
        g = grids[name]
        say(f"noalloc {prec} {pc} {name} k={k} dt={dt}")
        lmin, lmax = _bounds(g, pc, dt)
        r = torch.as_tensor(np.random.default_rng(k).standard_normal(g.n), dtype=dtype, device=dev())
        ref = _run(lib, "cuth_precond_apply", g, prec, pc, r, lmin, lmax, k, dt)
        z = _run(lib, "cuth_precond_apply_noalloc", g, prec, pc, r, lmin, lmax, k, dt)
        assert torch.isfinite(ref).all()
        assert torch.equal(z, ref), float((z - ref).abs().max())
    for g in grids.values():
        g.close()


def test_noalloc_rejects_grids_above_the_scratch():
    """8,388,608 cells: the FP64 iterate alone fills the 64 MiB scratch, so the
    call is rejected before any device work; the FP32 one fits and matches."""
    lib = _lib()
    import workloads as w
    st = w.Stack(2048, 2048, ["Si", "Cu"])
    st.dies = [[0]]
    g = grid_of(st)
    say("noalloc above the scratch: 2048x2048x2")
    r64 = torch.ones(g.n, dtype=torch.float64, device=dev())
    z64 = torch.zeros_like(r64)
    code = lib.cuth_precond_apply_noalloc(g.handle, ctypes.c_double(0.0), PRECS["fp64"], 0,
                                          ctypes.c_double(1e-6), ctypes.c_double(1.0), 30,
                                          ctypes.c_void_p(r64.data_ptr()),
                                          ctypes.c_void_p(z64.data_ptr()))
    assert code == 1
    assert b"scratch" in lib.cuth_last_error()
    torch.cuda.synchronize()
    assert float(z64.abs().max()) == 0.0   # nothing was written
    del r64, z64
    r = torch.as_tensor(np.random.default_rng(1).standard_normal(g.n), dtype=torch.float32,
                        device=dev())
    ref = _run(lib, "cuth_precond_apply", g, "mixed", "chebyshev", r, 1e-6, 1.0, 30)
    z = _run(lib, "cuth_precond_apply_noalloc", g, "mixed", "chebyshev", r, 1e-6, 1.0, 30)
    assert torch.equal(z, ref)
    g.close()

"""Python binding of the MI355X layered-stencil thermal solver (libcuth.so).

Every numeric step runs in the library's HIP kernels; this module only turns
torch tensors into device pointers and stream handles and back.  PyTorch is
used for device memory and streams.

    g = Grid(nx, ny, nz, dx, dy, dz, k_lat, k_vert, h_top=..., t_amb=...)
    T, stats = g.solve(P)                       # steady  G T = P
    T1, stats = g.transient_step(dt, P1, T0)    # (C/dt + G) T1 = P1 + C/dt T0
    dP, dk, stats = g.adjoint(T, dL_dT)         # gradients through one adjoint solve
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import CUTH_FP64, CUTH_MIXED, CUTH_MIXED16, PRECISIONS, STATUS_NAMES

__all__ = ["Grid", "CuthError", "solve_batch", "ThermalSolve", "options", "CUTH_FP64",
           "CUTH_MIXED", "CUTH_MIXED16", "library"]


class CuthError(RuntimeError):
    def __init__(self, status: int, msg: str, stats: Optional[dict] = None):
        super().__init__(f"cuth status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.stats = stats


def library() -> ctypes.CDLL:
    return _lib.load()


def _check(status: int, stats: Optional[_lib.Stats] = None):
    if status != _lib.CUTH_OK:
        msg = library().cuth_last_error().decode(errors="replace")
        raise CuthError(status, msg, stats.as_dict() if stats is not None else None)


def options(precision: str = "mixed", tol: Optional[float] = None, cheb_degree: int = 30,
            lanczos_steps: int = 30, max_inner: int = 2000, max_outer: int = 12,
            use_initial_guess: bool = False, check_period: int = 0,
            preconditioner: str = "chebyshev", storage: str = "stencil") -> _lib.Options:
    o = _lib.Options()
    library().cuth_default_options(ctypes.byref(o))
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, got {precision!r}")
    o.precision = PRECISIONS[precision]
    o.tol = 0.0 if tol is None else float(tol)
    o.cheb_degree = _lib.CUTH_DEGREE_AUTO if cheb_degree == "auto" else int(cheb_degree)
    o.lanczos_steps = lanczos_steps
    o.max_inner = max_inner
    o.max_outer = max_outer
    o.use_initial_guess = 1 if use_initial_guess else 0
    o.check_period = check_period
    if preconditioner not in _lib.PRECONDITIONERS:
        raise ValueError(f"preconditioner must be one of {sorted(_lib.PRECONDITIONERS)}, "
                         f"got {preconditioner!r}")
    o.preconditioner = _lib.PRECONDITIONERS[preconditioner]
    if storage not in _lib.STORAGES:
        raise ValueError(f"storage must be one of {sorted(_lib.STORAGES)}, got {storage!r}")
    o.storage = _lib.STORAGES[storage]
    return o


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, n: int, name: str, device) -> int:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must live on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t.data_ptr()


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _darr(x, nz: int, name: str):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (nz,)))
    return a


class Grid:
    """One layered grid on one device (see cuth_grid_desc in include/cuth.h)."""

    def __init__(self, nx: int, ny: int, nz: int, dx: float, dy: float, dz, k_lat, k_vert,
                 k_lat_mult: Optional[torch.Tensor] = None, heat_cap=None,
                 h_top: float = 0.0, h_bottom: float = 0.0, t_amb: float = 0.0,
                 device=None):
        lib = library()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.t_amb = float(t_amb)
        self._dz = _darr(dz, nz, "dz")
        self._kl = _darr(k_lat, nz, "k_lat")
        self._kv = _darr(k_vert, nz, "k_vert")
        self._cap = None if heat_cap is None else _darr(heat_cap, nz, "heat_cap")
        mult_ptr = _ptr(k_lat_mult, torch.float64, self.n, "k_lat_mult", self.device)
        # kept for set_conductivity (the library does not hold the field)
        self._mult = k_lat_mult
        d = _lib.GridDesc()
        d.nx, d.ny, d.nz = self.nx, self.ny, self.nz
        d.dx, d.dy = float(dx), float(dy)
        dp = lambda a: a.ctypes.data_as(_lib.c_double_p) if a is not None else None
        d.dz, d.k_lat, d.k_vert = dp(self._dz), dp(self._kl), dp(self._kv)
        d.k_lat_mult = mult_ptr
        d.heat_cap = dp(self._cap)
        d.h_top, d.h_bottom, d.t_amb = float(h_top), float(h_bottom), float(t_amb)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.cuth_grid_create(ctypes.byref(d), _stream_handle(self.device), ctypes.byref(h)))
        self._h = h

    def set_conductivity(self, k_lat, k_vert, k_lat_mult: Optional[torch.Tensor] = None):
        """New layer conductivities in place (cuth_grid_set_conductivity): the
        handle keeps its buffers; the next solve reruns the Lanczos setup.  A
        per-cell grid takes k_lat_mult, else reuses the field it was built
        with (or last given here)."""
        kl = _darr(k_lat, self.nz, "k_lat")
        kv = _darr(k_vert, self.nz, "k_vert")
        mult = k_lat_mult if k_lat_mult is not None else self._mult
        mult_ptr = _ptr(mult, torch.float64, self.n, "k_lat_mult", self.device)
        with torch.cuda.device(self.device):
            _check(library().cuth_grid_set_conductivity(
                self._h, kl.ctypes.data_as(_lib.c_double_p), kv.ctypes.data_as(_lib.c_double_p),
                mult_ptr))
        self._kl, self._kv, self._mult = kl, kv, mult

    @classmethod
    def from_stack(cls, stack, device=None) -> "Grid":
        """Build from a workloads.Stack-like object (attributes of the descriptor)."""
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        mult = None
        if getattr(stack, "k_lat_mult", None) is not None:
            mult = torch.as_tensor(np.ascontiguousarray(stack.k_lat_mult, dtype=np.float64).ravel(),
                                   device=dev)
        return cls(stack.nx, stack.ny, stack.nz, stack.dx, stack.dy, stack.dz, stack.k_lat,
                   stack.k_vert, k_lat_mult=mult, heat_cap=stack.heat_cap, h_top=stack.h_top,
                   h_bottom=stack.h_bottom, t_amb=stack.t_amb, device=dev)

    def close(self):
        if getattr(self, "_h", None):
            library().cuth_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def _vec(self, t, name, dtype=torch.float64):
        return _ptr(t, dtype, self.n, name, self.device)

    def _new(self, dtype=torch.float64):
        return torch.empty(self.n, dtype=dtype, device=self.device)

    # ------------------------------------------------------------ solves
    def solve(self, P: torch.Tensor, T: Optional[torch.Tensor] = None, opts=None, **kw):
        """Steady solve; returns (T, stats dict)."""
        o = opts if opts is not None else options(**kw)
        if T is None:
            T = self._new()
        st = _lib.Stats()
        with torch.cuda.device(self.device):
            s = library().cuth_solve(self._h, self._vec(P, "P"), self._vec(T, "T"), ctypes.byref(o),
                                     ctypes.byref(st))
        _check(s, st)
        return T, st.as_dict()

    def transient_step(self, dt: float, P_next: torch.Tensor, T_n: torch.Tensor,
                       T_next: Optional[torch.Tensor] = None, opts=None, **kw):
        o = opts if opts is not None else options(**kw)
        if T_next is None:
            T_next = self._new()
        st = _lib.Stats()
        with torch.cuda.device(self.device):
            s = library().cuth_transient_step(self._h, float(dt), self._vec(P_next, "P_next"),
                                              self._vec(T_n, "T_n"), self._vec(T_next, "T_next"),
                                              ctypes.byref(o), ctypes.byref(st))
        _check(s, st)
        return T_next, st.as_dict()

    def adjoint(self, T: torch.Tensor, dL_dT: torch.Tensor, opts=None, **kw):
        """Returns (dL/dP [N], dL/dk [nz] per layer conductivity, stats)."""
        o = opts if opts is not None else options(**kw)
        dP = self._new()
        dk = torch.empty(self.nz, dtype=torch.float64, device=self.device)
        st = _lib.Stats()
        with torch.cuda.device(self.device):
            s = library().cuth_adjoint(self._h, self._vec(T, "T"), self._vec(dL_dT, "dL_dT"),
                                       dP.data_ptr(), dk.data_ptr(), ctypes.byref(o),
                                       ctypes.byref(st))
        _check(s, st)
        return dP, dk, st.as_dict()

    # ------------------------------------------------------ step-level calls
    def apply(self, x: torch.Tensor, dt: float = 0.0, fp16_coef: bool = False) -> torch.Tensor:
        """y = A x (float64: FP64 operator, float32: FP32 operator; fp16_coef:
        the FP32 operator with the FP16-stored lateral conductances)."""
        prec = CUTH_FP64 if x.dtype == torch.float64 else (CUTH_MIXED16 if fp16_coef else CUTH_MIXED)
        y = self._new(x.dtype)
        with torch.cuda.device(self.device):
            _check(library().cuth_apply(self._h, float(dt), prec, self._vec(x, "x", x.dtype),
                                        y.data_ptr()))
        return y

    def residual(self, b: torch.Tensor, T: torch.Tensor, dt: float = 0.0) -> torch.Tensor:
        r = self._new()
        with torch.cuda.device(self.device):
            _check(library().cuth_residual(self._h, float(dt), self._vec(b, "b"), self._vec(T, "T"),
                                           r.data_ptr()))
        return r

    def apply_csr(self, x: torch.Tensor, dt: float = 0.0) -> torch.Tensor:
        """y = A x through the CSR copy of the FP64 operator (Ablation I baseline)."""
        y = self._new(torch.float64)
        with torch.cuda.device(self.device):
            _check(library().cuth_apply_csr(self._h, float(dt), self._vec(x, "x"), self._vec(y, "y")))
        return y

    def precond_apply(self, r: torch.Tensor, lmin: float, lmax: float, degree: int,
                      dt: float = 0.0, fp16_coef: bool = False,
                      preconditioner: str = "chebyshev") -> torch.Tensor:
        prec = CUTH_FP64 if r.dtype == torch.float64 else (CUTH_MIXED16 if fp16_coef else CUTH_MIXED)
        pc = _lib.PRECONDITIONERS[preconditioner]
        z = self._new(r.dtype)
        with torch.cuda.device(self.device):
            _check(library().cuth_precond_apply(self._h, float(dt), prec, pc, float(lmin),
                                                float(lmax), int(degree),
                                                self._vec(r, "r", r.dtype), z.data_ptr()))
        return z

    def precond_apply_noalloc(self, r: torch.Tensor, z: torch.Tensor, lmin: float, lmax: float,
                              degree: int, dt: float = 0.0, fp16_coef: bool = False,
                              preconditioner: str = "chebyshev") -> torch.Tensor:
        """As precond_apply, into the caller's z, through the entry point that
        allocates no device memory."""
        prec = CUTH_FP64 if r.dtype == torch.float64 else (CUTH_MIXED16 if fp16_coef else CUTH_MIXED)
        pc = _lib.PRECONDITIONERS[preconditioner]
        with torch.cuda.device(self.device):
            _check(library().cuth_precond_apply_noalloc(
                self._h, float(dt), prec, pc, float(lmin), float(lmax), int(degree),
                self._vec(r, "r", r.dtype), self._vec(z, "z", r.dtype)))
        return z

    def reset_bounds(self):
        _check(library().cuth_grid_reset_bounds(self._h))

    def profile_enable(self, on: bool = True):
        _check(library().cuth_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        ms, cnt, by, fu = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32()
        _check(library().cuth_profile_read(self._h, ctypes.byref(ms), ctypes.byref(cnt),
                                           ctypes.byref(by), ctypes.byref(fu)))
        # fused: sweeps per timed launch minus one (2 triples, 1 pairs, 0 single)
        return {"total_ms": ms.value, "launches": cnt.value, "bytes_per_launch": by.value,
                "fused": fu.value}

    def spectral_bounds(self, dt: float = 0.0, steps: int = 30,
                        v0: Optional[torch.Tensor] = None,
                        preconditioner: str = "chebyshev") -> dict:
        a = (ctypes.c_double * steps)()
        b = (ctypes.c_double * max(steps - 1, 1))()
        vals = [ctypes.c_double() for _ in range(4)]
        with torch.cuda.device(self.device):
            _check(library().cuth_spectral_bounds(
                self._h, float(dt), _lib.PRECONDITIONERS[preconditioner], int(steps),
                self._vec(v0, "v0", torch.float32) if v0 is not None else None,
                a, b, *[ctypes.byref(v) for v in vals]))
        return {"alpha": np.array(a[:]), "beta": np.array(b[: steps - 1]),
                "ritz_min": vals[0].value, "ritz_max": vals[1].value,
                "lmin": vals[2].value, "lmax": vals[3].value}


def solve_batch(grids: Sequence[Grid], P: Sequence[torch.Tensor], T: Optional[Sequence] = None,
                nrhs: int = 1, opts=None, **kw):
    """Solve len(grids) systems with nrhs right-hand sides each (P[s]: [nrhs*N_s])."""
    o = opts if opts is not None else options(**kw)
    ns = len(grids)
    if T is None:
        T = [torch.empty(nrhs * g.n, dtype=torch.float64, device=g.device) for g in grids]
    for s, g in enumerate(grids):
        _ptr(P[s], torch.float64, nrhs * g.n, f"P[{s}]", g.device)
        _ptr(T[s], torch.float64, nrhs * g.n, f"T[{s}]", g.device)
    hs = (ctypes.c_void_p * ns)(*[g.handle.value for g in grids])
    ps = (ctypes.c_void_p * ns)(*[p.data_ptr() for p in P])
    ts = (ctypes.c_void_p * ns)(*[t.data_ptr() for t in T])
    stats = (_lib.Stats * (ns * nrhs))()
    with torch.cuda.device(grids[0].device if ns else None):
        s = library().cuth_solve_batch(ns, hs, nrhs, ps, ts, ctypes.byref(o), stats)
    _check(s)
    return T, [st.as_dict() for st in stats]


class ThermalSolve(torch.autograd.Function):
    """T = solve(P, k) with gradients by one adjoint solve.

    forward(P, k, grid, opts): k is a [nz] tensor of layer conductivities, each
    setting both the lateral and the vertical conductivity of its layer (the
    lateral multiplier field, if any, stays fixed).  grid is a Grid, whose
    conductivities are set to k in place (set_conductivity: no new buffers,
    so a loop over k reuses one handle), or a callable that returns a Grid
    built with k.  backward returns the library's dL/dP and its per-layer
    dL/dk unchanged.
    """

    @staticmethod
    def forward(ctx, P, k, grid, opts=None):
        kh = k.detach().cpu().numpy()
        if isinstance(grid, Grid):
            g = grid
            g.set_conductivity(kh, kh)
        else:
            g = grid(kh)
        T, _ = g.solve(P.contiguous(), opts=opts)
        ctx.k = kh
        ctx.grid = g
        ctx.opts = opts
        ctx.k_device = k.device
        ctx.save_for_backward(T)
        return T

    @staticmethod
    def backward(ctx, gT):
        (T,) = ctx.saved_tensors
        g = ctx.grid
        # a later forward on the same Grid may have set other conductivities
        if not (np.array_equal(g._kl, ctx.k) and np.array_equal(g._kv, ctx.k)):
            g.set_conductivity(ctx.k, ctx.k)
        dP, dk, _ = g.adjoint(T, gT.contiguous(), opts=ctx.opts)
        return dP, dk.to(ctx.k_device), None, None

"""ctypes declarations of the C ABI in include/cuth.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcuth.so")

CUTH_OK = 0
CUTH_E_INVALID = 1
CUTH_E_NOMEM = 2
CUTH_E_DEVICE = 3
CUTH_E_NOT_CONVERGED = 4
CUTH_E_BREAKDOWN = 5
CUTH_FP64 = 0
CUTH_MIXED = 1
CUTH_MIXED16 = 2
CUTH_ADAPTIVE = 3
CUTH_FP32 = 4
CUTH_DEGREE_AUTO = -1
PRECISIONS = {"fp64": CUTH_FP64, "mixed": CUTH_MIXED, "mixed16": CUTH_MIXED16,
              "adaptive": CUTH_ADAPTIVE, "fp32": CUTH_FP32}
PRECONDITIONERS = {"chebyshev": 0, "jacobi": 1, "none": 2, "chebyshev_jacobi": 3}
STORAGES = {"stencil": 0, "csr": 1}

STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "NOT_CONVERGED", 5: "BREAKDOWN"}

EXPORTED = (
    "cuth_default_options", "cuth_grid_create", "cuth_grid_destroy",
    "cuth_grid_set_conductivity", "cuth_solve",
    "cuth_transient_step", "cuth_solve_batch", "cuth_adjoint", "cuth_last_error",
    "cuth_apply", "cuth_apply_csr", "cuth_residual", "cuth_precond_apply",
    "cuth_precond_apply_noalloc", "cuth_spectral_bounds",
    "cuth_grid_reset_bounds", "cuth_profile_enable", "cuth_profile_read",
)

c_double_p = ctypes.POINTER(ctypes.c_double)


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("dz", c_double_p), ("k_lat", c_double_p), ("k_vert", c_double_p),
        ("k_lat_mult", ctypes.c_void_p), ("heat_cap", c_double_p),
        ("h_top", ctypes.c_double), ("h_bottom", ctypes.c_double), ("t_amb", ctypes.c_double),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
        ("cheb_degree", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
        ("max_inner", ctypes.c_int32), ("max_outer", ctypes.c_int32),
        ("use_initial_guess", ctypes.c_int32), ("check_period", ctypes.c_int32),
        ("preconditioner", ctypes.c_int32), ("storage", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer_cycles", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
        ("stencil_applies", ctypes.c_int64), ("stop_reason", ctypes.c_int32),
        ("cheb_degree", ctypes.c_int32), ("drift_stops", ctypes.c_int32),
        ("stagnation_stops", ctypes.c_int32), ("rel_residual", ctypes.c_double),
        ("err_est", ctypes.c_double), ("setup_ms", ctypes.c_double),
        ("solve_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
        ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("_")}


_lib = None


def load() -> ctypes.CDLL:
    """Load libcuth.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2606_17850_amd.build` "
            "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "cuth_default_options": (None, [ctypes.POINTER(Options)]),
        "cuth_grid_create": (ctypes.c_int, [ctypes.POINTER(GridDesc), vp, ctypes.POINTER(vp)]),
        "cuth_grid_destroy": (None, [vp]),
        "cuth_grid_set_conductivity": (ctypes.c_int, [vp, c_double_p, c_double_p, vp]),
        "cuth_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(Options), ctypes.POINTER(Stats)]),
        "cuth_transient_step": (ctypes.c_int, [vp, dbl, vp, vp, vp, ctypes.POINTER(Options),
                                               ctypes.POINTER(Stats)]),
        "cuth_solve_batch": (ctypes.c_int, [i32, ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                            ctypes.POINTER(vp), ctypes.POINTER(Options),
                                            ctypes.POINTER(Stats)]),
        "cuth_adjoint": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.POINTER(Options),
                                        ctypes.POINTER(Stats)]),
        "cuth_last_error": (ctypes.c_char_p, []),
        "cuth_apply": (ctypes.c_int, [vp, dbl, i32, vp, vp]),
        "cuth_residual": (ctypes.c_int, [vp, dbl, vp, vp, vp]),
        "cuth_apply_csr": (ctypes.c_int, [vp, dbl, vp, vp]),
        "cuth_precond_apply": (ctypes.c_int, [vp, dbl, i32, i32, dbl, dbl, i32, vp, vp]),
        "cuth_precond_apply_noalloc": (ctypes.c_int, [vp, dbl, i32, i32, dbl, dbl, i32, vp, vp]),
        "cuth_spectral_bounds": (ctypes.c_int, [vp, dbl, i32, i32, vp, c_double_p, c_double_p,
                                                c_double_p, c_double_p, c_double_p, c_double_p]),
        "cuth_grid_reset_bounds": (ctypes.c_int, [vp]),
        "cuth_profile_enable": (ctypes.c_int, [vp, i32]),
        "cuth_profile_read": (ctypes.c_int, [vp, c_double_p, ctypes.POINTER(ctypes.c_int64),
                                             c_double_p, ctypes.POINTER(ctypes.c_int32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib

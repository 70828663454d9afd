"""ctypes wrapper and build step for the C oracle CG (``cpu_cg.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_cg.c")
_LIB = os.path.join(_HERE, "liboracle_cg.so")
_lib: Optional[ctypes.CDLL] = None


def build() -> str:
    """Compile the oracle CG with gcc -O3 -fopenmp (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_jacobi_cg.restype = ctypes.c_int
        lib.oracle_jacobi_cg.argtypes = [
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following solves."""
    _load().oracle_set_threads(int(n))


def jacobi_cg(A, b: np.ndarray, x0: Optional[np.ndarray] = None, rtol: float = 1e-14,
              maxit: int = 200000) -> Tuple[np.ndarray, int, float]:
    """Solve A x = b (A CSR, SPD).  Returns (x, iterations, true relative residual)."""
    lib = _load()
    ip = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(A.indices, dtype=np.int32)
    a = np.ascontiguousarray(A.data, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.shape[0]) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    st = lib.oracle_jacobi_cg(A.shape[0], ip.ctypes.data, ix.ctypes.data, a.ctypes.data,
                              bb.ctypes.data, x.ctypes.data, rtol, maxit,
                              ctypes.byref(it), ctypes.byref(rr))
    if st == 3:
        raise ValueError("oracle CG: bad input")
    if st == 2:
        raise FloatingPointError("oracle CG: breakdown (p^T A p <= 0)")
    return x, int(it.value), float(rr.value)

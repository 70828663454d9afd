"""Write sampled oracle values for full-size parity tests (calls only oracle/ and workloads/).

Usage: python tests/golden/make_reference.py [c1]

c1: the 512 x 512 x 16 steady system with lognormal lateral conductivity.  The
oracle's FP64 Jacobi-CG is run to relative residual 1e-14 and, as evidence of
convergence, once more to 1e-13; the file stores the rise theta* at 4096 seeded
cells plus the cell of the maximum rise, the maximum rise itself, and the
difference between the two oracle runs.
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle import assembly, cpu_cg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c1():
    st, P = w.config1()
    A = assembly.assemble(st)
    b = assembly.rhs_steady(P)
    t0 = time.time()
    x14, it14, rr14 = cpu_cg.jacobi_cg(A, b, rtol=1e-14, maxit=200000)
    t14 = time.time() - t0
    x13, it13, rr13 = cpu_cg.jacobi_cg(A, b, rtol=1e-13, maxit=200000)
    rise = float(np.abs(x14).max())
    rng = np.random.default_rng(np.random.SeedSequence([2606, 17850, 1, 0, 0, 3]))
    cells = np.sort(rng.choice(st.n, size=4096, replace=False))
    cells = np.unique(np.append(cells, int(np.argmax(np.abs(x14)))))
    out = {
        "_about": "Oracle (FP64 CSR Jacobi-CG) rise theta* = T* - T_amb of the 512x512x16 "
                  "config-1 steady system at seeded cells; written by tests/golden/make_reference.py",
        "n": st.n,
        "t_amb": st.t_amb,
        "max_rise": rise,
        "argmax": int(np.argmax(np.abs(x14))),
        "oracle": {"rtol": 1e-14, "iterations": it14, "true_relres": rr14, "seconds": t14,
                   "threads": cpu_cg.threads()},
        "convergence_check": {"rtol": 1e-13, "iterations": it13, "true_relres": rr13,
                              "max_rise_rel_diff": float(np.abs(x13 - x14).max() / rise)},
        "power_total_W": float(np.sum(P)),
        "cells": cells.tolist(),
        "theta": [float(v) for v in x14[cells]],
    }
    with open(os.path.join(HERE, "c1_oracle_samples.json"), "w") as f:
        json.dump(out, f)
    print({k: v for k, v in out.items() if k not in ("cells", "theta")})


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c1"
    {"c1": c1}[which]()

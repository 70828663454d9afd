"""Build the gfx950 shared library ``libcuth.so`` in-tree with hipcc.

Run as ``python -m paper_2606_17850_amd.build``.  Always recompiles.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcuth.so")
ARCH = os.environ.get("CUTH_OFFLOAD_ARCH", "gfx950")

# Device code: no packed-FP32 instructions (build flags).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the library needs ROCm to build")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="cuth_build_") as tmp:
        objs = []
        jobs = []
        for src, is_dev in (("kernels.hip", True), ("solver.cpp", False), ("api.cpp", False)):
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc] + COMMON + [f"--offload-arch={ARCH}"] + DEVICE_FLAGS
            if is_dev:
                cmd += ["-x", "hip"]
            cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
            jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
            objs.append(obj)
        fail = None
        for p in jobs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if verbose or p.returncode != 0:
                sys.stderr.write(text)
            if p.returncode != 0:
                fail = p.args
        if fail:
            raise RuntimeError(f"hipcc failed: {' '.join(fail)}")
        tmp_lib = LIB + ".tmp"
        link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib] + objs
        subprocess.run(link, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

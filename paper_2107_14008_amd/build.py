"""Build libpmfmm.so (HIP kernels for gfx950 + host planner + C ABI) in-tree.

Usage: python -m paper_2107_14008_amd.build   (or build() from Python)

Every HIP source is compiled with packed-FP32 instruction selection turned
off (``-Xclang -target-feature -Xclang -packed-fp32-ops``); the host planner
is compiled without floating-point contraction so that its geometry tests
are exactly the float64 operations they are written as.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpmfmm.so")
ARCH = os.environ.get("PMFMM_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{ROOT}/include", f"-I{CSRC}"]
HIP = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
       "-Xclang", "-packed-fp32-ops", "-ffp-contract=fast-honor-pragmas"]
HOST = ["-ffp-contract=off"]

SOURCES = [
    ("plan.cpp", "gxx"),
    ("abi.cpp", "hip-host"),
    ("p2p.hip", "hip"),
    ("far.hip", "hip"),
    ("adjoint.hip", "hip"),
    ("gpu_sort.hip", "hip"),
    ("gpu_plan.hip", "hip"),
    ("pm.hip", "hip"),
    ("step.hip", "hip"),
    ("peak.hip", "hip"),
]


def _cmd(src, kind, obj):
    path = os.path.join(CSRC, src)
    if kind == "gxx":
        return ["g++", *COMMON, *HOST, "-c", path, "-o", obj]
    if kind == "hip-host":
        return [HIPCC, *COMMON, *HOST, f"--offload-arch={ARCH}",
                "--offload-host-only", "-c", path, "-o", obj]
    return [HIPCC, *COMMON, *HIP, "-c", path, "-o", obj]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    todo = []
    for src, kind in SOURCES:
        if not os.path.exists(os.path.join(CSRC, src)):
            continue
        obj = os.path.join(BUILD, src + ".o")
        todo.append((_cmd(src, kind, obj), obj))
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(lambda t: _run(t[0], verbose), todo))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp,
          *[o for _, o in todo], "-L/opt/rocm/lib", "-lhipfft", "-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libmpk.so (host planner + C ABI + gfx950 kernels) in the package dir.

    python -m paper_2405_12525_amd.build          # build (always recompiles)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmpk.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
              f"-I{INC}", f"-I{CSRC}", f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__"]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{INC}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} ... ({r.returncode})")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    objs = []
    for src in ("planner.cpp", "capi.cpp"):
        o = os.path.join(OUT_DIR, src.replace(".cpp", ".o"))
        _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    for src in ("kernels.hip", "gpu_plan.hip"):
        o = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        _run([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lgomp",
          f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

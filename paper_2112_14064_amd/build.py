"""Build libriga.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: python -m paper_2112_14064_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libriga.so")

SOURCES = ["plan.cpp", "sweep_plan.cpp", "small_eig.cpp", "ks_host.cpp", "api.cpp", "toar.cpp", "hcurl.cpp", "k_assemble.hip", "k_factor.hip", "k_solve.hip",
           "k_krylov.hip", "k_toar.hip", "k_cshift.hip", "k_batch.hip", "batch.cpp", "noalloc.hip", "gep.cpp"]

ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libriga.so")


# host-only sources: plain complex multiplication (no IEEE inf/nan recovery
# calls) for the small projected eigenproblem, whose entries are finite and
# well scaled
HOST_FLAGS = ["-fcx-limited-range",
              # AVX2 + FMA (every x86 server CPU that hosts this GPU has them):
              # the dense Schur reduction of the projected matrix vectorises
              "-march=x86-64-v3"]


def _compile(src: str, hipcc: str, out_dir: str, defines: list) -> str:
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    extra = HOST_FLAGS if src.endswith(".cpp") else []
    cmd = [hipcc, *FLAGS, *extra, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, lib: str = LIB, out_dir: str = OUT_DIR, defines=()) -> str:
    """Compile every source for gfx950 and link `lib` (default: the in-tree
    libriga.so); `defines` are extra -D options (tile and launch-shape
    constants); returns the library path."""
    os.makedirs(out_dir, exist_ok=True)
    hipcc = _hipcc()
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc, out_dir, list(defines)), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

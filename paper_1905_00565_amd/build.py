"""Build libccm.so for gfx950 with hipcc (in-tree, so it travels with the repo).

    python -m paper_1905_00565_amd.build

Every HIP translation unit is compiled with contraction off (the binary32
distance arithmetic is fixed term by term) and with packed FP32 instructions
disabled.  Objects go to ``_build/`` at the repository root; the shared
library lands next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIBRARY = os.path.join(PKG, "libccm.so")

ARCH = os.environ.get("CCM_OFFLOAD_ARCH", "gfx950")
SOURCES = ["ccm_kernels.hip", "ccm_sort.hip", "ccm_noalloc.hip", "ccm_plan.cpp",
           "ccm_runtime.cpp", "ccm_server.cpp"]
# ccm_inst.hip is compiled once per embedding dimension (its kernels are the
# bulk of the build, so the ten compile in parallel).
INST_SOURCE = "ccm_inst.hip"
INST_E = tuple(range(1, 11))
# The causal-matrix kernels, also once per E, without machine-level
# loop-invariant hoisting (the unit's header says why).
MULTI_SOURCE = "ccm_inst_multi.hip"
MULTI_FLAGS = ("-mllvm", "-disable-machine-licm")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
                 shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def common_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]


def units(defines=()):
    """(source, object, extra flags) of every translation unit; ``defines``
    go to the units that hold kernels (the tuner's shape tables)."""
    out = []
    for src in SOURCES:
        extra = list(defines) if src == "ccm_kernels.hip" else []
        out.append((src, os.path.join(BUILD, os.path.splitext(src)[0] + ".o"), extra))
    for e in INST_E:
        out.append((INST_SOURCE, os.path.join(BUILD, f"ccm_inst_e{e}.o"),
                    [f"-DCCM_INST_E={e}", *defines]))
        out.append((MULTI_SOURCE, os.path.join(BUILD, f"ccm_inst_multi_e{e}.o"),
                    [f"-DCCM_INST_E={e}", *MULTI_FLAGS, *defines]))
    return out


def compile_unit(src: str, obj: str, extra=()) -> str:
    cmd = [hipcc(), *common_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {src} {' '.join(extra)}")
    return obj


def jobs() -> int:
    return max(1, min(16, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))


def build_library(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # the per-E units first, largest E first, so the long compiles start at once
    todo = units()
    todo = todo[len(SOURCES):][::-1] + todo[:len(SOURCES)]
    with ThreadPoolExecutor(max_workers=jobs()) as ex:
        objs = list(ex.map(lambda u: compile_unit(*u), todo))
    tmp = LIBRARY + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIBRARY)
    if verbose:
        print(f"built {LIBRARY}")
    return LIBRARY


if __name__ == "__main__":
    build_library(verbose=True)

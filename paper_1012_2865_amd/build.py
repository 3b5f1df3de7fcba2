"""Build libmoray.so (HIP kernels + C ABI runtime) for gfx950 with hipcc.

Usage: python -m paper_1012_2865_amd.build   (or build_library() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmoray.so")

ARCH = os.environ.get("MORAY_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I", CSRC, "-I", INCLUDE,
    # hardware float64 atomic add on coarse-grained memory
    "-munsafe-fp-atomics",
    # keep the compiler from forming packed-fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-pthread",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")


def build_library(out: str = LIB) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in ("moray_kernels.hip", "moray_equilibrium.hip", "moray_runtime.cpp", "moray_serve.cpp", "moray_td.cpp",
                "moray_td_kernels.hip", "moray_noalloc.hip", "moray_tune_cache.cpp"):
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


MICROBENCH_LIB = os.path.join(HERE, "libmoray_microbench.so")


def build_microbench(out: str = MICROBENCH_LIB) -> str:
    """The device-peak microbenchmark (scattered float64 atomics, streaming
    copy) that bench.py prices the trace kernel's rooflines against."""
    tmp = out + ".tmp"
    _run([HIPCC] + COMMON + ["-x", "hip", "-shared", os.path.join(CSRC, "moray_microbench.hip"), "-o", tmp])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library())
    print(build_microbench())

"""Build the HIP library libstokesmg.so in-tree for gfx950.

    python -m paper_1502_04070_amd.build        (or build() from Python)

The stencil header is regenerated from gen_stencils.py first.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstokesmg.so")
SOURCES = ["smg_kernels.hip", "smg_fused.hip", "smg_capi.hip"]
# host-only runtime (no device code): built by the host compiler, the same
# way the sanitizer check program builds it
HOST_SOURCES = ["smg_host.cpp"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# the HIP headers need to know the platform when a plain host compiler reads them
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")]
ARCH = os.environ.get("SMG_OFFLOAD_ARCH", "gfx950")

OBJDIR = os.path.join(HERE, "_build")
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return cand


def cxx() -> str:
    return os.environ.get("CXX") or shutil.which("g++") or "c++"


def build(verbose: bool = False) -> str:
    """Regenerate the stencil header, compile every translation unit in
    parallel (each launches only kernels it defines, so no relocatable device
    code is needed) and link the shared library."""
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_stencils.py"),
                           os.path.join(CSRC, "stencils.inc")], stdout=subprocess.DEVNULL)
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append((src, subprocess.Popen(cmd)))
    for src in HOST_SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".host.o")
        cmd = [cxx(), *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append((src, subprocess.Popen(cmd)))
    failed = [src for src, pr in procs if pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc {' '.join(failed)}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

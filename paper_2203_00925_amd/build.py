"""Build libmifvm.so for gfx950 in-tree (``python -m paper_2203_00925_amd.build``).

The host preprocessing (mesh.cpp) is plain C++17 built by g++; the kernels and
the C ABI are HIP built by hipcc for gfx950 only.  Packed-FP32 instructions
are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_lib")
LIB = os.path.join(OUT_DIR, "libmifvm.so")
ARCH = "gfx950"

HIP_SOURCES = ["api.hip", "nn_api.hip", "fv_kernels.hip", "solve_kernels.hip", "ir_kernels.hip",
               "nn_kernels.hip", "mf_kernels.hip", "gmres_kernels.hip", "streamer_kernels.hip",
               "amg_kernels.hip", "amg_api.hip", "noalloc.hip", "batch_kernels.hip",
               "batch_api.hip"]
CXX_SOURCES = ["mesh.cpp", "amg.cpp"]
HEADERS = ["mesh.h", "state.h", "reduce.h", "seg.h", "cg_scalars.h", "api_util.h", "nn.h", "gmres.h"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + proc.stdout)
    return proc.stdout


def build(verbose: bool = False) -> str:
    """Compile every source (always; no staleness check) and link the library."""
    hipcc = _hipcc()
    obj_dir = os.path.join(PKG, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in CXX_SOURCES:
        o = os.path.join(obj_dir, src + ".o")
        _run(["g++", "-O2", "-g0", "-fPIC", "-std=c++17", "-pthread", "-Wall", "-Wextra", *inc, "-c",
              os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    hipflags = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wall", "-munsafe-fp-atomics"]
    for src in HIP_SOURCES:
        o = os.path.join(obj_dir, src + ".o")
        out = _run([hipcc, *hipflags, *inc, "-c", os.path.join(CSRC, src), "-o", o])
        if verbose and out.strip():
            print(out)
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

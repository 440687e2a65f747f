"""Builds the HIP library libleja.so for gfx950 with hipcc (in-tree).

Usage: python -m paper_2211_08948_amd.build   (or via __graft_entry__.build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libleja.so")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "mlp.hip", "user_kernels.hip", "krylov_kernels.hip", "bandwidth.hip", "leja_lib.hip",
           "leja_points.cpp", "small_expm.cpp"]
HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-result",
    "-fvisibility=hidden",
    # packed FP32 instructions stay off (they are not used by this FP64 code either)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def torch_hip_libdir() -> str:
    """Directory of the HIP runtime that PyTorch loads.  The library links the
    same runtime (same soname), so one process holds one HIP runtime and the
    streams and allocations torch hands over are valid here."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        raise RuntimeError("PyTorch is required to locate its HIP runtime")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so under {d}")
    return d


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [cc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [cc, "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-x", "c++",
                   "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    hipdir = torch_hip_libdir()
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, "-L" + hipdir, "-l:libamdhip64.so",
           "-Wl,-rpath," + hipdir, "-Wl,--no-undefined", "-Wl,--exclude-libs,ALL"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

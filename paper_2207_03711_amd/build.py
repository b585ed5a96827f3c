"""Build libq2c.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2207_03711_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libq2c.so")

SOURCES = ["kernels.hip", "capi.cpp", "compile.cpp", "server.cpp", "optimize.cpp", "dmet.cpp", "hadamard.cpp"]

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def torch_hip_libdir() -> str:
    """Directory of the HIP runtime PyTorch loads.  libq2c links against that
    same runtime so that a process holds one HIP/HSA runtime and PyTorch's
    streams and device memory are valid handles inside the library."""
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        raise RuntimeError("PyTorch (ROCm build) is required to link libq2c")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}")
    return d


def _hip_link_stub(objs, objdir: str, verbose: bool) -> str:
    """Link-time stand-in for the HIP runtime: a stub libamdhip64.so whose
    SONAME is the unversioned name under which PyTorch's runtime is loaded,
    exporting the HIP entry points our objects reference.  libq2c then
    records DT_NEEDED libamdhip64.so, which the rpath resolves to PyTorch's
    runtime at load time; the stub itself is never loaded."""
    syms = set()
    for o in objs:
        out = subprocess.run(["nm", "-u", o], check=True, capture_output=True, text=True).stdout
        for line in out.splitlines():
            name = line.split()[-1]
            if name.startswith(("hip", "__hip")):
                syms.add(name)
    stubdir = os.path.join(objdir, "hipstub")
    os.makedirs(stubdir, exist_ok=True)
    src = os.path.join(stubdir, "stub.c")
    with open(src, "w") as f:
        for name in sorted(syms):
            f.write(f"void {name}(void) {{}}\n")
    lib = os.path.join(stubdir, "libamdhip64.so")
    cmd = ["gcc", "-shared", "-fPIC", src, "-o", lib, "-Wl,-soname,libamdhip64.so"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return stubdir


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc(), *HIP_FLAGS, *lang, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    hipdir = torch_hip_libdir()
    stubdir = _hip_link_stub(objs, objdir, verbose)
    cmd = ["g++", "-shared", "-fPIC", *objs, "-o", tmp, f"-L{stubdir}", "-lamdhip64",
           f"-Wl,-rpath,{hipdir}", "-Wl,--disable-new-dtags", "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

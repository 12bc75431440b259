"""Build the native library ``libbp.so`` for gfx950 with hipcc.

    python -m paper_1401_7494_amd.build        # compile into the package directory

Every source is compiled on every call (this is the "does it build" check);
the result lands next to this file so that it travels with the repository.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbp.so")
SOURCES = ["bp_kernels.hip", "bp_api.cpp", "bp_geometry.cpp", "fdk_kernels.hip", "fdk_api.cpp"]
# The seeded input generator's GPU kernels: a library of their own, not linked into libbp.so.
SYNTH_LIB = os.path.join(HERE, "libbpsynth.so")
SYNTH_SOURCES = ["synth_kernels.hip"]
# Measured roofs (update bandwidth, copy, VALU rates per instruction class): a library of their own.
PROBE_LIB = os.path.join(HERE, "libbpprobe.so")
PROBE_SOURCES = ["probe_kernels.hip"]

ARCH = "gfx950"
# Packed FP32 VALU ops are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    _build_lib(SYNTH_SOURCES, SYNTH_LIB, verbose)
    _build_lib(PROBE_SOURCES, PROBE_LIB, verbose)
    return _build_lib(SOURCES, LIB, verbose)


def _build_lib(sources, lib_path, verbose):
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in sources:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc(), f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS,
               "-I", os.path.join(ROOT, "include"), "-c", path, "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
        objs.append(obj)
    tmp = lib_path + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking {os.path.basename(lib_path)} failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

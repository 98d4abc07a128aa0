"""Build the FOFSE HIP library (libfofse.so) for gfx950, in the package folder.

The library is built with hipcc directly (no torch extension machinery): the
product is a plain C-ABI shared object, loaded by the ctypes binding.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfofse.so")
SOURCES = ["fofse_fwd.hip", "fofse_fwd128.hip", "fofse_group.hip", "fofse_bwd.hip", "fofse_bwd128.hip", "fofse_bwd_group.hip",
           "synth_mfma.hip", "fofse_dct.hip", "fofse_noalloc.hip", "fofse_multi.hip", "fofse_api.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # IEEE mode off: v_max_f64 needs no operand canonicalisation (the
         # kernels carry no NaNs; input checks test exponent bits instead)
         "-mno-amdgpu-ieee", "-fno-honor-nans",
         "-Wno-unused-command-line-argument"]

def _check(res, cmd):
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source for gfx950 (one object each, compiled side by side)
    and link libfofse.so; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj] + list(extra)
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    for cmd, proc in jobs:
        out, err = proc.communicate()
        _check(subprocess.CompletedProcess(cmd, proc.returncode, out, err), cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    _check(subprocess.run(cmd, capture_output=True, text=True), cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Builds liblw.so (HIP for gfx950) in-tree.

    python -m paper_2107_12437_amd.build          # always rebuilds
    python -m paper_2107_12437_amd.build --if-stale

All HIP code is compiled with CODEGEN_FLAGS (below): the packed-FP32 target
feature switched off, machine-level loop-invariant code motion off, and
multiply-add contraction within source expressions only.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblw.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ARCH = os.environ.get("LW_OFFLOAD_ARCH", "gfx950")


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def deps() -> list[str]:
    return sources() + glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(INCLUDE, "*.h"))


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in deps())


# Code-generation flags of every HIP source.
#  - packed FP32 off: the kernels use ordinary scalar FP32/FP64 arithmetic only.
#  - no machine-level loop-invariant code motion: it hoists the 64-bit polynomial
#    and range-reduction constants (SGPR operands of v_fma_f64) out of the kernels'
#    charge and step loops, where they then exceed the SGPR budget and spill into
#    VGPR lanes, and every spill or reload costs a VALU instruction.  Without it the
#    constants are rebuilt by scalar moves next to their use (no VALU cost), the grid
#    kernels drop from 165 to 146 VGPRs (mixed, two times per lane) with no spills,
#    and the grid step runs 4-5 % faster with bit-identical results.
#  - multiply-add contraction only within one source expression (-ffp-contract=on,
#    decided by the front end): with the default cross-statement contraction the
#    back end fuses a product into a sum only where the product has one use, so
#    two instances of one kernel template (say one and two times per lane, where
#    the second shares a product between its times) round differently, and the
#    outputs would depend on the launch shape the tuner picks.
CODEGEN_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-mllvm", "-disable-machine-licm", "-ffp-contract=on"]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not is_stale():
        return LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", *CODEGEN_FLAGS,
           "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
           "-I", INCLUDE, "-x", "hip", *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv, verbose=True))

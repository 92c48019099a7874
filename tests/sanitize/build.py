"""Builds the sanitizer test drivers (test infrastructure, CPU only):

- ``oracle_driver`` and ``oracle_driver_ld``: the oracle (FP64 and extended precision)
  with gcc's AddressSanitizer and UndefinedBehaviorSanitizer;
- ``host_driver``: the HIP library's sources with the same sanitizers on the host
  pass only (each ``-fsanitize=`` follows ``-Xarch_host``; the device code is built as
  usual and is never launched by the driver).

Executables go to ``tests/sanitize/_build/`` and are rebuilt when a source is newer.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
ORACLE_SRC = os.path.join(ROOT, "oracle", "lw_oracle.c")
CSRC = os.path.join(ROOT, "paper_2107_12437_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

SAN = ["address", "undefined"]
GCC_FLAGS = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
             "-Wall", "-Wno-unused-function", *[f"-fsanitize={s}" for s in SAN], "-fno-sanitize-recover=all"]


def _stale(target: str, deps: list[str]) -> bool:
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(d) > t for d in deps)


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def oracle_driver(extended: bool = False) -> str:
    src = os.path.join(HERE, "oracle_driver.c")
    exe = os.path.join(OUT, "oracle_driver_ld" if extended else "oracle_driver")
    if _stale(exe, [src, ORACLE_SRC, __file__]):
        os.makedirs(OUT, exist_ok=True)
        defs = ["-DOR_REAL=long double", "-DOR_LONG"] if extended else []
        subprocess.run(["gcc", *GCC_FLAGS, *defs, "-o", exe + ".tmp", src, "-lm"], check=True)
        os.replace(exe + ".tmp", exe)
    return exe


def host_driver() -> str:
    src = os.path.join(HERE, "host_driver.cpp")
    lib_srcs = sorted(glob.glob(os.path.join(CSRC, "*.cpp")) + glob.glob(os.path.join(CSRC, "*.hip")))
    deps = [src, __file__, *lib_srcs, *glob.glob(os.path.join(CSRC, "*.hpp")), os.path.join(INCLUDE, "lw.h")]
    exe = os.path.join(OUT, "host_driver")
    if _stale(exe, deps):
        os.makedirs(OUT, exist_ok=True)
        host_san = []
        for flag in [*[f"-fsanitize={s}" for s in SAN], "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]:
            host_san += ["-Xarch_host", flag]
        cmd = [_hipcc(), "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               *host_san, "-Wno-unused-command-line-argument", "-I", INCLUDE,
               "-x", "hip", *lib_srcs, "-x", "c++", src, "-o", exe + ".tmp"]
        p = subprocess.run(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed ({p.returncode}):\n{p.stderr[-4000:]}")
        os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    for path in (oracle_driver(False), oracle_driver(True), host_driver()):
        print(path)
    sys.exit(0)

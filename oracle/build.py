"""Builds the oracle's shared libraries (plain C, gcc, no fast-math, no FMA contraction):
the FP64 oracle and the same source in x87 extended precision (long double).

The oracle is test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline load it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lw_oracle.c")
LIB = os.path.join(HERE, "_liblworacle.so")
LIB_EXT = os.path.join(HERE, "_liblworacle_ld.so")
FLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _build_one(path: str, defs: list[str], force: bool) -> str:
    if not force and os.path.exists(path) and os.path.getmtime(path) >= os.path.getmtime(SRC):
        return path
    tmp = path + ".tmp"
    subprocess.run(["gcc", *FLAGS, *defs, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, path)
    return path


def build(force: bool = True, extended: bool = False) -> str:
    """Builds both libraries when stale (or always with force); returns the path of the
    FP64 one, or of the extended-precision one when `extended`."""
    _build_one(LIB, [], force)
    _build_one(LIB_EXT, ["-DOR_REAL=long double", "-DOR_LONG"], force)
    return LIB_EXT if extended else LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))

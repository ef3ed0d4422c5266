"""Compile the oracle's C part (plain gcc, FP64, IEEE: no fast-math, no FMA
contraction) into ``oracle/_cp_law.so``.  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cp_law.c")
LIB = os.path.join(HERE, "_cp_law.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The same source under AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal), for the host-side memory and UB checks of the
    tests; loaded by pointing ``CP_ORACLE_LIB`` at ``out`` in a process that
    preloads the sanitizer runtimes."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

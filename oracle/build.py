"""Compile the C oracles (D2Q8 and D3Q14 steppers) into ``oracle/libphonon_oracle.so``
(gcc, OpenMP, -O2, no fast-math).

Test infrastructure: the product build never links this library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("phonon_oracle.c", "phonon_oracle_d3q14.c")]
LIB = os.path.join(HERE, "libphonon_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-o", tmp] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the FP64 oracle shared library (test infrastructure only).

Plain gcc, -O2, no fast-math (IEEE double semantics), OpenMP over rows.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "tsne_oracle.c"), os.path.join(HERE, "mlp_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [s for s in SRC if os.path.exists(s)]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-fvisibility=hidden", "-Wall", "-Wextra", "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

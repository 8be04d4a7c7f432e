"""Compile libtsne355.so (HIP kernels + C ABI) for gfx950 with hipcc.

The library is built in-tree next to this file. Packed-FP32 VALU
instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["tsne_api.hip", "tsne_affinity.hip", "tsne_iterate.hip", "tsne_mlp.hip", "tsne_pt.hip", "tsne_kde.hip"]
LIB = os.path.join(HERE, "libtsne355.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]


def build(verbose: bool = False, jobs: int = 8) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *[f for f in FLAGS if f != "-shared"], "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    errs = []
    for p, src in zip(procs, SOURCES):
        _, err = p.communicate()
        err = "\n".join(ln for ln in err.splitlines()
                        if "packed-fp32-ops' is not a recognized feature" not in ln)
        if p.returncode != 0:
            errs.append(f"{src}:\n{err}")
        elif err.strip() and verbose:
            print(err, file=sys.stderr)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

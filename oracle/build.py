"""Compile the oracle's C core (test infrastructure) into oracle/_liboracle.so."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "core.c")
    out = os.path.join(_HERE, "_liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

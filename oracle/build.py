"""Compile the oracle's C core (test infrastructure) into oracle/_liboracle.so."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


# AddressSanitizer + UndefinedBehaviorSanitizer build: same arithmetic flags, checks abort the
# process at the first finding.
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    src = os.path.join(_HERE, "core.c")
    out = out or os.path.join(_HERE, "_liboracle_san.so" if sanitize else "_liboracle.so")
    tmp = out + ".tmp"
    opt = SANITIZE_FLAGS if sanitize else ["-O3"]
    cmd = ["gcc", *opt, "-march=x86-64-v3", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

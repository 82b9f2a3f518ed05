"""Build the gfx950 shared library libsarabande_hip.so from csrc/ (hipcc, in-tree)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libsarabande_hip.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("SB_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off (the compiler would otherwise form them from float2 code)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is built as usual): the
# sanitizer build of the host logic (plan creation, tables, layouts) that tests/test_sanitizers.py
# drives on a CPU.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _compile(src: str, objdir: str = OBJ, extra=()) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = ["hipcc", "-x", "hip", *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 6, verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link the shared library (in-tree).  sanitize=True
    builds the host-sanitizer variant into _build_sanitize/ instead (not loaded by the package)."""
    objdir = os.path.join(HERE, "_build_sanitize") if sanitize else OBJ
    out = os.path.join(objdir, "libsarabande_hip.so") if sanitize else OUT
    extra = SANITIZE_FLAGS if sanitize else ()
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, extra), srcs))
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, jobs=int(sys.argv[1]) if len(sys.argv) > 1 else 6)

"""Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the library.

    python -m paper_2603_07387_amd.build_sanitize

Compiles every source under csrc/ for gfx950 with -fsanitize=address,undefined
on the host pass only (the argument validation, planners, sizing rules,
regressor files and checksums; device code is built as usual) and links
libtnsketch_san.so under csrc/_build_san/.  It serves the host-only tests, run
in a process that preloads the compiler's ASan runtime (``runtime()``) and
points the binding at it with TN_SKETCH_LIB.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(CSRC, "_build_san")
LIB = os.path.join(OBJ, "libtnsketch_san.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Each sanitizer flag applies to the host compilation only.
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
CFLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", *SAN,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]


def runtime():
    """Path of the compiler's ASan runtime (it carries the UBSan handlers too)."""
    r = subprocess.run([HIPCC, "--offload-host-only", "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = found[0] if found else ""
    return path


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    r = subprocess.run([HIPCC, *CFLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False, force=False):
    """Build unless the library is newer than every source and header."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    deps = srcs + glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) > max(os.path.getmtime(d) for d in deps):
        return LIB
    with cf.ThreadPoolExecutor(min(len(srcs), 8)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

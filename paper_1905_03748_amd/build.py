"""Build ``libct.so`` (HIP for gfx950) from ``csrc/`` with hipcc, in-tree.

Every source compiles to an object in ``_build/`` (in parallel), then one shared library is linked
next to this file.  Packed-FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libct.so")
ARCH = os.environ.get("CT_OFFLOAD_ARCH", "gfx950")

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"--offload-arch={ARCH}",
          "-I", os.path.join(HERE, "..", "include")]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str, verbose: bool, defines=(), tag="", device_extra=()) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    dflags = [f"-D{d}" for d in defines]
    cmd = [_hipcc(), "-c", src, "-o", obj] + COMMON + dflags
    if src.endswith(".hip"):
        cmd = [_hipcc(), "-x", "hip", "-c", src, "-o", obj] + COMMON + DEVICE_FLAGS + list(device_extra) + dflags
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, defines=(), out: str | None = None, device_extra=()) -> str:
    """Compile and link.  `defines` (NAME=VALUE strings), `device_extra` (additional hipcc flags for
    the HIP sources) and `out` build a variant library for tuning experiments; the default builds
    libct.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    lib = out or LIB
    tag = "" if out is None else "." + os.path.basename(out)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, defines, tag, device_extra), srcs))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build libmbbs.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed FP32
instructions disabled (`-Xclang -target-feature -Xclang -packed-fp32-ops`),
then linked into one shared library next to this file.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbbs.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
UNITS = ["lattice.hip", "dslash.hip", "tile.hip", "ssor.hip", "clover.hip", "blas.hip", "solver.hip", "capi.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]


def source_hash() -> str:
    """SHA-256 over the library's sources and public header (the kernels as
    built): counter summaries record it, so stale ones can be recognised."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(SRC) if f.endswith((".hip", ".h")))
    for f in files:
        with open(os.path.join(SRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(HERE, "..", "include", "mbbs.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def _compile(unit: str) -> str:
    obj = os.path.join(BUILD, unit.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(SRC, unit), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {unit}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), 7)) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

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


# The host-checked build: the address and undefined-behaviour sanitizers on
# the host pass only (device code as in the product build).  It serves the
# CPU tests of the C ABI's host paths (argument checks, sizes, defaults);
# its users preload the sanitizer runtime.  A stamp holds the source hash it
# was built from, so an unchanged tree is not rebuilt.
SAN_BUILD = os.path.join(HERE, "_build_san")
SAN_OUT = os.path.join(SAN_BUILD, "libmbbs_san.so")
SAN_FLAGS = ["-Xarch_host", "-O1", "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _compile(unit: str, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, unit.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(SRC, unit), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {unit}:\n{r.stderr[-6000:]}")
    return obj


def build_sanitized(verbose: bool = False) -> str:
    """Build the host-checked library (SAN_FLAGS) at SAN_OUT, unless it was
    built from the present sources."""
    stamp = SAN_OUT + ".srchash"
    if os.path.exists(SAN_OUT) and os.path.exists(stamp) and open(stamp).read().strip() == source_hash():
        return SAN_OUT
    os.makedirs(SAN_BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), 7)) as ex:
        objs = list(ex.map(lambda u: _compile(u, SAN_BUILD, SAN_FLAGS), UNITS))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", *objs, "-o", SAN_OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    with open(stamp, "w") as f:
        f.write(source_hash() + "\n")
    if verbose:
        print("built", SAN_OUT)
    return SAN_OUT


def sanitizer_runtime() -> str:
    """Path of the address-sanitizer runtime of hipcc's clang (to preload)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


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
    if "--sanitized" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)

"""Build the gfx950 shared library libburgers.so from csrc/*.hip with hipcc (cross-compiles without a GPU).

Each source compiles to an object in parallel, then one link step makes the library.  Flags:
contraction off (every kernel variant of a scheme rounds identically and like a plain scalar evaluation
of the update), packed-FP32 instruction forms disabled.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
ARCH = "gfx950"


def library_path() -> str:
    return os.path.join(PKG, "libburgers.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def sources() -> list:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def compile_flags(extra=()) -> list:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}", *extra]


def compile_command(out: str, extra=()) -> list:
    """One-step command (all sources, one hipcc call)."""
    return [hipcc(), *compile_flags(extra), "-shared", "-o", out, *sources()]


def _compile_one(src: str, extra, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc(), *compile_flags(extra), "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, extra=(), jobs: int = 0) -> str:
    out = library_path()
    tmp = out + ".tmp"
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(lambda s: _compile_one(s, extra, verbose), srcs))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    extra = sys.argv[1:]
    print(build(verbose=True, extra=extra))

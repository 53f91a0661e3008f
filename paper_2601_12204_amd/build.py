"""Build the gfx950 shared library libburgers.so from csrc/*.hip with hipcc (cross-compiles without a GPU).

Flags: contraction off (every kernel variant of a scheme rounds identically and like a plain scalar
evaluation of the update), packed-FP32 instruction forms disabled.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
ARCH = "gfx950"


def library_path() -> str:
    return os.path.join(PKG, "libburgers.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def compile_command(out: str, extra=()) -> list:
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}", *extra, "-o", out, *sources]


def build(verbose: bool = False, extra=()) -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = compile_command(tmp, extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    extra = sys.argv[1:]
    print(build(verbose=True, extra=extra))

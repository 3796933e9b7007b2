"""Build libgdpm.so (HIP, gfx950) in-tree: paper_1107_3355_amd/libgdpm.so."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgdpm.so")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # hardware FP64 atomic add for the dose tallies
    "-munsafe-fp-atomics",
    # no floating-point contraction: the exact energy splits need every product
    # rounded on its own (fused multiply-adds are written out with fmaf)
    "-ffp-contract=off",
    # no packed FP32 instructions (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source and link libgdpm.so; always recompiles."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    for src in ("transport.hip", "gdpm.cpp", "tables.cpp"):
        obj = os.path.join(build_dir, src + ".o")
        cmd = [hipcc()] + HIP_FLAGS + list(extra) + ["-I", os.path.join(ROOT, "include"), "-c",
                                                      os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

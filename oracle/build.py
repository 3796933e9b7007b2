"""Compile the reference CPU transport into oracle/liboracle.so (plain C, gcc)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", tmp, os.path.join(HERE, "oracle.c"), "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

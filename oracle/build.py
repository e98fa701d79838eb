"""Build the FP64 oracle shared library (test infrastructure only).

    python -m oracle.build       # writes oracle/libwdlb_ref.so
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wdlb_ref.c")
LIB = os.path.join(HERE, "libwdlb_ref.so")


def build(verbose: bool = False) -> str:
    """Compile wdlb_ref.c with gcc (FP64, OpenMP).  Always recompiles."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

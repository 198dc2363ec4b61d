"""Build the CPU oracle (test infrastructure) with the host C compiler.

The oracle is compiled as plain C11, -O2, with floating-point contraction off and
no fast-math, so that every expression is evaluated as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csph_oracle.c")
LIB = os.path.join(HERE, "libcsph_oracle.so")

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(cc: str = "gcc", verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [cc, *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> str:
    """Build only if the library is missing or older than its sources."""
    srcs = [SRC, os.path.join(HERE, "csph_oracle.h")]
    if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB) for s in srcs):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

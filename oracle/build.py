"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liblf_oracle.so.

Plain gcc, OpenMP over rays, no fast-math and no floating-point contraction so
that the single-precision ray generation is exactly the IEEE operation
sequence it is defined as.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lf_oracle.c")
LIB = os.path.join(HERE, "liblf_oracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compiles `src` (default: the oracle) into the shared library `out`."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-I", HERE, src, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

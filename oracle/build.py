"""Build the FP64 CPU oracle (test infrastructure) as oracle/libsymoracle.so with gcc.

Plain C, -O2, OpenMP, no SIMD intrinsics. Run by the package build step so that the
checker exists wherever the tests run; building it does not make the product use it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "sym_oracle.c"), os.path.join(HERE, "fat_oracle.c"),
        os.path.join(HERE, "wilson_oracle.c")]
LIB = os.path.join(HERE, "libsymoracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

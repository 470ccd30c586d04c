"""Build the CPU oracle shared library (``oracle/libhsgo.so``) with gcc.

Test infrastructure only: the oracle is the plain, slow reference the GPU library
is checked against.  Built with ``-ffp-contract=off`` so that every multiply-add
the sources do not write as ``fma`` stays two rounded operations.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["hsgo_common.c", "hsgo_f32.c", "hsgo_f64.c"]
LIB = os.path.join(HERE, "libhsgo.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=gnu11", "-Wall", "-Wextra", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

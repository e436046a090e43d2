"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/libfldo.so``.

Plain gcc, ``-O2 -ffp-contract=off`` (every multiply and add rounds on its
own), OpenMP over x-planes inside a colour.  Run as a script or call
``build()``.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libfldo.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "fldo.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

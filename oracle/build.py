"""Compile the FP64 CPU oracle into oracle/liborc.so (test infrastructure only).

Built with gcc, no fast-math and no FMA contraction, so every operation is the
IEEE double operation written in lbm_oracle.c.  OpenMP only splits the node
loops over rows (orc_set_threads); it changes no arithmetic.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lbm_oracle.c")
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
        "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-o", LIB + ".tmp", src, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

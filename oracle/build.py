"""Build the FP64 CPU oracle (test infrastructure only) as liboracle.so, and
its op-counting build as liboracle_ops.so.

The oracle is plain C compiled with gcc, with floating-point contraction
switched off so that every product and sum is rounded as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tk_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    from oracle import opcount   # its op-counting build (same source, counting scalar)
    opcount.build(verbose=verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

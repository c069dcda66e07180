"""Build step for the CPU checker: compiles bp_oracle.c into liboracle.so with gcc.

Plain -O2, no fast-math and no floating-point contraction, so the double arithmetic
is exactly the IEEE operations written in the source.  OpenMP spreads row loops over the
host's cores (OMP_NUM_THREADS); results do not depend on the thread count.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    src = os.path.join(_HERE, "bp_oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())

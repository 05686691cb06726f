"""Build step of the FP64 CPU oracle (test infrastructure only).

Compiles ``sc_oracle.c`` with gcc into ``libsc_oracle.so`` beside it.  Plain ``-O2``, no
``-march`` (the library also runs on the benchmark host), no fast-math, no FMA contraction, so
every floating-point operation is the one written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sc_oracle.c")
LIB = os.path.join(HERE, "libsc_oracle.so")


def build_oracle(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-ffp-contract=off",
        "-fno-fast-math", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))

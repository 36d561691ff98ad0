"""Build the CPU oracle shared library (test infrastructure only).

The oracle is compiled without floating-point contraction so that every
expression is evaluated exactly in the order it is written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gks_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, native: bool = False, out: str = LIB) -> str:
    """Compile gks_oracle.cpp into `out`.  The library the tests load is built
    for the baseline x86-64 instruction set (it also runs on other hosts);
    native=True adds -march=native for timing it on the machine that builds
    it (the CPU baseline).  No floating-point contraction either way, so both
    give identical results."""
    cmd = [
        "g++", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-o", out + ".tmp", SRC,
    ]
    if native:
        cmd.insert(2, "-march=native")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

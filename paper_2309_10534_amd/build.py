"""Build the HIP library libtgks.so for gfx950 (in-tree).

    python -m paper_2309_10534_amd.build [-v] [--resource-usage]
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "tgks_capi.hip")
LIB = os.path.join(PKG, "libtgks.so")
ARCH = os.environ.get("TGKS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
]


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    cmd = ["hipcc"] + FLAGS + ["-o", LIB + ".tmp", SRC]
    if resource_usage:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, resource_usage="--resource-usage" in sys.argv)

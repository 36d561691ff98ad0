"""Build the HIP library libtgks.so for gfx950 (in-tree).

Every translation unit under csrc/ is compiled to an object in parallel, then
linked into one shared library.

    python -m paper_2309_10534_amd.build [-v] [--resource-usage]
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtgks.so")
ARCH = os.environ.get("TGKS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# host-only translation units whose speed does not matter (large template
# instantiations of the operation-counting type): a lighter optimisation
OPT = {"tgks_opcount.hip": "-O1"}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ, os.path.splitext(os.path.basename(src))[0] + ".o")
        flags = [OPT.get(os.path.basename(src), f) if f == "-O3" else f for f in FLAGS]
        cmd = ["hipcc"] + flags + ["-c", "-o", obj, src]
        if resource_usage:
            cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
        jobs.append((cmd, obj))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))

    def run(job):
        cmd, _ = job
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd).returncode

    with ThreadPoolExecutor(workers) as ex:
        codes = list(ex.map(run, jobs))
    if any(codes):
        raise RuntimeError(f"hipcc failed: {[j[0][-1] for j, c in zip(jobs, codes) if c]}")
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for _, o in jobs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, resource_usage="--resource-usage" in sys.argv)

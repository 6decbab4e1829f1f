"""Build libspin.so (gfx950) in-tree with hipcc.

Every HIP translation unit is compiled for gfx950 only, with packed FP32
instructions disabled and no floating-point contraction (the host thresholds
and derived observables are defined by plain IEEE double arithmetic).
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libspin.so")
SOURCES = ["kernels.hip", "batch_kernels.hip", "corr.hip", "spin.hip", "batch.hip", "measure_noalloc.hip", "cluster.hip",
           "equilibrium.hip"]
ARCH = "gfx950"
# The kernels branch on wave-uniform values (per-plane threshold patterns of
# the Blume-Capel groups, separation groups of the correlation sums); left
# unstructured, such regions are plain scalar compare-and-branch trees
# instead of flag-merged ones.
SOURCE_FLAGS = {src: ["-mllvm", "-structurizecfg-skip-uniform-regions"]
                for src in ("kernels.hip", "batch_kernels.hip", "corr.hip", "cluster.hip")}


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmds.append([hipcc(), *flags(), *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the sources compile independently: a few at a time
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for proc in pool.map(lambda c: subprocess.run(c), cmds):
            if proc.returncode != 0:
                raise subprocess.CalledProcessError(proc.returncode, proc.args)
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build librace.so for gfx950 in-tree.

Host schedule code is plain C++17 built with g++ without floating-point
contraction (the schedule is reproduced bit for bit); kernels and the C ABI
are HIP built by hipcc for gfx950.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librace.so")

HOST_SRC = ["schedule.cpp", "layout.cpp", "costmodel.cpp", "gauss_seidel.cpp"]
HIP_SRC = ["race_kernels.hip", "csr_kernels.hip", "mpk_kernels.hip", "mlp_kernels.hip", "bandwidth.hip", "vendor.hip",
           "gs_kernels.hip", "api.hip"]
ARCH = os.environ.get("RACE_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and "ignoring feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    steps = [(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")])
             for src in HOST_SRC]
    steps += [(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")])
              for src in HIP_SRC]
    objs = [cmd[-1] for cmd in steps]
    # the objects are independent: compile them side by side
    jobs = max(1, min(len(steps), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd in steps]:
            f.result()
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lrocsparse"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the gfx950 shared library libbpm.so in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbpm.so")
ARCH = "gfx950"

# Packed FP32 instructions are switched off for every device compile.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Kernel units named *_ilp.hip hold the transform lengths for which the
# instruction-level-parallelism machine scheduler measured faster.
ILP_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every source (the kernel units in parallel) and link
    libbpm.so; returns its path."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    # host plan: strict FP64 evaluation order for the plan constants
    host_obj = os.path.join(objdir, "bpm_host.o")
    jobs.append([hipcc, "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-c",
                 os.path.join(CSRC, "bpm_host.cpp"), "-o", host_obj])
    objs = [host_obj]
    for src in sorted(os.listdir(CSRC)):
        if src.endswith(".hip"):
            obj = os.path.join(objdir, src[:-4] + ".o")
            unit_flags = ILP_FLAGS if src.endswith("_ilp.hip") else []
            jobs.append([hipcc, *DEVICE_FLAGS, *unit_flags, *extra_flags, "-c",
                         os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o",
          tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

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


def _stale(obj: str, src: str) -> bool:
    """True when obj is missing or older than src or any header of the
    library (csrc/*.h and the public include/bpm.h)."""
    if not os.path.exists(obj):
        return True
    deps = [src, os.path.join(HERE, "..", "include", "bpm.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, extra_flags=(), incremental: bool = False) -> str:
    """Compile every source (the kernel units in parallel) and link
    libbpm.so; returns its path.  incremental=True recompiles only the
    sources whose object is older than the source or a header."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    # host plan: strict FP64 evaluation order for the plan constants
    host_obj = os.path.join(objdir, "bpm_host.o")
    host_src = os.path.join(CSRC, "bpm_host.cpp")
    if not incremental or _stale(host_obj, host_src):
        jobs.append([hipcc, "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-c",
                     host_src, "-o", host_obj])
    objs = [host_obj]
    for src in sorted(os.listdir(CSRC)):
        if src.endswith(".hip"):
            obj = os.path.join(objdir, src[:-4] + ".o")
            unit_flags = ILP_FLAGS if src.endswith("_ilp.hip") else []
            if not incremental or _stale(obj, os.path.join(CSRC, src)):
                jobs.append([hipcc, *DEVICE_FLAGS, *unit_flags, *extra_flags, "-c",
                             os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
    workers = max(1, min(max(1, len(jobs)),
                         int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o",
          tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))

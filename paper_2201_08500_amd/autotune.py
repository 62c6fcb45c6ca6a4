"""Schedule autotuner for the z-march.

For each (precision, Nx) it times every transform schedule of the library
(BPM_SCHED_STOCKHAM, _FOURSTEP, _SPLIT) on the device.  It uses a problem
with enough slices to fill every compute unit, and HIP events on the launch
stream.  It keeps the fastest schedule and writes the choices to a JSON
cache:

    {"device": "<name>", "nz": 400,
     "choices": {"fp32s": {"2048": "split", ...}, ...},
     "times_ms": {"fp32s": {"2048": {"stockham": 2.1, ...}}}}

Plan(schedule=None) applies a cached choice from the file named by the
environment variable BPM_SCHEDULE_CACHE or, when that is unset, from the
default cache file ($XDG_CACHE_HOME or ~/.cache, then
bpm_mi355x/schedules.json) if it exists; BPM_SCHEDULE_CACHE set to an empty
string disables the cache.  Without a cache the library's built-in default
(measured the same way) is used.  The cache is not checked against the
device it was measured on.

    python -m paper_2201_08500_amd.autotune              # writes the default cache
    python -m paper_2201_08500_amd.autotune --out schedules.json
"""

from __future__ import annotations

import argparse
import json
import os
from typing import Callable, Dict, Iterable, Optional

SCHEDULES = ("stockham", "fourstep", "split")
PRECISIONS = ("fp32s", "fp32", "fp64")
SIZES = (256, 512, 1024, 2048, 4096)
ENV = "BPM_SCHEDULE_CACHE"

_cache = None
_cache_path = None


def select(times: Dict[str, float]) -> str:
    """Fastest schedule; ties (within 1%) go to the earlier, simpler one."""
    best = None
    for name in SCHEDULES:
        if name not in times:
            continue
        if best is None or times[name] < 0.99 * times[best]:
            best = name
    if best is None:
        raise ValueError("no schedule was timed")
    return best


def time_schedule(prec: str, Nx: int, schedule: str, nz: int, reps: int) -> float:
    """Median milliseconds of one march on the device (synthetic bent-crystal
    slices; enough slices to fill every compute unit)."""
    import numpy as np
    import torch
    import workloads as W
    from . import Plan
    nw = max(256, (1 << 18) // Nx)
    w = W.small(Nx=Nx, Nz=nz, Nomega=nw, seed=Nx)
    p = Plan.from_workload(w, precision=prec, schedule=schedule)
    E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
    u = torch.from_numpy(w.u).cuda()
    ws = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
    a, b = torch.empty_like(E0), torch.empty_like(E0)
    p.deformation_table(u, ws)
    p.march(E0, ws, a, b)
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        p.march(E0, ws, a, b)
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def tune(precisions: Iterable[str] = PRECISIONS, sizes: Iterable[int] = SIZES,
         nz: int = 400, reps: int = 3, out: Optional[str] = None,
         timer: Optional[Callable[[str, int, str, int, int], float]] = None,
         device_name: str = "") -> dict:
    """Time every schedule for every (precision, Nx); return (and write to
    `out`) the cache dictionary."""
    timer = timer or time_schedule
    if not device_name:
        try:
            import torch
            device_name = torch.cuda.get_device_name(0)
        except Exception:      # noqa: BLE001 -- informational only
            device_name = "unknown"
    res = {"device": device_name, "nz": int(nz), "choices": {}, "times_ms": {}}
    for prec in precisions:
        res["choices"][prec] = {}
        res["times_ms"][prec] = {}
        for Nx in sizes:
            t = {s: timer(prec, int(Nx), s, int(nz), int(reps)) for s in SCHEDULES}
            res["times_ms"][prec][str(Nx)] = t
            res["choices"][prec][str(Nx)] = select(t)
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
    return res


def default_cache_path() -> str:
    """$XDG_CACHE_HOME (or ~/.cache)/bpm_mi355x/schedules.json."""
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "bpm_mi355x", "schedules.json")


def cache_path() -> Optional[str]:
    """The cache file in effect: BPM_SCHEDULE_CACHE when set (empty: none),
    else the default cache file when it exists, else None."""
    path = os.environ.get(ENV)
    if path is not None:
        return path or None
    path = default_cache_path()
    return path if os.path.exists(path) else None


def cached_choice(prec: str, Nx: int) -> Optional[str]:
    """Schedule chosen by the cache in effect (cache_path), or None."""
    global _cache, _cache_path
    path = cache_path()
    if not path:
        return None
    if _cache is None or _cache_path != path:
        with open(path) as f:
            _cache = json.load(f)
        _cache_path = path
    choice = _cache.get("choices", {}).get(prec, {}).get(str(int(Nx)))
    if choice is not None and choice not in SCHEDULES:
        raise ValueError(f"{path}: unknown schedule {choice!r}")
    return choice


def main():
    ap = argparse.ArgumentParser(description="time the march schedules")
    ap.add_argument("--out", default=None,
                    help="cache file to write (default: the default cache file)")
    ap.add_argument("--precisions", default=",".join(PRECISIONS))
    ap.add_argument("--sizes", default=",".join(str(s) for s in SIZES))
    ap.add_argument("--nz", type=int, default=400)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    out = a.out or default_cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    res = tune(a.precisions.split(","), [int(s) for s in a.sizes.split(",")],
               a.nz, a.reps, out)
    print(json.dumps(res["choices"]))


if __name__ == "__main__":
    main()

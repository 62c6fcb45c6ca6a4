#!/usr/bin/env python3
"""Throughput of the FFT beam-propagation z-march on one MI355X.

Workload: the time-dependent bent crystal -- Nx = 2048 transverse points,
Nz = 4000 steps of 0.5 um, Nomega = 256 frequency slices of a 10 fs pulse,
u = x^2 / (2R), R = 10 m (seeded synthetic inputs, workloads.c2_bent_crystal).
One benchmark step is one pass of the whole hot path: the deformation
pre-pass (exp(i h u) table) plus the march of all slices, inputs resident in
HBM.  Metric: cell-updates/s = Nx * Nz * Nomega / step time.

--workload thermal-bump runs the same measurement on the 4096 x 8192 x 1024
thermal-bump configuration; batch, serve and extensions time the batched
launch, the served request stream and the march's extensions.

Prints one JSON line.  The oracle (CPU, FP64 numpy) is timed on a bounded
sample of slices on the host's cores as a reported baseline.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("cell-updates/s (Nx·Nz·Nω) fp32 vs fp64 at relL2≤1e-5; "
          "p50/p99 request latency")
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X vector peaks (published)
HBM_PEAK_GBS = 8000.0


def flops_per_cell_update(Nx: int) -> float:
    """Algorithmic flops of one (x, z-step, slice) update: four complex FFTs
    (two envelopes, forward and inverse) at 5 N log2 N each, two complex
    propagator multiplies (6 each) and the deformed coupling (six complex
    multiplies and two complex adds)."""
    return 4 * 5 * math.log2(Nx) + 2 * 6 + (6 * 6 + 2 * 2)


def lds_bytes_per_cell_update(Nx: int, storage_bytes: int) -> float:
    """LDS bytes per cell-update of the default (envelope-split four-step)
    schedule at Nx = 1024/2048: per envelope and z-step, two work-group
    exchanges and four wavefront-local Stockham exchanges of the 512-point
    inner transform, each sample written and read once per exchange."""
    accesses = 2 + 4 + 4 + 2   # fwd exchange, 2x2 local fwd, 2x2 local inv, inv exchange
    return 2 * accesses * storage_bytes


def kernel_source_sha256() -> str:
    """sha256 over the sources that define the kernels (csrc/bpm_device.h,
    bpm_internal.h and the kernel units march_*.hip, sorted by name): the key
    under which hardware-counter records are valid.  Host-side dispatch
    (bpm_march.hip, bpm_host.cpp) is not part of it."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2201_08500_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith(".h") or (name.startswith("march_") and name.endswith(".hip")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str):
    """HBM bytes per march launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record (scaled by the reference copy), or None when that
    record is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"march_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_source_sha256() or rec.get("precision") != precision:
        return None
    return float(rec["traffic_bytes_per_launch"])


def _cpu_worker(args):
    slices, seed, barrier_t0 = args
    import numpy as np
    import oracle as O
    import workloads as W
    w = W.c2_bent_crystal(seed=seed).subset(slices)
    p = O.Problem.from_workload(w)
    while time.time() < barrier_t0:   # common start after every worker's setup
        time.sleep(0.001)
    t0 = time.time()
    O.march(p, w.E0_in, w.u)
    t1 = time.time()
    return w.cell_updates, t0, t1


def cpu_baseline(slices_per_core: int = 12, cores: int | None = None) -> dict:
    """Time the oracle, unmodified, on the host: `cores` processes, each
    marching `slices_per_core` slices of the workload through all Nz steps
    with one FFT thread."""
    import multiprocessing as mp
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    ncpu = os.cpu_count() or 1
    cores = min(cores or ncpu, 16, ncpu)
    start = time.time() + 15.0 + 0.5 * cores   # leaves time for input setup
    jobs = [([(c * slices_per_core + i) % 256 for i in range(slices_per_core)], 2,
             start) for c in range(cores)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    cells = sum(r[0] for r in res)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": cells / wall, "unit": "cell-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} processes x {slices_per_core} slices x 4000 steps "
                      f"x 2048 points of the bent-crystal workload "
                      f"({cells:.3e} cell-updates, {wall:.1f} s wall, {model})"}


def run_variant(w, prec, steps, warmup, E0_np, u_t):
    import numpy as np
    import torch
    from paper_2201_08500_amd import Plan
    plan = Plan.from_workload(w, precision=prec)
    E0 = torch.from_numpy(E0_np).to(plan.field_dtype).cuda()
    a = torch.empty_like(E0)
    b = torch.empty_like(E0)
    ws = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.deformation_table(u_t, ws, stream)
        if ev is not None:
            ev[1].record(stream)
        plan.march(E0, ws, a, b, stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)]
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    march_ms = [e[1].elapsed_time(e[2]) for e in evs]
    deform_ms = [e[0].elapsed_time(e[1]) for e in evs]
    out = (a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128))
    return dict(total_s=t1 - t0, march_ms=float(np.mean(march_ms)),
                deform_ms=float(np.mean(deform_ms)), out=out)


def bench_batch(args):
    """Uneven batch: 512 problems (seeded sizes: Nx 256..4096, Nz 500..8000,
    Nomega 1..256), one prepared batch captured in a hipGraph and replayed.
    Reports cell-updates/s of the replay and of running the same jobs one
    after another on the stream."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_08500_amd import Batch, Job, Plan

    torch.cuda.set_device(0)
    specs = W.c4_problem_specs(args.batch_problems, seed=4)
    jobs = []
    cells = 0
    for s in specs:
        w = W.c4_problem(s, with_u=False)
        row, gz, gx, amp = w.meta["u_factors"]
        p = Plan.from_workload(w, precision=args.headline)
        E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
        # same operation order as the numpy generator: row + (amp gz) gx
        u = torch.outer(torch.from_numpy(amp * gz).cuda(), torch.from_numpy(gx).cuda())
        u.add_(torch.from_numpy(row).cuda())
        jobs.append(Job(p, E0, u))
        cells += w.cell_updates
    print(f"[bench] batch: {len(jobs)} problems, {cells:.3e} cell-updates",
          file=sys.stderr, flush=True)
    t_prep = time.perf_counter()
    batch = Batch(jobs)
    t_prep = time.perf_counter() - t_prep
    batch.launch()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            batch.launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    seq = None
    if args.batch_compare:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        outs = [(torch.empty_like(j.E0_out), torch.empty_like(j.Eh_out)) for j in jobs]
        e0.record()
        for j, (oa, ob) in zip(jobs, outs):
            j.plan.propagate(j.E0_in, j.u, oa, ob, workspace=j.workspace)
        e1.record()
        torch.cuda.synchronize()
        seq = e0.elapsed_time(e1) / 1e3
        same = all(torch.equal(oa, j.E0_out) and torch.equal(ob, j.Eh_out)
                   for j, (oa, ob) in zip(jobs, outs))
        del outs
    t = float(np.median(times))
    line = {
        "metric": METRIC, "value": cells / t, "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32s": "f64", "fp32": "f32", "fp64": "f64"}[args.headline],
        "data": "synthetic",
        "config": {"workload": f"uneven-batch-{len(jobs)}-problems",
                   "precision": args.headline, "cell_updates": cells,
                   "graph": "one hipGraph replay per step"},
        "batch": dict(batch.info(), prepare_s=t_prep,
                      replay_s=[float(x) for x in times],
                      sequential_s=seq,
                      sequential_cell_updates_per_s=(cells / seq) if seq else None,
                      sequential_bitwise_equal=(same if seq else None)),
    }
    print(json.dumps(line))


def bench_extensions(args):
    """The extensions of the march on the bent-crystal workload, each timed
    against the plain first-order march of the same precision: 2nd- and
    4th-order splitting, a shaped crystal mask, a march in segments, and the
    pulse pipeline (time -> frequency, march, frequency -> time).  Accuracy of
    each against the fp64 GPU run of the same configuration (all slices)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_08500_amd import Plan
    from workloads.metrics import rel_l2

    torch.cuda.set_device(0)
    w = W.c2_bent_crystal()
    u = torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    cells = w.cell_updates
    prec = args.headline
    x = (np.arange(w.Nx) - w.Nx // 2) * w.dx
    z = np.arange(w.Nz) * w.dz
    # tilted entrance surface (asymmetric cut) x >= -40 um + 0.05 z
    mask = x[None, :] >= (-40e-6 + 0.05 * z)[:, None]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def both(a, b):
        return np.concatenate([a.cpu().numpy().ravel(), b.cpu().numpy().ravel()]).astype(np.complex128)

    def march_case(precision, **kw):
        p = Plan.from_workload(w, precision=precision, **kw)
        E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
        a, b = torch.empty_like(E0), torch.empty_like(E0)
        ws = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
        p.deformation_table(u, ws)
        ms = timed(lambda: p.march(E0, ws, a, b), args.steps)
        return p, E0, ws, a, b, ms

    out = {}
    _, _, _, a, b, base_ms = march_case(prec)
    out["first_order"] = {"march_ms": base_ms, "cell_updates_per_s": cells / (base_ms * 1e-3)}
    for name, kw in [("order2", dict(split_order=2)), ("order4", dict(split_order=4)),
                     ("mask", dict(mask=mask))]:
        print(f"[bench] extensions: {name}", file=sys.stderr, flush=True)
        _, _, _, a, b, ms = march_case(prec, **kw)
        _, _, _, ra, rb, _ = march_case("fp64", **kw)
        out[name] = {"march_ms": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                     "relative_to_first_order": ms / base_ms,
                     "rel_l2_vs_fp64_gpu": float(rel_l2(both(a, b), both(ra, rb)))}
    # segments: 8 x 500 steps chained through their outputs
    print("[bench] extensions: segments", file=sys.stderr, flush=True)
    p, E0, ws, a, b, _ = march_case(prec)
    sa, sb = torch.empty_like(E0), torch.empty_like(E0)
    seg = w.Nz // 8

    def segmented():
        p.march_segment(E0, None, ws, 0, seg, sa, sb)
        for k in range(1, 8):
            p.march_segment(sa, sb, ws, k * seg, seg, sa, sb)
    ms = timed(segmented, args.steps)
    p.march(E0, ws, a, b)
    torch.cuda.synchronize()
    out["segments8"] = {"march_ms": ms, "relative_to_first_order": ms / base_ms,
                        "rel_l2_vs_monolithic": float(rel_l2(both(sa, sb), both(a, b)))}
    # pulse: the slices on a DFT grid spanning +-5 Darwin widths
    print("[bench] extensions: pulse", file=sys.stderr, flush=True)
    eps = W.darwin_relative_width(w.chih, w.chihbar, w.theta_B)
    omega0 = 2 * math.pi * 299792458.0 / w.lam
    dt = 2 * math.pi / (10 * eps * omega0)
    pp = Plan(w.Nx, w.dx, w.dz, w.Nz, w.chi0, w.chih, w.chihbar, w.theta_B, w.lam,
              w.Nomega, precision=prec, time_step=dt)
    f = W.pulse_field(w.Nx, w.dx, w.Nomega, dt, w.lam, w.theta_B, w.theta_B, 40 * dt)
    ft = torch.from_numpy(f).to(pp.field_dtype).cuda()
    ew = torch.empty_like(ft)
    t_ms = timed(lambda: pp.to_frequency(ft, out=ew), args.steps)
    back = pp.to_time(pp.to_frequency(ft))
    torch.cuda.synchronize()
    pa, pb = pp.propagate_pulse(ft, u)
    torch.cuda.synchronize()
    tot = timed(lambda: pp.propagate_pulse(ft, u), max(2, args.steps // 2))
    out["pulse"] = {"transform_ms": t_ms, "pipeline_ms": tot,
                    "pipeline_cell_updates_per_s": cells / (tot * 1e-3),
                    "round_trip_rel_l2": float(rel_l2(back.cpu().numpy().astype(np.complex128), f)),
                    "dt_fs": dt * 1e15}
    line = {
        "metric": METRIC, "value": out["first_order"]["cell_updates_per_s"],
        "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": base_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32s": "f64", "fp32": "f32", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": w.name + "-extensions", "precision": prec},
        "extensions": out,
    }
    print(json.dumps(line))


def bench_serve(args):
    """Served request stream: Poisson arrivals (seeded), sizes as the uneven
    batch, half fp64 and half fp32-storage requests, admission by an HBM
    footprint budget, continuous batching over in-flight slots.  Reports
    p50/p99 latency (arrival to outputs ready) and cell-updates/s."""
    import queue
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_08500_amd.serve import GpuBackend, Request, Server

    torch.cuda.set_device(0)
    trace = W.c5_request_trace(rate=args.serve_rate, duration=args.serve_duration,
                               seed=5)
    prec_map = {"fp64": "fp64", "fp32": args.serve_fp32}
    if args.serve_all_fp64:
        prec_map = {"fp64": "fp64", "fp32": "fp64"}
    # 16 GiB of the device stay outside torch's allocator for the HIP runtime
    backend = GpuBackend(streams=args.serve_streams, keep_outputs=False,
                         headroom_bytes=16 * 2**30)
    srv = Server(backend, budget_bytes=args.serve_budget_gb * 1e9,
                 max_in_flight=args.serve_streams)
    # warm the kernels once outside the measured stream
    for prec in set(prec_map.values()):
        w0 = W.small(Nx=256, Nz=4, Nomega=1)
        srv.backend.materialize(Request(spec=w0, precision=prec))
    torch.cuda.synchronize()
    srv.start()
    pool = ThreadPoolExecutor(max_workers=6)
    futs = [pool.submit(W.c4_problem, spec, False) for _, spec, _ in trace[:64]]
    nxt = 64
    t0 = time.perf_counter()
    submitted = []
    last_note = t0
    for i, (t_arr, spec, prec) in enumerate(trace):
        w = futs[i].result()
        futs[i] = None
        if nxt < len(trace):
            futs.append(pool.submit(W.c4_problem, trace[nxt][1], False))
            nxt += 1
        delay = t0 + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        r = Request(spec=w, precision=prec_map[prec])
        srv.submit(r)
        submitted.append(r)
        if time.perf_counter() - last_note > 10:
            last_note = time.perf_counter()
            print(f"[bench] serve: {i + 1}/{len(trace)} submitted, "
                  f"{len(srv.completed)} done", file=sys.stderr, flush=True)
    lag = time.perf_counter() - t0 - trace[-1][0]
    last, t_last = -1, time.perf_counter()
    while not srv.drain(timeout=10):
        n = len(srv.completed)
        print(f"[bench] serve: draining, {n} done", file=sys.stderr, flush=True)
        if n != last:
            last, t_last = n, time.perf_counter()
        elif time.perf_counter() - t_last > 120:
            srv.stop()
            sys.exit("serve: no request completed for 120 s")
    srv.stop()
    if srv.broken is not None:
        sys.exit(f"serve: device error, {len(srv.failed)} requests failed: {srv.broken}")
    pool.shutdown()
    st = srv.stats()
    line = {
        "metric": METRIC, "value": st["cell_updates_per_s"], "unit": "cell-updates/s",
        "n_gpus": 1, "steps": len(trace), "warmup": 0,
        "ms_per_step": st["p50_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed f64" if not args.serve_all_fp64 else "f64",
        "data": "synthetic",
        "config": {"workload": f"served-stream-{args.serve_rate:g}rps-{args.serve_duration:g}s",
                   "precisions": sorted(set(prec_map.values())),
                   "budget_GB": args.serve_budget_gb, "streams": args.serve_streams},
        "serve": dict(st, requests=len(trace), submit_lag_s=lag,
                      materialize_parts_s=backend.timing,
                      allocator={k: torch.cuda.memory_stats().get(k) for k in (
                          "num_alloc_retries", "num_device_alloc", "num_device_free",
                          "num_sync_all_streams")},
                      offered_cell_updates_per_s=sum(
                          s["Nx"] * s["Nz"] * s["Nomega"] for _, s, _ in trace)
                      / args.serve_duration),
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--headline", default="fp32s",
                    choices=["fp32s", "fp32", "fp64"])
    ap.add_argument("--variants", default="fp32s,fp32,fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices-per-core", type=int, default=96)
    ap.add_argument("--workload", default="bent-crystal",
                    choices=["bent-crystal", "thermal-bump", "batch", "serve",
                             "extensions"])
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-duration", type=float, default=60.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-streams", type=int, default=2,
                    help="launch streams = launches in flight (torch caches freed "
                         "blocks per stream, so more streams split the cache)")
    ap.add_argument("--serve-fp32", default="fp32s", choices=["fp32s", "fp32"],
                    help="precision used for the stream's FP32 requests")
    ap.add_argument("--serve-all-fp64", action="store_true",
                    help="run every request of the same trace in fp64")
    ap.add_argument("--batch-problems", type=int, default=512)
    ap.add_argument("--batch-compare", action="store_true",
                    help="also time the same jobs run one after another")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size, the "
                         "reference kernel for scaling HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the "
              "march shards over frequency slices with no exchange, so N GPUs "
              "would each run this same single-GPU launch on Nomega/N slices.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "extensions":
        bench_extensions(args)
        return

    import numpy as np
    import torch
    import workloads as W
    from workloads.metrics import report

    torch.cuda.set_device(0)
    if args.workload == "thermal-bump":
        # 4096 x 8192 x 1024: the largest configuration, a precision check
        w = W.c3_thermal_bump()
    else:
        w = W.c2_bent_crystal()
    u_t = torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    cells = w.cell_updates
    variants = [v for v in args.variants.split(",") if v]
    if args.headline not in variants:
        variants.insert(0, args.headline)

    if args.copy_probe_mib:
        # reference device copy of known size for scaling HBM byte counters;
        # a 1 GiB fill in between evicts the source from the 256 MB MALL
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush

    results = {}
    for prec in variants:
        print(f"[bench] {prec}: warmup {args.warmup}, timing {args.steps} steps",
              file=sys.stderr, flush=True)
        results[prec] = run_variant(w, prec, args.steps, args.warmup, w.E0_in, u_t)

    # precision report: every variant against the FP64 GPU run on all slices
    # (parity with the oracle is established by the GPU tests)
    prec_report = {}
    for prec, r in results.items():
        a, b = r["out"]
        entry = {}
        if prec != "fp64" and "fp64" in results:
            entry["vs_fp64_gpu_all_slices"] = report(a, b, *results["fp64"]["out"])
        march_s = r["march_ms"] / 1e3
        entry.update(cell_updates_per_s=cells * args.steps / r["total_s"],
                     march_ms=r["march_ms"], deform_ms=r["deform_ms"],
                     march_cell_updates_per_s=cells / march_s)
        prec_report[prec] = entry

    head = results[args.headline]
    dtype = {"fp32s": "f64", "fp32": "f32", "fp64": "f64"}[args.headline]
    storage = 8 if args.headline in ("fp32s", "fp32") else 16
    F = flops_per_cell_update(w.Nx)
    achieved = F * cells / (head["march_ms"] / 1e3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    lds_b = lds_bytes_per_cell_update(w.Nx, storage)
    line = {
        "metric": METRIC,
        "value": cells * args.steps / head["total_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["total_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "Nx": w.Nx, "Nz": w.Nz,
                   "Nomega": w.Nomega, "precision": args.headline,
                   "storage": "complex64" if storage == 8 else "complex128"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(w.name, args.headline),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
                     "kernel": "march", "flops_per_cell_update": F,
                     "march_ms": head["march_ms"],
                     "lds_bytes_per_cell_update": lds_b,
                     "lds_TBps": lds_b * cells / (head["march_ms"] / 1e3) / 1e12},
        "precision_variants": prec_report,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on host cores)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.cpu_slices_per_core)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

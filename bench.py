#!/usr/bin/env python3
"""Throughput of the FFT beam-propagation z-march on one MI355X.

Default workload: the time-dependent crystal with a thermal bump, the
largest configuration -- Nx = 4096 transverse points, Nz = 8192 steps of
0.5 um, Nomega = 1024 frequency slices of a 10 fs pulse, u = Gaussian bump
(1e-10 m, sigma 100 um) plus seeded white-noise strain of rms 1e-7 (seeded
synthetic inputs, workloads.c3_thermal_bump).  One benchmark step is one
pass of the whole hot path: the deformation pre-pass (exp(i h u) table) plus
the march of all slices, inputs resident in HBM.  Metric: cell-updates/s =
Nx * Nz * Nomega / step time, for the FP32-storage/FP64-arithmetic headline
mode, with the FP32-butterfly and FP64 modes and their errors against the
FP64 GPU run beside it.

The same JSON line carries the served request stream (Poisson arrivals,
mixed sizes, half fp64 requests) at 200 req/s (above what one GPU
delivers: the latencies are queueing) and at 150 req/s (below it): p50/p99
latency and cell-updates/s, and the 200 req/s trace served all in fp64.

--workload bent-crystal runs the march measurement on the 2048 x 4000 x 256
bent crystal; batch, serve and extensions time the batched launch, the
served request stream alone and the march's extensions.

The oracle (CPU, FP64 numpy) is timed on a bounded sample of slices on the
host's cores as a reported baseline.
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
    (two envelopes, forward and inverse) at 5 N log2 N each, 2 x 6 for the
    two propagator multiplies and 28 for the 2 x 2 coupling: 20 log2 Nx + 40
    (240, 260, 280 at Nx = 1024, 2048, 4096).  The deformation phase factors
    of the deformed coupling (two more complex multiplies, 12 flops) are
    not counted."""
    return 4 * 5 * math.log2(Nx) + 2 * 6 + 28


def lds_bytes_per_cell_update(Nx: int, storage_bytes: int) -> float:
    """LDS bytes per cell-update of the default schedule at Nx = 1024, 2048
    and 4096 (envelope-split four-step, four-step): per envelope and z-step,
    two work-group exchanges and four wavefront-local Stockham exchanges of
    the 512-point inner transform, each sample written and read once per
    exchange."""
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


# Host cores one GPU's job may use on the measurement machines (the box's
# CPU share per GPU); the oracle baseline runs one process per core up to it.
HOST_CORE_SHARE = 16


def _cpu_worker(args):
    workload, slices, barrier_t0 = args
    import oracle as O
    import workloads as W
    w = W.by_name(workload).subset(slices)
    p = O.Problem.from_workload(w)
    while time.time() < barrier_t0:   # common start after every worker's setup
        time.sleep(0.001)
    t0 = time.time()
    O.march(p, w.E0_in, w.u)
    t1 = time.time()
    return w.cell_updates, t0, t1


def cpu_baseline(workload, slices_per_core: int, total_cells: int) -> dict:
    """Time the oracle, unmodified, on the host: one process per available
    core (at most the per-GPU share), each marching `slices_per_core` seeded
    slices of the workload through all Nz steps with one FFT thread.  The
    rate is measured on that sample; the time the whole workload would take
    at it is an extrapolation and labelled so."""
    import multiprocessing as mp
    import numpy as np
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    ncpu = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = ncpu
    cores = max(1, min(avail, HOST_CORE_SHARE))
    w_nomega = W_NOMEGA[workload]
    pick = np.random.default_rng(11).permutation(w_nomega)
    start = time.time() + 20.0 + 0.5 * cores   # leaves time for input setup
    jobs = [(workload, sorted(int(pick[(c * slices_per_core + i) % w_nomega])
                              for i in range(slices_per_core)), start)
            for c in range(cores)]
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
    rate = cells / wall
    return {"value": rate, "unit": "cell-updates/s", "cores": cores,
            "kind": "oracle",
            "host_cpu_count": ncpu, "host_cores_available": avail,
            "cpu_model": model,
            "extrapolated_full_workload_s": total_cells / rate,
            "sample": f"{cores} processes (one per core, the host's per-GPU share "
                      f"of {HOST_CORE_SHARE}; os.cpu_count() = {ncpu}) x "
                      f"{slices_per_core} seeded slices of {workload}, every slice "
                      f"through all steps ({cells:.3e} cell-updates, {wall:.1f} s "
                      f"wall, {model}); the whole workload would take "
                      f"{total_cells / rate:.0f} s at this rate (extrapolated)"}


W_NOMEGA = {"thermal-bump-4096x8192x1024": 1024, "bent-crystal-2048x4000x256": 256,
            "perfect-crystal-1024x2000x1": 1}


def run_variant(w, prec, steps, warmup, E0_np, u_t, schedule=None):
    import numpy as np
    import torch
    from paper_2201_08500_amd import Plan
    plan = Plan.from_workload(w, precision=prec, schedule=schedule)
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


def bench_3d(args):
    """The march on the 3D grid of the paper's finite-element example,
    22 x 4267 x 1842 (the x step of every row a cyclic convolution computed
    with transforms of length L = 9216 = 9 x 1024, direct 22-point DFTs
    along y), --slices-3d frequency slices: one step is the whole march
    (deformation table, 2 Nz + 1 launches), timed with HIP events on the
    stream; the plan's row tables are built once, in the warm-up.  fp64,
    fp32s (the headline) and fp32 run, and the FP32-storage modes are
    compared with the fp64 run over every slice; their parity with the
    oracle on a sampled slice is the GPU tests' job.  Flops: the
    2D-transform count of flops_per_cell_update with Nx Ny points."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_08500_amd import Plan3D
    from workloads.metrics import report

    torch.cuda.set_device(0)
    w = W.heat_bump_3d(Nomega=args.slices_3d)
    u = torch.from_numpy(np.ascontiguousarray(w.u)).cuda()
    cells = w.cell_updates
    out = {}
    fields = {}
    for prec in ("fp64", "fp32s", "fp32"):
        p = Plan3D.from_workload(w, precision=prec)
        E0 = torch.from_numpy(w.E0_in).to(p.field_dtype).cuda()
        a, b = torch.empty_like(E0), torch.empty_like(E0)
        ws = torch.empty(p.workspace_bytes(), dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream()
        for _ in range(max(1, args.warmup)):     # builds the row tables
            p.propagate(E0, u, a, b, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        ts = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            p.propagate(E0, u, a, b, workspace=ws, stream=stream)
            e1.record(stream)
            ts.append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ts]))
        fields[prec] = (a.cpu().numpy().astype(np.complex128),
                        b.cpu().numpy().astype(np.complex128))
        out[prec] = {"march_ms": ms, "cell_updates_per_s": cells * args.steps / wall}
        print(f"[bench] 3d {prec}: {ms:.1f} ms per march", file=sys.stderr, flush=True)
    for prec in ("fp32s", "fp32"):
        out[f"{prec}_vs_fp64"] = report(*fields[prec], *fields["fp64"])
    head = out["fp32s"]
    F = flops_per_cell_update(w.Nx * w.Ny)
    achieved = F * cells / (head["march_ms"] / 1e3) / 1e12
    line = {
        "metric": METRIC, "value": head["cell_updates_per_s"], "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["march_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "Nx": w.Nx, "Ny": w.Ny, "Nz": w.Nz,
                   "Nomega": w.Nomega, "precision": "fp32s", "storage": "complex64",
                   "x_transform": "cyclic convolution, L = 9216"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["f64"],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f64"],
                     "flops_per_cell_update": F, "traffic": None,
                     "kernel": "3D march (row and column kernels)"},
        "variants": out,
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


def run_serve(rate, duration, all_fp64, args) -> dict:
    """Served request stream: Poisson arrivals (seeded), sizes as the uneven
    batch, half fp64 and half fp32-storage requests (all fp64 when
    all_fp64), admission by an HBM footprint budget, continuous batching
    over in-flight slots.  Returns the server's statistics: p50/p99 latency
    (arrival to outputs ready) and cell-updates/s, among others."""
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import workloads as W
    from paper_2201_08500_amd.serve import GpuBackend, Request, Server

    trace = W.c5_request_trace(rate=rate, duration=duration, seed=5)
    prec_map = {"fp64": "fp64", "fp32": args.serve_fp32}
    if all_fp64:
        prec_map = {"fp64": "fp64", "fp32": "fp64"}
    # 16 GiB of the device stay outside torch's allocator for the HIP
    # runtime; results are consumed at completion (not kept on the device)
    backend = GpuBackend(streams=args.serve_streams, keep_outputs=False,
                         headroom_bytes=16 * 2**30)
    srv = Server(backend, budget_bytes=args.serve_budget_gb * 1e9,
                 max_in_flight=args.serve_streams)
    # warm the kernels once outside the measured stream
    for prec in set(prec_map.values()):
        w0 = W.small(Nx=256, Nz=4, Nomega=1)
        r0 = Request(spec=w0, precision=prec)
        srv.backend.materialize(r0)
        srv.backend.launch([r0])
    torch.cuda.synchronize()
    srv.start()
    pool = ThreadPoolExecutor(max_workers=6)
    futs = [pool.submit(W.c4_problem, spec, False) for _, spec, _ in trace[:64]]
    nxt = 64
    t0 = time.perf_counter()
    last_note = t0
    tag = f"serve {rate:g} req/s{' all fp64' if all_fp64 else ''}"
    for i, (t_arr, spec, prec) in enumerate(trace):
        w = futs[i].result()
        futs[i] = None
        if nxt < len(trace):
            futs.append(pool.submit(W.c4_problem, trace[nxt][1], False))
            nxt += 1
        delay = t0 + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        srv.submit(Request(spec=w, precision=prec_map[prec]))
        if time.perf_counter() - last_note > 10:
            last_note = time.perf_counter()
            print(f"[bench] {tag}: {i + 1}/{len(trace)} submitted, "
                  f"{len(srv.completed)} done", file=sys.stderr, flush=True)
    lag = time.perf_counter() - t0 - trace[-1][0]
    last, t_last = -1, time.perf_counter()
    while not srv.drain(timeout=10):
        n = len(srv.completed)
        print(f"[bench] {tag}: draining, {n} done", file=sys.stderr, flush=True)
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
    st.update(rate_per_s=rate, duration_s=duration, requests=len(trace),
              precisions=sorted(set(prec_map.values())), submit_lag_s=lag,
              budget_GB=args.serve_budget_gb, streams=args.serve_streams,
              materialize_parts_s=dict(backend.timing),
              staging_fallbacks=backend.ring.fallbacks if backend.ring else None,
              offered_cell_updates_per_s=sum(
                  s["Nx"] * s["Nz"] * s["Nomega"] for _, s, _ in trace) / duration)
    del srv, backend
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return st


def serve_runs(args) -> dict:
    """The served stream at each rate of --serve-rates (mixed precisions),
    and at each rate of --serve-fp64-rates the same trace all in fp64."""
    out = {}
    for rate in [float(r) for r in args.serve_rates.split(",") if r]:
        print(f"[bench] serve: {rate:g} req/s mixed", file=sys.stderr, flush=True)
        out[f"{rate:g}rps_mixed"] = run_serve(rate, args.serve_duration, False, args)
    for rate in [float(r) for r in args.serve_fp64_rates.split(",") if r]:
        print(f"[bench] serve: {rate:g} req/s all fp64", file=sys.stderr, flush=True)
        out[f"{rate:g}rps_all_fp64"] = run_serve(rate, args.serve_duration, True, args)
    return out


def bench_serve(args):
    """--workload serve: the served streams alone, one JSON line."""
    import torch
    torch.cuda.set_device(0)
    runs = serve_runs(args)
    head = next(iter(runs.values()))
    line = {
        "metric": METRIC, "value": head["cell_updates_per_s"], "unit": "cell-updates/s",
        "n_gpus": 1, "steps": head["requests"], "warmup": 0,
        "ms_per_step": head["p50_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "mixed f64",
        "data": "synthetic",
        "config": {"workload": f"served-stream-{head['rate_per_s']:g}rps-"
                               f"{args.serve_duration:g}s",
                   "budget_GB": args.serve_budget_gb, "streams": args.serve_streams},
        "serve": runs,
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
    ap.add_argument("--schedule", default=None,
                    choices=["auto", "stockham", "fourstep", "split"],
                    help="transform schedule of every variant (default: the "
                         "library's per-size default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices-per-core", type=int, default=None,
                    help="oracle slices per host process (default: 24 of the "
                         "thermal bump, 96 of the bent crystal)")
    ap.add_argument("--workload", default="thermal-bump",
                    choices=["thermal-bump", "bent-crystal", "batch", "serve",
                             "extensions", "3d"])
    ap.add_argument("--slices-3d", type=int, default=16,
                    help="frequency slices of the 3D workload")
    ap.add_argument("--no-serve", action="store_true",
                    help="leave the served stream out of the march measurement")
    ap.add_argument("--serve-rates", default="200,150",
                    help="arrival rates (req/s) of the mixed-precision served runs")
    ap.add_argument("--serve-fp64-rates", default="200",
                    help="arrival rates of the same traces served all in fp64")
    ap.add_argument("--serve-duration", type=float, default=60.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-streams", type=int, default=3,
                    help="launch streams = launches in flight (three: shorter waits "
                         "below capacity than two, p50/p99 at 200 req/s kept)")
    ap.add_argument("--serve-fp32", default="fp32s", choices=["fp32s", "fp32"],
                    help="precision used for the stream's FP32 requests")
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
    if args.workload == "3d":
        bench_3d(args)
        return

    import numpy as np
    import torch
    import workloads as W
    from workloads.metrics import report, within

    torch.cuda.set_device(0)
    if args.workload == "thermal-bump":
        # 4096 x 8192 x 1024: the largest configuration that fits one GPU
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
        results[prec] = run_variant(w, prec, args.steps, args.warmup, w.E0_in, u_t,
                                    args.schedule)

    # precision report: every variant against the FP64 GPU run on all slices
    # (parity with the oracle is established by the GPU tests)
    prec_report = {}
    for prec, r in results.items():
        a, b = r["out"]
        entry = {}
        if prec != "fp64" and "fp64" in results:
            rep_ = report(a, b, *results["fp64"]["out"])
            entry["vs_fp64_gpu_all_slices"] = rep_
            # the target of the precision modes: relL2 <= 1e-5 over the
            # result and per field, phase error <= 1e-4 rad
            entry["meets_relL2_1e-5"] = not within(
                rep_, 1e-5, phase_tol=1e-4, keys=("rel_l2", "rel_l2_E0", "rel_l2_Eh"))
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
                   "schedule": args.schedule or "auto",
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
    del results, u_t
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_serve:
        line["serve"] = serve_runs(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on host cores)", file=sys.stderr, flush=True)
        per_core = args.cpu_slices_per_core or (24 if w.Nx == 4096 else 96)
        line["cpu_baseline"] = cpu_baseline(w.name, per_core, cells)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

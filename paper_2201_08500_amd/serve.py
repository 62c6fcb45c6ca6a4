"""Continuous-batching server for z-march requests.

Requests (one problem each: a plan, its incident field and its displacement)
arrive at any time.  A scheduler thread admits them, in arrival order, as
device memory (an HBM footprint budget) and in-flight slots allow:
- it materialises each admitted request's buffers on the device;
- it packs everything admitted since the last launch into ONE batched
  persistent launch (bpm_propagate_batch) on a stream with no launch in
  flight (StreamSlots);
- it polls completion events, so requests that arrive while others run are
  launched as soon as memory and a slot free up, and their work overlaps
  the running work on the device.

Every slice runs the same code alone or in any mix, so a request's result
does not depend on what it was batched with.  Latency is arrival to outputs
ready (completion event observed).

Outputs stay device-resident.  The bytes a finished request keeps on the
device (backend.retained(), its two output fields when the backend keeps
them) stay charged to the budget until the caller hands them back with
Server.release_outputs(); only the rest of its footprint (inputs,
displacement, workspace) returns to the budget when it completes.  Retained
outputs therefore hold back admission: a caller that never releases them
stalls the queue once they fill the budget, instead of the device running
out of memory outside the budget.

The device side is a backend object, so the scheduling logic is testable on
the CPU with a simulated device; GpuBackend drives libbpm.so.

Failure handling:
- a request larger than the whole budget fails at submit;
- a backend that cannot place an admitted request right now (device memory
  fragmented or held by the allocator) raises Retry: the request goes back to
  the head of the queue and waits for running work to finish (it fails only
  if nothing is running to wait for);
- any other materialise or launch error fails only the requests concerned;
- an error while polling a running launch (a device fault) is sticky: every
  running, admitted and queued request fails with it, later submissions fail
  at once, and drain() returns instead of waiting for work that can never
  complete.
"""

from __future__ import annotations

import collections
import math
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Any, Optional


class Retry(Exception):
    """Raised by a backend's materialize() when the request cannot be placed
    now but may fit once running work releases its memory."""


@dataclass
class Request:
    """One problem.  `spec` is backend-specific (GpuBackend: a Workload-like
    object with plan parameters, E0_in and a displacement description)."""
    spec: Any
    precision: str = "fp32s"
    arrival: float = 0.0                 # server clock (s); set by submit()
    rid: int = -1
    footprint: int = 0                   # device bytes while admitted
    cell_updates: int = 0
    future: Future = field(default_factory=Future)
    state: str = "new"                   # new, queued, running, done, failed, cancelled
    admitted: float = math.nan
    launched: float = math.nan
    finished: float = math.nan
    device: Any = None                   # backend's per-request device state
    outputs: Any = None                  # backend's retained outputs, if any
    retained: int = 0                    # budget bytes still charged after done


class Server:
    """Admission by footprint, continuous batching over in-flight slots."""

    def __init__(self, backend, budget_bytes: float = 200e9,
                 max_in_flight: int = 4, tick_s: float = 0.0005,
                 max_batch: int = 512):
        self.backend = backend
        self.budget = float(budget_bytes)
        self.max_in_flight = int(max_in_flight)
        self.tick = float(tick_s)
        self.max_batch = int(max_batch)
        self._lock = threading.Lock()
        self._incoming = collections.deque()
        self._pending = collections.deque()
        self._in_flight = []                 # (handle, [requests])
        self._used = 0.0                     # footprints admitted + retained outputs
        self._retained = 0.0                 # part of _used held by finished outputs
        self._active = 0                     # admitted and not finished
        self._next_id = 0
        self._t0 = time.perf_counter()
        self._stop = threading.Event()
        self._thread = None
        self.completed = []
        self.failed = []
        self.launches = 0
        self.retries = 0
        self.peak_used = 0.0
        self.broken = None                   # sticky device error, if any
        # where the scheduler's time goes (host seconds) and what held back
        # admission (scheduler passes with requests waiting)
        self.host_materialize_s = 0.0
        self.host_launch_s = 0.0
        self.held_by_slots = 0
        self.held_by_budget = 0
        self.launch_log = []                 # (launched, finished, requests)

    # ---------------------------------------------------------------- API --
    def now(self) -> float:
        return time.perf_counter() - self._t0

    def start(self):
        self._thread = threading.Thread(target=self._run, name="bpm-serve",
                                        daemon=True)
        self._thread.start()
        return self

    def submit(self, req: Request) -> Future:
        req.footprint = int(self.backend.footprint(req))
        req.cell_updates = int(self.backend.cell_updates(req))
        with self._lock:
            req.rid = self._next_id
            self._next_id += 1
            req.arrival = self.now()
            req.state = "queued"
            if self.broken is not None:
                req.state = "failed"
                req.future.set_exception(RuntimeError(f"server stopped: {self.broken}"))
                self.failed.append(req)
            elif req.footprint > self.budget:
                req.state = "failed"
                req.future.set_exception(MemoryError(
                    f"request {req.rid} needs {req.footprint} B, more than the "
                    f"whole budget {self.budget:.0f} B"))
                self.failed.append(req)
            else:
                self._incoming.append(req)
        return req.future

    def cancel(self, req: Request) -> bool:
        """Cancel a request that has not been admitted yet."""
        with self._lock:
            for q in (self._incoming, self._pending):
                if req in q:
                    q.remove(req)
                    req.state = "cancelled"
                    req.future.cancel()
                    return True
        return False

    def release_outputs(self, req: Request) -> None:
        """Hand a finished request's retained outputs back: the backend drops
        them and their bytes return to the budget."""
        with self._lock:
            n = req.retained
            req.retained = 0
            self._used -= n
            self._retained -= n
        if hasattr(self.backend, "drop_outputs"):
            self.backend.drop_outputs(req)
        else:
            req.outputs = None

    def drain(self, timeout: Optional[float] = None) -> bool:
        """Wait until every submitted request has finished."""
        t_end = None if timeout is None else time.perf_counter() + timeout
        while True:
            with self._lock:
                busy = self._incoming or self._pending or self._active
            if not busy:
                return True
            if t_end is not None and time.perf_counter() > t_end:
                return False
            time.sleep(self.tick)

    def stop(self):
        self._stop.set()
        if self._thread is not None:
            self._thread.join()
        if hasattr(self.backend, "idle"):
            self.backend.idle()

    def stats(self) -> dict:
        done = [r for r in self.completed if r.state == "done"]
        lat = sorted(r.finished - r.arrival for r in done)

        def pct(p):
            if not lat:
                return math.nan
            k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
            return lat[k]
        span = (max(r.finished for r in done) - min(r.arrival for r in done)) if done else math.nan
        cells = sum(r.cell_updates for r in done)
        # time with at least one launch in flight, and mean launches in flight
        busy, area, end = 0.0, 0.0, -math.inf
        for t0, t1, _ in sorted(self.launch_log):
            area += t1 - t0
            if t1 > end:
                busy += t1 - max(t0, end)
                end = t1
        return dict(completed=len(done), failed=len(self.failed),
                    launches=self.launches, retries=self.retries,
                    p50_s=pct(50), p99_s=pct(99),
                    max_s=lat[-1] if lat else math.nan,
                    cell_updates=cells, span_s=span,
                    cell_updates_per_s=(cells / span) if done and span > 0 else math.nan,
                    peak_budget_used=self.peak_used,
                    retained_bytes=self._retained,
                    in_flight_time_s=busy,
                    mean_launches_in_flight=(area / busy) if busy > 0 else math.nan,
                    host_materialize_s=self.host_materialize_s,
                    host_launch_s=self.host_launch_s,
                    held_by_slots=self.held_by_slots,
                    held_by_budget=self.held_by_budget)

    # ---------------------------------------------------------- scheduler --
    def _run(self):
        while not self._stop.is_set():
            try:
                progressed = self._poll() | self._admit_and_launch()
            except Exception as e:          # noqa: BLE001 -- never leave waiters hanging
                self._break(e)
                progressed = False
            if not progressed:
                time.sleep(self.tick)

    def _break(self, err):
        """Sticky failure: fail everything in flight, admitted or queued."""
        if self.broken is None:
            self.broken = err
        for _, reqs in self._in_flight:
            for r in reqs:
                self._fail_now(r, err)
        self._in_flight = []
        with self._lock:
            waiting = list(self._incoming) + list(self._pending)
            self._incoming.clear()
            self._pending.clear()
        for r in waiting:
            r.state = "failed"
            r.finished = self.now()
            self.failed.append(r)
            r.future.set_exception(RuntimeError(f"server stopped: {err}"))

    def _poll(self) -> bool:
        done_any = False
        still = []
        for k, (handle, reqs) in enumerate(self._in_flight):
            try:
                status = self.backend.poll(handle)
            except Exception as e:          # noqa: BLE001 -- device fault: sticky
                self._in_flight = still + self._in_flight[k:]
                self._break(e)
                return True
            if status is None:
                still.append((handle, reqs))
                continue
            done_any = True
            t = self.now()
            if reqs:
                self.launch_log.append((reqs[0].launched, t, len(reqs)))
            for r in reqs:
                r.finished = t
                self.backend.release(r)
                keep = 0
                if status is True and hasattr(self.backend, "retained"):
                    keep = min(int(self.backend.retained(r)), r.footprint)
                r.retained = keep
                with self._lock:
                    # the outputs a finished request keeps stay charged
                    self._used -= r.footprint - keep
                    self._retained += keep
                    self._active -= 1
                if status is True:
                    r.state = "done"
                    self.completed.append(r)
                    r.future.set_result(r)
                else:
                    r.state = "failed"
                    self.failed.append(r)
                    r.future.set_exception(RuntimeError(str(status)))
        self._in_flight = still
        if done_any and not still and hasattr(self.backend, "idle"):
            self.backend.idle()              # nothing runs: deferred cleanup
        return done_any

    def _admit_and_launch(self) -> bool:
        if self.broken is not None:
            self._break(self.broken)
            return False
        with self._lock:
            while self._incoming:
                self._pending.append(self._incoming.popleft())
            if not self._pending:
                return False
            if len(self._in_flight) >= self.max_in_flight:
                self.held_by_slots += 1
                return False
            batch = []
            while (self._pending and len(batch) < self.max_batch
                   and self._used + self._pending[0].footprint <= self.budget):
                r = self._pending.popleft()
                self._used += r.footprint
                self._active += 1
                self.peak_used = max(self.peak_used, self._used)
                r.admitted = self.now()
                batch.append(r)
            if not batch:
                self.held_by_budget += 1
        if not batch:
            return False
        ok = []
        for k, r in enumerate(batch):
            try:
                t_m = time.perf_counter()
                try:
                    self.backend.materialize(r)
                finally:
                    self.host_materialize_s += time.perf_counter() - t_m
                ok.append(r)
            except Retry as e:
                if not self._in_flight and not ok:
                    self._fail_now(r, MemoryError(str(e)))   # nothing to wait for
                    continue
                # back to the head of the queue, in order, with the rest of
                # this batch; wait for running work to release memory
                rest = batch[k:]
                with self._lock:
                    for q in reversed(rest):
                        self._used -= q.footprint
                        self._active -= 1
                        q.admitted = math.nan
                        self._pending.appendleft(q)
                self.retries += 1
                break
            except Exception as e:          # noqa: BLE001 -- reported per request
                self._fail_now(r, e)
        if not ok:
            return True
        t_l = time.perf_counter()
        try:
            handle = self.backend.launch(ok)
        except Exception as e:              # noqa: BLE001
            for r in ok:
                self._fail_now(r, e)
            return True
        finally:
            self.host_launch_s += time.perf_counter() - t_l
        t = self.now()
        for r in ok:
            r.launched = t
            r.state = "running"
        self._in_flight.append((handle, ok))
        self.launches += 1
        return True

    def _fail_now(self, r, err):
        r.state = "failed"
        r.finished = self.now()
        try:
            self.backend.release(r)
        finally:
            self.failed.append(r)
            with self._lock:
                self._used -= r.footprint
                self._active -= 1
            r.future.set_exception(err if isinstance(err, Exception) else RuntimeError(str(err)))


class StreamSlots:
    """Launch streams and the completion event of the last launch on each.

    pick() returns the index of a stream whose last launch has completed (or
    that never ran one), the one picked least recently first; launches finish
    out of order (request sizes differ by ~1000x), so a round-robin choice
    would queue a new launch behind a long one while another stream idles.
    With every stream busy it returns the least recently picked one."""

    def __init__(self, streams):
        self.streams = list(streams)
        self.last = [None] * len(self.streams)
        self._order = list(range(len(self.streams)))   # least recently picked first

    def pick(self) -> int:
        choice = None
        for i in self._order:
            ev = self.last[i]
            if ev is None or ev.query():
                choice = i
                break
        if choice is None:
            choice = self._order[0]
        self._order.remove(choice)
        self._order.append(choice)
        return choice

    def record(self, i: int, event) -> None:
        self.last[i] = event


class PinnedRing:
    """Page-locked host staging for request inputs.

    A host array is copied into the next region of a ring of pinned memory
    and sent to the device with an asynchronous copy on the current stream.
    Copies from pinned memory go to the DMA engines; copies from pageable
    memory are staged by the runtime through a copy kernel, which has to
    wait for compute units that a running persistent march holds, so
    materialising the next requests stalled for as long as the running
    launch.  A region is written again only after the event recorded
    behind its copy has completed; the ring never waits for one (a copy
    can sit behind kernels of the same batch that wait for the running
    launch): when the next region is still in use, or an array is larger
    than the ring, that array takes the ordinary (pageable) path."""

    ALIGN = 256

    def __init__(self, torch, nbytes: int, device):
        import numpy as np
        self.torch = torch
        self.device = device
        self.n = int(nbytes)
        self.buf = torch.empty(self.n, dtype=torch.uint8, pin_memory=True)
        self.host = self.buf.numpy()
        self.head = 0
        self.live = collections.deque()      # (start, end, event), oldest first
        self.fallbacks = 0                   # arrays sent the pageable way
        self._tdt = {np.dtype(np.complex128): torch.complex128,
                     np.dtype(np.complex64): torch.complex64,
                     np.dtype(np.float64): torch.float64}

    def _reserve(self, nbytes: int):
        size = (nbytes + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        if size > self.n:
            return None
        start = 0 if self.head + size > self.n else self.head
        end = start + size
        self.live = collections.deque(r for r in self.live if not r[2].query())
        if any(a < end and start < b for (a, b, _) in self.live):
            self.fallbacks += 1
            return None                       # still being copied: do not wait
        self.head = end
        return start, end

    def to_device(self, arr, dtype=None):
        """Device copy of host array arr (cast to numpy dtype `dtype` on the
        way), asynchronous on the current stream."""
        import numpy as np
        torch = self.torch
        dt = np.dtype(dtype) if dtype is not None else np.asarray(arr).dtype
        nbytes = int(np.prod(np.shape(arr))) * dt.itemsize
        region = self._reserve(nbytes) if dt in self._tdt else None
        if region is None:
            return torch.from_numpy(np.ascontiguousarray(arr, dtype=dt)).to(self.device)
        start, end = region
        view = self.host[start:start + nbytes].view(dt).reshape(np.shape(arr))
        np.copyto(view, arr, casting="same_kind")
        src = self.buf[start:start + nbytes].view(self._tdt[dt]).view(np.shape(arr))
        out = torch.empty(np.shape(arr), dtype=self._tdt[dt], device=self.device)
        out.copy_(src, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        self.live.append((start, end, ev))
        return out


class GpuBackend:
    """Device side over libbpm.so: buffers from torch, one bpm_propagate_batch
    per launch on a pool of streams, completion by events.

    A request's spec is a Workload-like object (plan parameters, E0_in on the
    host, `meta['u_factors'] = (row, gz, gx, amp)` describing
    u[n, j] = row[j] + (amp gz[n]) gx[j], or `u` as an array, or no u)."""

    def __init__(self, streams: int = 3, device: int = 0, keep_outputs=True,
                 headroom_bytes: float = 0.0, staging_bytes: int = 2 << 30):
        """streams: launch streams, one launch in flight on each.  Below the
        GPU's capacity more launches in flight shorten the wait for a slot
        (at 150 req/s of the uneven mix, p50 0.72 / 0.45 / 0.25 s with two /
        three / four streams) at the same throughput; above capacity (200
        req/s) four streams raised p99 by 10-15% and three kept it.  Torch
        caches freed blocks per stream, so each stream splits the
        allocator's cache; with the inputs staged through the pinned ring
        that no longer stalls the scheduler.

        headroom_bytes > 0 caps torch's caching allocator at the device's
        memory minus that much, so the HIP runtime (queues, kernel scratch)
        can always allocate while the allocator holds cached blocks.

        staging_bytes: size of the pinned host ring that request inputs go
        through (PinnedRing); 0 copies from pageable memory."""
        import torch
        self.keep_outputs = keep_outputs
        self.torch = torch
        self.device = torch.device("cuda", device)
        if headroom_bytes > 0:
            total = torch.cuda.get_device_properties(self.device).total_memory
            torch.cuda.set_per_process_memory_fraction(
                max(0.05, 1.0 - float(headroom_bytes) / total), self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.slots = StreamSlots(self.streams)
        self._cur = None                     # slot of the batch being assembled
        self._retired = []                   # plans of finished requests
        # bound on retired plans (208 B of device constants per slice each,
        # a few hundred MB at most) before they are destroyed even while
        # launches run
        self.max_retired = 20000
        self.timing = {"plan_s": 0.0, "fields_s": 0.0, "u_s": 0.0, "job_s": 0.0}
        self.ring = PinnedRing(torch, staging_bytes, self.device) if staging_bytes > 0 else None

    @staticmethod
    def _cell(prec):
        return 16 if prec == "fp64" else 8

    def footprint(self, req) -> int:
        w = req.spec
        c = self._cell(req.precision)
        has_u = w.u is not None or "u_factors" in w.meta
        per_u = (8 + c) * w.Nz * w.Nx if has_u else 0
        return per_u + 3 * c * w.Nomega * w.Nx

    def cell_updates(self, req) -> int:
        w = req.spec
        return w.Nx * w.Nz * w.Nomega

    def retained(self, req) -> int:
        """Device bytes a finished request keeps: its two output fields when
        outputs are kept."""
        if not self.keep_outputs:
            return 0
        w = req.spec
        return 2 * self._cell(req.precision) * w.Nomega * w.Nx

    def drop_outputs(self, req):
        req.outputs = None

    def _slot(self) -> int:
        """Stream slot of the batch being assembled: chosen at its first
        materialize (a stream with no launch in flight) and used by its
        launch, so its buffers and its kernels share one stream."""
        if self._cur is None:
            self._cur = self.slots.pick()
        return self._cur

    def materialize(self, req):
        """Device buffers of one request, with no device temporaries: E0 is
        converted to the field type on the host, and u is formed in place
        from its separable description (u[n, j] = row[j] + (amp gz[n]) gx[j],
        the generator's operation order, so bitwise equal to it)."""
        import numpy as np
        from . import Job, Plan
        torch = self.torch
        w = req.spec
        s = self.streams[self._slot()]
        tm = self.timing
        try:
            with torch.cuda.stream(s):
                t0 = time.perf_counter()
                plan = Plan.from_workload(w, precision=req.precision)
                t1 = time.perf_counter()
                host_dtype = np.complex128 if plan.field_dtype == torch.complex128 \
                    else np.complex64
                E0 = self._to_device(w.E0_in, host_dtype)
                t2 = time.perf_counter()
                u = None
                if w.u is not None:
                    u = self._to_device(w.u, np.float64)
                elif "u_factors" in w.meta:
                    row, gz, gx, amp = w.meta["u_factors"]
                    gzs = self._to_device(amp * gz, np.float64)
                    u = torch.outer(gzs, self._to_device(gx, np.float64))
                    u.add_(self._to_device(row, np.float64))
                t3 = time.perf_counter()
                req.device = Job(plan, E0, u)
                t4 = time.perf_counter()
                tm["plan_s"] += t1 - t0
                tm["fields_s"] += t2 - t1
                tm["u_s"] += t3 - t2
                tm["job_s"] += t4 - t3
        except torch.OutOfMemoryError as e:
            req.device = None
            raise Retry(str(e)) from e

    def _to_device(self, arr, dtype):
        import numpy as np
        if self.ring is not None:
            return self.ring.to_device(arr, dtype)
        return self.torch.from_numpy(np.ascontiguousarray(arr, dtype=dtype)).to(self.device)

    def launch(self, reqs):
        from . import propagate_batch
        torch = self.torch
        i = self._slot()
        self._cur = None
        s = self.streams[i]
        with torch.cuda.stream(s):
            propagate_batch([r.device for r in reqs], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.slots.record(i, ev)
        return ev

    def poll(self, ev):
        return True if ev.query() else None

    def release(self, req):
        # inputs and workspace go back to the caching allocator; the outputs
        # stay with the request (device-resident) unless keep_outputs is off.
        # The plan is retired, not destroyed: destroying it frees its device
        # constants with hipFree, which waits for every launch on the device,
        # so plans are destroyed together when nothing is in flight (idle()).
        j = req.device
        if j is not None:
            req.device = None
            req.outputs = (j.E0_out, j.Eh_out) if self.keep_outputs else None
            self._retired.append(j.plan)
            if len(self._retired) > self.max_retired:
                self.idle()

    def idle(self):
        """Destroy the retired plans (called when no launch is in flight)."""
        self._retired.clear()

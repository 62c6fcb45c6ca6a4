"""Scheduling logic of the continuous-batching server, on the CPU with a
simulated device (no GPU): admission by footprint in arrival order,
continuous batching while earlier work runs, rejection of oversized
requests, failure isolation, cancellation and latency statistics."""

import threading
import time

import pytest

from paper_2201_08500_amd.serve import Request, Retry, Server


class FakeBackend:
    """Each launch 'runs' for the sum of its requests' durations / speedup."""

    def __init__(self, fail_launch=None, fail_materialize=None, speedup=1.0,
                 retry_materialize=None, poll_error_launch=None):
        self.lock = threading.Lock()
        self.retry_materialize = dict(retry_materialize or {})   # name -> times
        self.poll_error_launch = poll_error_launch
        self.launched = []            # list of (t, [rid...])
        self.live = 0
        self.max_live = 0
        self.fail_launch = fail_launch or set()
        self.fail_materialize = fail_materialize or set()
        self.speedup = speedup
        self.n = 0

    def footprint(self, req):
        return req.spec["bytes"]

    def cell_updates(self, req):
        return req.spec.get("cells", 1)

    def materialize(self, req):
        name = req.spec.get("name")
        if name in self.fail_materialize:
            raise RuntimeError("materialize failed")
        if self.retry_materialize.get(name, 0) > 0:
            self.retry_materialize[name] -= 1
            raise Retry("no room yet")
        req.device = object()

    def launch(self, reqs):
        with self.lock:
            k = self.n
            self.n += 1
            self.live += 1
            self.max_live = max(self.max_live, self.live)
        if k in self.fail_launch:
            with self.lock:
                self.live -= 1
            raise RuntimeError("launch failed")
        dur = max(r.spec.get("dur", 0.01) for r in reqs) / self.speedup
        self.launched.append((time.perf_counter(), [r.spec["name"] for r in reqs]))
        return (k, time.perf_counter() + dur)

    def poll(self, handle):
        k, t_end = handle
        if k == self.poll_error_launch and time.perf_counter() >= t_end:
            raise RuntimeError("device fault")
        if time.perf_counter() >= t_end:
            with self.lock:
                self.live -= 1
            return True
        return None

    def release(self, req):
        req.device = None


def req(name, nbytes, dur=0.01):
    return Request(spec=dict(name=name, bytes=nbytes, dur=dur))


def test_admission_by_footprint_in_arrival_order():
    be = FakeBackend()
    srv = Server(be, budget_bytes=100, max_in_flight=4).start()
    try:
        a = req("a", 60, 0.15)
        b = req("b", 60, 0.01)     # does not fit while a runs
        c = req("c", 30, 0.01)     # would fit, but waits behind b (FIFO)
        for r in (a, b, c):
            srv.submit(r)
            time.sleep(0.01)
        assert srv.drain(timeout=5)
        order = [names for _, names in be.launched]
        assert order[0] == ["a"]
        flat = [n for names in order for n in names]
        assert flat.index("b") < flat.index("c")
        assert srv.peak_used <= 100
        assert b.admitted >= a.finished - 1e-3
    finally:
        srv.stop()


def test_continuous_batching_packs_arrivals_while_others_run():
    be = FakeBackend()
    srv = Server(be, budget_bytes=1e9, max_in_flight=2).start()
    try:
        first = req("first", 10, 0.2)
        srv.submit(first)
        time.sleep(0.02)
        later = [req(f"r{i}", 10, 0.05) for i in range(6)]
        for r in later:
            srv.submit(r)
        assert srv.drain(timeout=5)
        # the six late arrivals were launched while `first` was still running,
        # packed into few launches
        assert max(r.launched for r in later) < first.finished
        assert len(be.launched) <= 3
        assert be.max_live == 2
        assert all(r.state == "done" for r in [first] + later)
    finally:
        srv.stop()


def test_oversized_request_is_rejected_at_submit():
    srv = Server(FakeBackend(), budget_bytes=100).start()
    try:
        r = req("big", 101)
        f = srv.submit(r)
        with pytest.raises(MemoryError):
            f.result(timeout=1)
        ok = req("ok", 50)
        assert srv.submit(ok).result(timeout=5) is ok
    finally:
        srv.stop()


def test_failed_launch_fails_only_its_requests():
    be = FakeBackend(fail_launch={0})
    srv = Server(be, budget_bytes=1e9, max_in_flight=1).start()
    try:
        a = req("a", 10)
        fa = srv.submit(a)
        with pytest.raises(RuntimeError):
            fa.result(timeout=5)
        b = req("b", 10)
        assert srv.submit(b).result(timeout=5) is b
        assert a.state == "failed" and b.state == "done"
        assert srv.drain(timeout=5)
        assert srv._used == 0
    finally:
        srv.stop()


def test_failed_materialize_is_isolated():
    be = FakeBackend(fail_materialize={"bad"})
    srv = Server(be, budget_bytes=1e9).start()
    try:
        bad, good = req("bad", 10), req("good", 10)
        fb, fg = srv.submit(bad), srv.submit(good)
        with pytest.raises(RuntimeError):
            fb.result(timeout=5)
        assert fg.result(timeout=5) is good
        assert srv.drain(timeout=5) and srv._used == 0
    finally:
        srv.stop()


def test_cancel_before_admission():
    be = FakeBackend()
    srv = Server(be, budget_bytes=100, max_in_flight=1).start()
    try:
        a = req("a", 90, 0.2)
        b = req("b", 90, 0.01)
        srv.submit(a)
        time.sleep(0.02)
        fb = srv.submit(b)
        assert srv.cancel(b)
        assert fb.cancelled()
        assert srv.drain(timeout=5)
        assert all("b" not in names for _, names in be.launched)
        assert not srv.cancel(a)           # already admitted
    finally:
        srv.stop()


def test_latency_statistics():
    be = FakeBackend()
    srv = Server(be, budget_bytes=1e9, max_in_flight=4).start()
    try:
        rs = [Request(spec=dict(name=str(i), bytes=1, dur=0.01, cells=100))
              for i in range(20)]
        for r in rs:
            srv.submit(r)
        assert srv.drain(timeout=5)
        st = srv.stats()
        assert st["completed"] == 20 and st["failed"] == 0
        assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
        assert st["cell_updates"] == 2000
    finally:
        srv.stop()


def test_retry_waits_for_running_work():
    """A request the device cannot place yet goes back to the head of the
    queue and is launched after running work completes, in order."""
    be = FakeBackend(retry_materialize={"b": 1})
    srv = Server(be, budget_bytes=1e9, max_in_flight=2).start()
    try:
        a = req("a", 10, 0.1)
        srv.submit(a)
        time.sleep(0.02)
        b, c = req("b", 10), req("c", 10)
        srv.submit(b)
        srv.submit(c)
        assert srv.drain(timeout=5)
        assert a.state == b.state == c.state == "done"
        flat = [n for _, names in be.launched for n in names]
        assert flat.index("b") < flat.index("c")
        assert srv.retries >= 1 and srv._used == 0
    finally:
        srv.stop()


def test_retry_with_nothing_running_fails_the_request():
    be = FakeBackend(retry_materialize={"x": 10})
    srv = Server(be, budget_bytes=1e9).start()
    try:
        f = srv.submit(req("x", 10))
        with pytest.raises(MemoryError):
            f.result(timeout=5)
        assert srv.submit(req("y", 10)).result(timeout=5).state == "done"
    finally:
        srv.stop()


def test_device_fault_fails_everything_and_drain_returns():
    """An error while polling a launch is sticky: running, queued and later
    requests fail, and drain() returns instead of hanging."""
    be = FakeBackend(poll_error_launch=0)
    srv = Server(be, budget_bytes=100, max_in_flight=1).start()
    try:
        a = req("a", 60, 0.05)
        fa = srv.submit(a)
        time.sleep(0.01)
        fb = srv.submit(req("b", 60))          # queued behind a (budget)
        with pytest.raises(RuntimeError):
            fa.result(timeout=5)
        with pytest.raises(RuntimeError):
            fb.result(timeout=5)
        assert srv.drain(timeout=5)
        assert srv.broken is not None
        with pytest.raises(RuntimeError):
            srv.submit(req("c", 1)).result(timeout=5)
    finally:
        srv.stop()


def test_scheduler_accounting():
    """stats() reports the time with launches in flight, their mean count,
    the host time per phase and why admission waited: two requests that
    each fill the budget run one after the other, so one launch is in flight
    at a time and the second request is held by the budget."""
    be = FakeBackend()
    srv = Server(be, budget_bytes=100, max_in_flight=4).start()
    try:
        r1 = srv.submit(req("a", 100, dur=0.05))
        r2 = srv.submit(req("b", 100, dur=0.05))
        assert srv.drain(timeout=5)
        r1.result(timeout=1)
        r2.result(timeout=1)
    finally:
        srv.stop()
    st = srv.stats()
    assert st["launches"] == 2
    assert st["held_by_budget"] > 0 and st["held_by_slots"] == 0
    assert 0.09 <= st["in_flight_time_s"] <= st["span_s"] + 1e-9
    assert st["mean_launches_in_flight"] == pytest.approx(1.0, abs=0.05)
    assert st["host_materialize_s"] >= 0.0 and st["host_launch_s"] >= 0.0


def test_backend_idle_hook_runs_when_nothing_is_in_flight():
    """A backend with idle() (deferred cleanup, e.g. destroying retired plans
    without waiting for running launches) is called only when no launch is
    in flight, and again at stop."""
    class IdleBackend(FakeBackend):
        def __init__(self):
            super().__init__()
            self.idle_live = []

        def idle(self):
            self.idle_live.append(self.live)

    be = IdleBackend()
    srv = Server(be, budget_bytes=100, max_in_flight=4).start()
    try:
        futs = [srv.submit(req(f"r{i}", 60, dur=0.02)) for i in range(3)]
        assert srv.drain(timeout=5)
        for f in futs:
            f.result(timeout=1)
    finally:
        srv.stop()
    assert len(be.idle_live) >= 2 and all(n == 0 for n in be.idle_live)


def test_retained_outputs_hold_back_admission():
    """A finished request's kept outputs stay charged to the budget until the
    caller releases them: the next request waits for that, not just for the
    launch to finish."""
    class KeepBackend(FakeBackend):
        def retained(self, r):
            return r.spec.get("keep", 0)

        def drop_outputs(self, r):
            r.outputs = None
            r.spec["dropped"] = True

    be = KeepBackend()
    srv = Server(be, budget_bytes=100, max_in_flight=2).start()
    try:
        a = Request(spec=dict(name="a", bytes=60, keep=50, dur=0.01))
        srv.submit(a).result(timeout=5)
        b = req("b", 60)
        fb = srv.submit(b)
        time.sleep(0.1)
        # 50 retained + 60 > 100: b stays queued while a's outputs are held
        assert b.state == "queued" and srv.stats()["retained_bytes"] == 50
        assert srv.peak_used <= 100
        srv.release_outputs(a)
        assert fb.result(timeout=5) is b
        assert a.spec["dropped"] and a.retained == 0
        assert srv.drain(timeout=5) and srv._used == 0
    finally:
        srv.stop()


def test_failed_request_retains_nothing():
    class KeepBackend(FakeBackend):
        def retained(self, r):
            return r.spec.get("keep", 0)

    be = KeepBackend(fail_launch={0})
    srv = Server(be, budget_bytes=100, max_in_flight=1).start()
    try:
        a = Request(spec=dict(name="a", bytes=60, keep=50))
        with pytest.raises(RuntimeError):
            srv.submit(a).result(timeout=5)
        assert srv.drain(timeout=5) and srv._used == 0 and a.retained == 0
    finally:
        srv.stop()


class _Event:
    def __init__(self, done=False):
        self.done = done

    def query(self):
        return self.done


def test_stream_slots_pick_an_idle_stream():
    """Launches finish out of order: with a long launch on stream 0 and a
    short one on stream 1 that has finished, the next launch goes to stream
    1, not back to stream 0 (round robin would queue it behind the long
    one)."""
    from paper_2201_08500_amd.serve import StreamSlots
    slots = StreamSlots(["s0", "s1"])
    i0 = slots.pick()
    long_ev = _Event(False)
    slots.record(i0, long_ev)
    i1 = slots.pick()
    assert i1 != i0
    short_ev = _Event(False)
    slots.record(i1, short_ev)
    short_ev.done = True
    assert slots.pick() == i1          # the idle stream, again
    slots.record(i1, _Event(False))
    # every stream busy: the least recently picked one
    assert slots.pick() == i0
    long_ev.done = True
    # both idle: the one picked least recently first
    s = StreamSlots(["a", "b", "c"])
    assert [s.pick() for _ in range(4)] == [0, 1, 2, 0]

"""Serving loop scheduler on the CPU with a fake executor: admission by slots and memory budget,
first-come-first-served order, per-request errors, latency percentiles."""

import threading
import time

import pytest

from paper_1103_6031_amd.serve import Request, Server, percentile, summarize


class FakeExec:
    """Sleeps for a request's service time and records what runs at the same time."""

    def __init__(self, service, footprint, fail_ids=()):
        self.service, self.footprint, self.fail_ids = service, footprint, set(fail_ids)
        self.lock = threading.Lock()
        self.running = {}
        self.max_conc = 0
        self.max_bytes = 0
        self.started = []

    def __call__(self, req, slot):
        with self.lock:
            assert slot not in self.running.values()
            self.running[req.id] = slot
            self.started.append(req.id)
            self.max_conc = max(self.max_conc, len(self.running))
            self.max_bytes = max(self.max_bytes, sum(self.footprint(Request(i, 0, 0)) for i in self.running))
        time.sleep(self.service(req))
        with self.lock:
            del self.running[req.id]
        if req.id in self.fail_ids:
            raise RuntimeError("planted failure")
        return 1000 * (req.id + 1)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([7.0], 99) == 7.0
    assert percentile([3, 1, 2], 50) == 2


def test_slots_and_budget_bound_concurrency():
    fp = lambda r: 3 if r.id % 2 else 5          # noqa: E731
    ex = FakeExec(lambda r: 0.02, fp)
    reqs = [Request(i, 0.002 * i, 32) for i in range(24)]
    srv = Server(ex, fp, slots=4, budget_bytes=10)
    recs = srv.run(reqs)
    assert all(r.error is None and r.done >= r.admitted >= r.arrival for r in recs.values())
    assert ex.max_conc <= 4
    assert ex.max_bytes <= 10
    assert srv.peak_bytes <= 10
    assert ex.started == sorted(ex.started)       # first come, first served
    assert all(r.latency >= 0.02 - 1e-3 for r in recs.values())


def test_budget_forces_queueing():
    fp = lambda r: 8                              # noqa: E731
    ex = FakeExec(lambda r: 0.03, fp)
    reqs = [Request(i, 0.0, 32) for i in range(4)]
    srv = Server(ex, fp, slots=4, budget_bytes=10)
    recs = srv.run(reqs)
    assert ex.max_conc == 1                        # only one request fits at a time
    q = sorted(r.queued for r in recs.values())
    assert q[-1] >= 0.08


def test_waits_are_attributed_to_memory_or_slots():
    # a large request at the head of the queue waits for memory while a slot is free, and the
    # small ones behind it wait too (first come, first served); with memory to spare and one slot,
    # requests wait for the slot instead
    fp = lambda r: 8 if r.id == 1 else 2          # noqa: E731
    ex = FakeExec(lambda r: 0.03, fp)
    reqs = [Request(0, 0.0, 32), Request(1, 0.001, 32), Request(2, 0.002, 32)]
    srv = Server(ex, fp, slots=4, budget_bytes=9)
    recs = srv.run(reqs)
    assert recs[1].waited_for_memory and not recs[1].waited_for_slot
    assert recs[2].admitted >= recs[1].admitted
    s = summarize(recs, srv)
    assert s["waited_for_memory"] >= 1 and s["queue_max_ms"] >= 20
    ex = FakeExec(lambda r: 0.02, lambda r: 1)
    recs = Server(ex, lambda r: 1, slots=1, budget_bytes=100).run([Request(i, 0.0, 32) for i in range(3)])
    assert sum(r.waited_for_slot for r in recs.values()) == 2
    assert not any(r.waited_for_memory for r in recs.values())


def test_overlap_when_resources_allow():
    fp = lambda r: 1                              # noqa: E731
    ex = FakeExec(lambda r: 0.05, fp)
    reqs = [Request(i, 0.0, 32) for i in range(4)]
    t0 = time.perf_counter()
    Server(ex, fp, slots=4, budget_bytes=100).run(reqs)
    assert ex.max_conc == 4
    assert time.perf_counter() - t0 < 0.15          # run together, not one after another


def test_errors_are_per_request_and_summary():
    fp = lambda r: 1                              # noqa: E731
    ex = FakeExec(lambda r: 0.005, fp, fail_ids={3})
    reqs = [Request(i, 0.001 * i, 32) for i in range(8)]
    srv = Server(ex, fp, slots=2, budget_bytes=100)
    recs = srv.run(reqs)
    assert recs[3].error and "planted" in recs[3].error
    assert all(recs[i].error is None for i in range(8) if i != 3)
    s = summarize(recs, srv)
    assert s["requests"] == 8 and s["failed"] == 1
    assert s["p99_ms"] >= s["p50_ms"] > 0
    assert s["mcell_updates_per_s"] > 0


def test_oversized_request_rejected():
    with pytest.raises(ValueError):
        Server(lambda r, s: 0, lambda r: 100, slots=1, budget_bytes=10).run([Request(0, 0.0, 32)])

"""The serving loop's scheduler on the CPU, with a fake executor whose
"device" work is a sleep: admission order, the memory budget, LRU eviction
of resident stencils, skip-ahead with its starvation bound, slot
concurrency and error propagation."""
import threading
import time

import pytest

from paper_2304_14690_amd import serve

F64, MIXED = 1, 3


class FakeExecutor:
    """Bytes and service times per grid size; tracks what is really held."""

    def __init__(self, sizes, service, fail_on=None):
        self.sizes = sizes          # (d, N) -> (geom bytes, ws bytes, field bytes)
        self.service = service      # (d, N) -> seconds
        self.fail_on = fail_on
        self.lock = threading.Lock()
        self.held = 0
        self.peak = 0
        self.running = 0
        self.max_running = 0
        self.built = []
        self.freed = []

    def _add(self, b):
        with self.lock:
            self.held += b
            self.peak = max(self.peak, self.held)

    def geometry_bytes(self, key):
        return self.sizes[key[:2]][0]

    def actual_geometry_bytes(self, handle, estimate):
        return handle[1]

    def workspace_bytes(self, key, mode, geom=None):
        return self.sizes[key[:2]][1] * (2 if mode == MIXED else 1)

    def field_bytes(self, key, mode):
        return self.sizes[key[:2]][2]

    def build_geometry(self, key, slot):
        b = self.geometry_bytes(key)
        self._add(b)
        self.built.append(key)
        time.sleep(0.001)
        return (key, b)

    def free_geometry(self, h):
        self._add(-h[1])
        self.freed.append(h[0])

    def make_workspace(self, key, geom, mode):
        b = self.workspace_bytes(key, mode)
        self._add(b)
        return (key, b)

    def free_workspace(self, h):
        self._add(-h[1])

    def run(self, r, geom, ws, slot):
        if self.fail_on is not None and r.rid == self.fail_on:
            raise RuntimeError("device error")
        fb = self.field_bytes(r.key, r.mode)
        self._add(fb)
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
        time.sleep(self.service[r.key[:2]])
        with self.lock:
            self.running -= 1
        self._add(-fb)
        return {"rc": 0, "n_it": 3}


SIZES = {(2, 64): (100, 10, 5), (2, 128): (400, 40, 20), (3, 32): (300, 30, 15)}
SERVICE = {(2, 64): 0.002, (2, 128): 0.005, (3, 32): 0.004}


def trace(n=60, rate=2000.0, seed=1, n_geom=3):
    return serve.poisson_trace(n, rate, seed, list(SIZES), {k: n_geom for k in SIZES}, 2,
                               [F64, MIXED])


def test_poisson_trace_is_seeded():
    a, b = trace(seed=5), trace(seed=5)
    assert [(r.arrival, r.d, r.N, r.geom, r.vel, r.mode) for r in a] == \
           [(r.arrival, r.d, r.N, r.geom, r.vel, r.mode) for r in b]
    gaps = [y.arrival - x.arrival for x, y in zip(a, a[1:])]
    assert all(g >= 0 for g in gaps) and a[0].arrival == 0.0


@pytest.mark.parametrize("slots", [1, 4])
def test_all_complete_with_ordered_times(slots):
    ex = FakeExecutor(SIZES, SERVICE)
    sch = serve.Scheduler(ex, budget=10_000, slots=slots)
    out = sch.run(trace())
    assert len(out) == 60
    for r in out:
        assert r.arrival <= r.admitted <= r.done and r.n_it == 3 and r.slot in range(slots)
    assert ex.max_running <= slots
    if slots == 1:
        # one in flight: first come, first served
        order = sorted(out, key=lambda r: r.admitted)
        assert [r.rid for r in order] == sorted(r.rid for r in out)
    # every geometry built once when everything fits
    assert len(ex.built) == len(set(ex.built))
    s = serve.summarize(out)
    assert s["requests"] == 60 and s["p99_ms"] >= s["p50_ms"] > 0 and 0 < s["utilisation"] <= 1
    sch.release()
    assert ex.held == 0


def test_budget_is_never_exceeded_and_lru_evicts():
    ex = FakeExecutor(SIZES, SERVICE)
    budget = 1200  # room for a few geometries only
    sch = serve.Scheduler(ex, budget=budget, slots=3)
    out = sch.run(trace(n=80, n_geom=4))
    assert len(out) == 80
    assert ex.peak <= budget and sch.peak_bytes <= budget
    assert sch.evictions > 0 and len(ex.freed) > 0
    # an evicted geometry that is requested again is built again
    assert len(ex.built) > len(set(ex.built))
    sch.release()
    assert ex.held == 0


def test_skip_ahead_is_bounded():
    """A large head that does not fit while small requests hold memory lets
    smaller ones pass at most max_skip times, then waits for room."""
    sizes = {(2, 64): (100, 10, 5), (2, 128): (700, 40, 20)}
    service = {(2, 64): 0.004, (2, 128): 0.001}
    ex = FakeExecutor(sizes, service)
    reqs = [serve.Request(i, 0.0, 2, 64, i % 4, 0, F64) for i in range(4)]
    reqs.append(serve.Request(4, 0.0005, 2, 128, 0, 0, F64))
    reqs += [serve.Request(5 + i, 0.001 + 0.0001 * i, 2, 64, i % 4, 0, F64) for i in range(20)]
    sch = serve.Scheduler(ex, budget=900, slots=4, max_skip=3)
    out = {r.rid: r for r in sch.run(reqs)}
    big = out[4]
    passed = [r for r in out.values() if r.rid > 4 and r.admitted < big.admitted]
    assert big.skipped <= 3 and len(passed) <= 3
    assert ex.peak <= 900


def test_request_larger_than_budget_is_refused():
    ex = FakeExecutor(SIZES, SERVICE)
    sch = serve.Scheduler(ex, budget=200, slots=2)
    with pytest.raises(MemoryError):
        sch.run([serve.Request(0, 0.0, 2, 128, 0, 0, F64)])


def test_executor_error_propagates():
    ex = FakeExecutor(SIZES, SERVICE, fail_on=7)
    sch = serve.Scheduler(ex, budget=10_000, slots=2)
    with pytest.raises(RuntimeError, match="device error"):
        sch.run(trace(n=20))


def test_same_geometry_built_once_under_concurrency():
    """Requests of one geometry admitted together share one build."""
    ex = FakeExecutor(SIZES, SERVICE)
    reqs = [serve.Request(i, 0.0, 3, 32, 0, i % 2, F64) for i in range(8)]
    sch = serve.Scheduler(ex, budget=10_000, slots=4)
    out = sch.run(reqs)
    assert ex.built == [(3, 32, 0)]
    assert sum(r.built for r in out) == 1


def test_pooled_workspace_counted_on_is_not_evicted():
    """Admission that counts on a pooled workspace (and so leaves its bytes
    out of the need) must not free that workspace to make room: the request
    would then allocate a new one beyond the budget."""
    sizes = {(2, 64): (100, 50, 20), (2, 8): (10, 10, 10)}
    service = {(2, 64): 0.002, (2, 8): 0.08}
    ex = FakeExecutor(sizes, service)
    reqs = [serve.Request(0, 0.0, 2, 64, 0, 0, F64),
            serve.Request(1, 0.001, 2, 8, 0, 0, F64),   # long-running
            serve.Request(2, 0.03, 2, 64, 0, 0, F64)]   # A again, while B runs
    sch = serve.Scheduler(ex, budget=195, slots=2)
    out = {r.rid: r for r in sch.run(reqs)}
    assert ex.peak <= 195 and sch.peak_bytes <= 195
    # A waited for B: the only room was A's own pooled workspace
    assert out[2].admitted >= out[1].done - 1e-3
    sch.release()
    assert ex.held == 0

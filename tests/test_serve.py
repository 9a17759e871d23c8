"""Serving loop: scheduling, admission and latency bookkeeping on a CPU executor (no GPU)."""
import numpy as np
import pytest

from paper_1712_00403_amd import serve


class FakePC:
    def __init__(self, N):
        self.N = N
        self.closed = False

    def close(self):
        self.closed = True


class VirtualExecutor:
    """Runs steps on a virtual clock: a step takes base + per_dof * DOFs after the previous one."""

    def __init__(self, sizes, plan_bytes, base=1e-4, per_dof=1e-9):
        self.sizes, self.plan_bytes = sizes, plan_bytes
        self.base, self.per_dof = base, per_dof
        self.now = 0.0
        self.busy_until = 0.0
        self.builds = []
        self.launched = []

    def build(self, rc):
        self.builds.append(rc.name)
        return FakePC(self.sizes[rc.name]), self.plan_bytes[rc.name]

    def io_bytes(self, pc):
        return 4 * pc.N

    def launch(self, items):
        start = max(self.now, self.busy_until)
        self.busy_until = start + self.base + self.per_dof * sum(pc.N for pc, _ in items)
        self.launched.append([r.rid for _, r in items])
        return self.busy_until

    def finished(self, handle, wait):
        if wait or handle <= self.now:
            return handle
        return None


def _classes(names):
    return {k: serve.RequestClass(k, None, "f32") for k in names}


def test_continuous_batching_and_latency():
    ex = VirtualExecutor({"a": 1000, "b": 5000}, {"a": 100, "b": 100}, base=1e-3)
    srv = serve.Server(_classes(["a", "b"]), ex, hbm_budget=10 ** 9, max_inflight=1)
    arrivals = [(0.0, "a"), (0.0001, "b"), (0.0002, "a"), (0.0005, "a")]
    reqs = []
    for i, (t, c) in enumerate(arrivals):
        r = serve.Request(i, c, t)
        reqs.append(r)
    # step 1 at t = 0: only request 0 has arrived
    ex.now = 0.0
    srv.submit(reqs[0])
    assert srv.step() == 1
    # requests 1..3 arrive while step 1 runs: no step while the device is busy,
    # then they go together in step 2
    for r in reqs[1:]:
        srv.submit(r)
    ex.now = 0.0006
    assert srv.step() == 0
    ex.now = 0.0011
    assert srv.step() == 3
    assert ex.launched == [[0], [1, 2, 3]]
    srv.collect(wait=True)
    assert all(r.done is not None for r in reqs)
    assert reqs[0].done == pytest.approx(1e-3 + 1e-6)
    # step 2 starts at t = 0.0011 (after step 1 ended)
    assert reqs[1].done == pytest.approx(0.0011 + 1e-3 + 7000e-9)
    summ = serve.latency_summary(reqs, 1.0)
    lat = [r.done - r.arrival for r in reqs]
    assert summ["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert summ["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert summ["requests"] == 4


def test_hbm_budget_evicts_idle_classes_lru():
    ex = VirtualExecutor({"a": 10, "b": 10, "c": 10}, {"a": 400, "b": 400, "c": 400})
    srv = serve.Server(_classes(["a", "b", "c"]), ex, hbm_budget=1000)
    for i, c in enumerate(["a", "b", "c", "a"]):
        srv.submit(serve.Request(i, c, 0.0))
        srv.step()
        srv.collect(wait=True)
        assert srv.cache.bytes <= 1000
    # a, b cached; c needs room: a (least recently used, idle) goes; a again: b goes
    assert ex.builds == ["a", "b", "c", "a"]
    assert srv.cache.evictions == 2
    assert list(srv.cache.entries) == ["c", "a"]


def test_class_larger_than_budget_is_an_error():
    ex = VirtualExecutor({"a": 10}, {"a": 5000})
    srv = serve.Server(_classes(["a"]), ex, hbm_budget=1000)
    srv.submit(serve.Request(0, "a", 0.0))
    with pytest.raises(RuntimeError):
        srv.step()


def test_step_respects_io_budget():
    # plans 100 B, residual results 4 N B: three requests of N = 100 need 1200 B of results
    ex = VirtualExecutor({"a": 100}, {"a": 100})
    srv = serve.Server(_classes(["a"]), ex, hbm_budget=100 + 800)
    for i in range(3):
        srv.submit(serve.Request(i, "a", 0.0))
    assert srv.step() == 2
    assert srv.step() == 1


def test_poisson_arrivals_rate_and_mix():
    arr = serve.poisson_arrivals(2000.0, 5.0, {"x": 0.7, "y": 0.25, "z": 0.05}, seed=4)
    assert abs(len(arr) / 5.0 - 2000.0) < 100
    times = [t for t, _ in arr]
    assert times == sorted(times) and times[-1] < 5.0
    frac = {k: sum(1 for _, c in arr if c == k) / len(arr) for k in "xyz"}
    assert abs(frac["x"] - 0.7) < 0.03 and abs(frac["z"] - 0.05) < 0.01
    assert serve.poisson_arrivals(2000.0, 5.0, {"x": 0.7, "y": 0.25, "z": 0.05}, seed=4) == arr

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
        self.busy_until = {}
        self.builds = []
        self.launched = []
        self.lanes = []

    def build(self, rc):
        self.builds.append(rc.name)
        return FakePC(self.sizes[rc.name]), self.plan_bytes[rc.name]

    def io_bytes(self, pc):
        return 4 * pc.N

    def launch(self, items, lane=0):
        # lanes run concurrently on the virtual device; steps of one lane in order
        start = max(self.now, self.busy_until.get(lane, 0.0))
        self.busy_until[lane] = start + self.base + self.per_dof * sum(pc.N for pc, _ in items)
        self.launched.append([r.rid for _, r in items])
        self.lanes.append(lane)
        return self.busy_until[lane]

    def finished(self, handle, wait):
        if wait or handle <= self.now:
            return handle
        return None


def _classes(names, lanes=None):
    lanes = lanes or {}
    return {k: serve.RequestClass(k, None, "f32", lanes.get(k, 0)) for k in names}


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
    # the results of the step in flight still hold 800 B: the third request waits
    assert srv.step() == 0
    assert srv.waits == 1
    ex.now = 1.0
    assert srv.step() == 1


def test_blocked_class_evicts_classes_with_pending_requests():
    # a and b cached (400 B each, budget 1000); a burst c, a, b: c must evict an
    # idle class although a and b have requests queued behind it
    ex = VirtualExecutor({"a": 10, "b": 10, "c": 10}, {"a": 400, "b": 400, "c": 400})
    srv = serve.Server(_classes(["a", "b", "c"]), ex, hbm_budget=1000)
    for i, c in enumerate(["a", "b"]):
        srv.submit(serve.Request(i, c, 0.0))
        srv.step()
        srv.collect(wait=True)
    assert list(srv.cache.entries) == ["a", "b"]
    for i, c in enumerate(["c", "a", "b"]):
        srv.submit(serve.Request(10 + i, c, 0.0))
    while srv.pending or srv.inflight:
        srv.step()
        ex.now += 1.0
        srv.collect()
    assert all(r.done is not None for r in srv.done)
    assert sorted(r.rid for r in srv.done) == [0, 1, 10, 11, 12]
    assert srv.cache.bytes <= 1000
    assert srv.cache.evictions >= 1


def test_class_bytes_are_remembered_no_rebuild_while_waiting():
    # b (600 B) cannot be admitted while a step of a (400 B) is in flight:
    # it is built once, refused, and later admitted without a rebuild attempt per retry
    ex = VirtualExecutor({"a": 10, "b": 10}, {"a": 400, "b": 600})
    srv = serve.Server(_classes(["a", "b"]), ex, hbm_budget=900)
    srv.submit(serve.Request(0, "a", 0.0))
    assert srv.step() == 1
    srv.submit(serve.Request(1, "b", 0.0))
    for _ in range(5):
        assert srv.step() == 0
    assert ex.builds == ["a", "b"]
    ex.now = 1.0
    assert srv.step() == 1
    assert ex.builds == ["a", "b", "b"]
    assert srv.cache.evictions == 1


def test_lanes_do_not_block_each_other():
    # a slow class in lane 1 and a fast class in lane 0: the fast requests run
    # beside the slow step, not behind it
    ex = VirtualExecutor({"small": 10, "big": 10 ** 7}, {"small": 10, "big": 10}, base=1e-4, per_dof=1e-9)
    srv = serve.Server(_classes(["small", "big"], {"small": 0, "big": 1}), ex, hbm_budget=10 ** 9,
                       max_inflight=1)
    srv.submit(serve.Request(0, "big", 0.0))
    srv.submit(serve.Request(1, "small", 0.0))
    assert srv.step() == 2
    assert ex.lanes == [0, 1] and ex.launched == [[1], [0]]
    srv.collect(wait=True)
    small = next(r for r in srv.done if r.cls == "small")
    big = next(r for r in srv.done if r.cls == "big")
    assert small.done == pytest.approx(1e-4 + 1e-8)
    assert big.done > 1e-2


def test_poisson_arrivals_rate_and_mix():
    arr = serve.poisson_arrivals(2000.0, 5.0, {"x": 0.7, "y": 0.25, "z": 0.05}, seed=4)
    assert abs(len(arr) / 5.0 - 2000.0) < 100
    times = [t for t, _ in arr]
    assert times == sorted(times) and times[-1] < 5.0
    frac = {k: sum(1 for _, c in arr if c == k) / len(arr) for k in "xyz"}
    assert abs(frac["x"] - 0.7) < 0.03 and abs(frac["z"] - 0.05) < 0.01
    assert serve.poisson_arrivals(2000.0, 5.0, {"x": 0.7, "y": 0.25, "z": 0.05}, seed=4) == arr


def test_requests_waiting_past_max_wait_are_rejected():
    # b (600 B plan) cannot be admitted while a's 2-s step (400 B plan, 400 B of
    # results) is in flight; with max_wait 0.5 s, b's request of t = 0 is shed at
    # t = 1, a later one is served
    ex = VirtualExecutor({"a": 100, "b": 10}, {"a": 400, "b": 600}, base=0.0, per_dof=0.02)
    srv = serve.Server(_classes(["a", "b"]), ex, hbm_budget=900, max_inflight=1, max_wait=0.5)
    srv.submit(serve.Request(0, "a", 0.0))
    assert srv.step(0.0) == 1
    srv.submit(serve.Request(1, "b", 0.0))
    assert srv.step(0.3) == 0 and not srv.rejected
    ex.now = 1.0
    srv.submit(serve.Request(2, "b", 0.9))
    assert srv.step(1.0) == 0  # a's step (2 s) is still on the device
    assert [r.rid for r in srv.rejected] == [1] and srv.rejected[0].rejected
    ex.now = 2.0
    srv.collect()
    assert srv.step(1.2) == 1  # request 2 has waited 0.3 s: admitted
    srv.collect(wait=True)
    assert sorted(r.rid for r in srv.done) == [0, 2]
    assert all(r.done is None for r in srv.rejected)


def test_no_request_is_rejected_without_max_wait():
    ex = VirtualExecutor({"a": 100, "b": 10}, {"a": 400, "b": 600}, base=0.0, per_dof=0.02)
    srv = serve.Server(_classes(["a", "b"]), ex, hbm_budget=900, max_inflight=1)
    srv.submit(serve.Request(0, "a", 0.0))
    srv.submit(serve.Request(1, "b", 0.0))
    for t in (0.0, 5.0, 50.0):
        srv.step(t)
    assert not srv.rejected
    ex.now = 100.0
    while srv.pending or srv.inflight:
        srv.step(100.0)
        srv.collect(wait=True)
    assert sorted(r.rid for r in srv.done) == [0, 1]


def test_run_stream_sheds_and_reports_rejections():
    # one slow class on one lane, arrivals faster than it is served: with
    # max_wait the stream ends with rejections counted in the summary
    ex = VirtualExecutor({"a": 10}, {"a": 10}, base=0.05, per_dof=0.0)
    clock_t = [0.0]

    def clock():
        clock_t[0] += 0.01
        ex.now = clock_t[0]
        return clock_t[0]

    srv = serve.Server(_classes(["a"]), ex, hbm_budget=10 ** 6, max_inflight=1, max_step_dofs=10, max_wait=0.1)
    arrivals = [(0.02 * i, "a") for i in range(50)]
    reqs = serve.run_stream(srv, arrivals, clock, {"a": 1}, idle_sleep=0)
    summ = serve.latency_summary(reqs, 1.0)
    assert summ["rejected"] == len(srv.rejected) > 0
    assert summ["requests"] + summ["rejected"] == len(arrivals)
    assert max(r.done - r.arrival for r in reqs if r.done is not None) <= 0.1 + 0.05 + 0.02

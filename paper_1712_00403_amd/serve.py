"""Serving loop for FD-apply requests: continuous batching over cached device plans.

A request asks for z = P_D^{-1} r for one block vector of a named problem
class (a Taylor-Hood patch in a precision). The server

* keeps the block preconditioners of the classes it has seen on the device
  (factors, eigenvalues, scalings) in an LRU cache bounded by an HBM budget;
  a class whose plans do not fit is admitted after evicting idle classes;
* batches continuously: with at most ``max_inflight`` steps on the device,
  every step takes the requests that have arrived and are admitted (FIFO,
  while the result buffers of the step stay within the budget) and applies
  all of their blocks with one fd_apply_batched call; requests arriving while
  the device is busy join the next step;
* records the completion of each step with an event on the launch stream, so
  the latency of a request is completion time minus arrival time.

The executor is pluggable: ``GpuExecutor`` runs the library on a HIP stream;
tests drive the same scheduler with a CPU executor.
"""
import collections
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass(frozen=True)
class RequestClass:
    """A problem class served: the patch and the precision of its plans."""
    name: str
    problem_factory: Callable  # () -> workloads.Problem
    precision: str


@dataclass
class Request:
    rid: int
    cls: str
    arrival: float                 # seconds on the server clock
    slot: int = 0                  # residual pool slot
    done: Optional[float] = None   # completion time on the server clock
    dofs: int = 0


class PlanCache:
    """Device plans per request class, LRU-evicted under an HBM budget (bytes)."""

    def __init__(self, build: Callable, budget: int):
        self.build = build                     # RequestClass -> (preconditioner, device bytes)
        self.budget = int(budget)
        self.entries: "collections.OrderedDict[str, tuple]" = collections.OrderedDict()
        self.bytes = 0
        self.evictions = 0

    def get(self, rc: RequestClass, busy: set, reserve: int = 0):
        """The class's preconditioner, building (and evicting idle classes) if needed; None if it cannot fit."""
        if rc.name in self.entries:
            self.entries.move_to_end(rc.name)
            return self.entries[rc.name][0]
        pc, nbytes = self.build(rc)
        while self.bytes + nbytes + reserve > self.budget:
            victim = next((k for k in self.entries if k not in busy), None)
            if victim is None:
                self._release(pc)
                return None
            old, ob = self.entries.pop(victim)
            self._release(old)
            self.bytes -= ob
            self.evictions += 1
        self.entries[rc.name] = (pc, nbytes)
        self.bytes += nbytes
        return pc

    @staticmethod
    def _release(pc):
        close = getattr(pc, "close", None)
        if close:
            close()


class Server:
    """Continuous-batching scheduler; the executor runs the batches."""

    def __init__(self, classes: Dict[str, RequestClass], executor, hbm_budget: int, max_step_dofs: int = 1 << 28,
                 max_inflight: int = 2):
        self.max_inflight = int(max_inflight)
        self.classes = classes
        self.ex = executor
        self.cache = PlanCache(executor.build, hbm_budget)
        self.budget = int(hbm_budget)
        self.max_step_dofs = int(max_step_dofs)
        self.pending: "collections.deque[Request]" = collections.deque()
        self.inflight: List[tuple] = []        # (handle, [requests])
        self.done: List[Request] = []
        self.steps = 0

    def submit(self, req: Request):
        self.pending.append(req)

    def _busy(self):
        return {r.cls for _, reqs in self.inflight for r in reqs}

    def step(self):
        """Launch one batch of admitted pending requests; returns the number launched."""
        self.collect()
        if not self.pending or len(self.inflight) >= self.max_inflight:
            return 0
        busy = self._busy() | {r.cls for r in self.pending}
        batch: List[Request] = []
        io_bytes = 0
        dofs = 0
        while self.pending:
            req = self.pending[0]
            rc = self.classes[req.cls]
            pc = self.cache.get(rc, busy - {req.cls}, reserve=io_bytes)
            if pc is None:
                if not batch and not self.inflight:
                    raise RuntimeError(f"class {req.cls} does not fit the HBM budget on its own")
                break
            need = self.ex.io_bytes(pc)
            if batch and (self.cache.bytes + io_bytes + need > self.budget or dofs + pc.N > self.max_step_dofs):
                break
            self.pending.popleft()
            req.dofs = pc.N
            batch.append(req)
            io_bytes += need
            dofs += pc.N
        if not batch:
            return 0
        handle = self.ex.launch([(self.cache.entries[r.cls][0], r) for r in batch])
        self.inflight.append((handle, batch))
        self.steps += 1
        return len(batch)

    def collect(self, wait=False):
        """Retire finished steps (all of them if ``wait``)."""
        still = []
        for handle, reqs in self.inflight:
            t = self.ex.finished(handle, wait)
            if t is None:
                still.append((handle, reqs))
                continue
            for r in reqs:
                r.done = t
                self.done.append(r)
        self.inflight = still


def poisson_arrivals(rate, duration, mix, seed):
    """(time, class name) pairs of a Poisson stream; ``mix`` maps class name -> probability."""
    rng = np.random.default_rng(seed)
    names = list(mix)
    probs = np.array([mix[k] for k in names], dtype=np.float64)
    probs /= probs.sum()
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append((t, names[int(rng.choice(len(names), p=probs))]))


def run_stream(server: Server, arrivals, clock, pool_slots: Dict[str, int], idle_sleep=0.0002):
    """Feed ``arrivals`` at their times (``clock()`` gives server seconds) and serve until all finish."""
    reqs = []
    i = 0
    slot_next = collections.Counter()
    while i < len(arrivals) or server.pending or server.inflight:
        now = clock()
        while i < len(arrivals) and arrivals[i][0] <= now:
            t, name = arrivals[i]
            slot = slot_next[name] % max(pool_slots.get(name, 1), 1)
            slot_next[name] += 1
            r = Request(rid=i, cls=name, arrival=t, slot=slot)
            reqs.append(r)
            server.submit(r)
            i += 1
        launched = server.step()
        if not launched:
            server.collect()
            if i < len(arrivals) and not server.pending:
                wait = arrivals[i][0] - clock()
                if wait > 0:
                    time.sleep(min(wait, 0.002))
            elif idle_sleep:
                time.sleep(idle_sleep)
    server.collect(wait=True)
    return reqs


def latency_summary(reqs, duration):
    lat = np.array([r.done - r.arrival for r in reqs if r.done is not None])
    dofs = sum(r.dofs for r in reqs if r.done is not None)
    span = max((r.done for r in reqs if r.done is not None), default=duration)
    by_cls = collections.defaultdict(list)
    for r in reqs:
        if r.done is not None:
            by_cls[r.cls].append(r.done - r.arrival)
    return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "dof_per_s": dofs / max(span, 1e-9),
            "per_class": {k: {"n": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3),
                              "p99_ms": float(np.percentile(v, 99) * 1e3)} for k, v in by_cls.items()}}


class GpuExecutor:
    """Runs a step as one fd_apply_batched call on a HIP stream; completion from a HIP event.

    Residuals come from a device pool per class (``slots`` vectors each,
    drawn once from seeded generators); each request writes its own result
    buffer, which the executor allocates per step from a reusable arena.
    """

    def __init__(self, classes: Dict[str, RequestClass], slots: int = 4, seed: int = 4, t0: Optional[float] = None):
        import torch
        from . import fd
        self.torch = torch
        self.fd = fd
        self.classes = classes
        self.slots = slots
        self.seed = seed
        self.stream = torch.cuda.Stream()
        self.pools = {}
        self.arena = None
        self.t0 = time.perf_counter() if t0 is None else t0
        self.ev_ref = None

    def build(self, rc: RequestClass):
        from .precond import BlockPreconditioner
        from . import workloads
        pc = BlockPreconditioner(rc.problem_factory(), precision=rc.precision)
        if rc.name not in self.pools:
            dt = self.torch.float64 if pc.io_dtype == "float64" else self.torch.float32
            cls_idx = sorted(self.classes).index(rc.name)
            host = workloads.residuals(self.seed * 1000 + cls_idx, self.slots, pc.N)
            self.pools[rc.name] = self.torch.from_numpy(host).to(dt).cuda()
        nbytes = sum(p.device_bytes for p in pc.plans)
        return pc, nbytes

    def io_bytes(self, pc):
        # the request's result vector plus what the library reports it needs per apply
        return pc.N * (8 if pc.io_dtype == "float64" else 4) + sum(p.workspace_bytes(1) for p in pc.plans)

    def launch(self, items):
        torch = self.torch
        works, outs = [], []
        if self.ev_ref is None:
            # clock origin of the device timeline: recorded on the idle stream
            self.ev_ref = torch.cuda.Event(enable_timing=True)
            self.ev_ref.record(self.stream)
            self.ref_host = time.perf_counter() - self.t0
        with torch.cuda.stream(self.stream):
            for pc, req in items:
                r = self.pools[req.cls][req.slot]
                z = torch.empty_like(r)
                outs.append(z)
                works += pc.works(r.data_ptr(), z.data_ptr(), 1)
            self.fd.apply_batched(works, self.stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.stream)
        return (ev, outs, [r for _, r in items])

    def finished(self, handle, wait):
        ev, outs, reqs = handle
        if not wait and not ev.query():
            return None
        ev.synchronize()
        # completion on the server clock: the event's time after the reference event
        return self.ref_host + self.ev_ref.elapsed_time(ev) * 1e-3

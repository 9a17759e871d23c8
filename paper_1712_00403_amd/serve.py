"""Serving loop for FD-apply requests: continuous batching over cached device plans.

A request asks for z = P_D^{-1} r for one block vector of a named problem
class (a Taylor-Hood patch in a precision). The server

* keeps the block preconditioners of the classes it has seen on the device
  (factors, eigenvalues, scalings, and the class's residual pool) in an LRU
  cache bounded by an HBM budget; a class that is not cached is admitted
  after evicting classes that no step in flight uses;
* counts against the same budget the result buffers of every step still on
  the device and of the step being formed, so cached plans plus live
  results never exceed it;
* batches continuously, per lane: every class belongs to a lane (one HIP
  stream each, all at the default priority); with at most ``max_inflight``
  steps of a lane on the device, a step takes the requests of that lane that
  have arrived and fit (FIFO) and applies all of their blocks with one
  fd_apply_batched call. Requests arriving while the device is busy join the
  next step of their lane; small classes in a lane of their own never queue
  behind the steps of large ones;
* records the completion of each step with an event on its lane's stream,
  so the latency of a request is completion time minus arrival time;
* optionally sheds load: with ``max_wait`` set, a request still queued that
  many seconds after its arrival is rejected (``Request.rejected``, listed
  in ``Server.rejected``) instead of being served late.

The executor is pluggable: ``GpuExecutor`` runs the library on HIP streams;
tests drive the same scheduler with a CPU executor.
"""
import collections
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass(frozen=True)
class RequestClass:
    """A problem class served: the patch, the precision of its plans, and its lane."""
    name: str
    problem_factory: Callable  # () -> workloads.Problem
    precision: str
    lane: int = 0


@dataclass
class Request:
    rid: int
    cls: str
    arrival: float                 # seconds on the server clock
    slot: int = 0                  # residual pool slot
    done: Optional[float] = None   # completion time on the server clock
    dofs: int = 0
    rejected: bool = False         # shed after waiting longer than the server's max_wait


class PlanCache:
    """Device entries per request class, LRU-evicted under an HBM budget (bytes).

    The device bytes of a class are learned at its first build and kept, so a
    class that does not fit later is refused before anything is allocated.
    """

    def __init__(self, build: Callable, budget: int):
        self.build = build                     # RequestClass -> (entry, device bytes)
        self.budget = int(budget)
        self.entries: "collections.OrderedDict[str, tuple]" = collections.OrderedDict()
        self.known: Dict[str, int] = {}
        self.bytes = 0
        self.evictions = 0
        self.builds = 0

    def make_room(self, need: int, protected: set, reserve: int) -> bool:
        """Evict unprotected entries (least recently used first) until ``need`` more bytes fit."""
        while self.bytes + need + reserve > self.budget:
            victim = next((k for k in self.entries if k not in protected), None)
            if victim is None:
                return False
            old, ob = self.entries.pop(victim)
            self._release(old)
            self.bytes -= ob
            self.evictions += 1
        return True

    def get(self, rc: RequestClass, protected: set, reserve: int = 0):
        """The class's entry, building it (after evicting unprotected classes) if needed; None if it cannot fit.

        ``reserve``: bytes that must stay free besides the cached entries
        (result buffers of the steps in flight and of the step being formed).
        """
        if rc.name in self.entries:
            self.entries.move_to_end(rc.name)
            return self.entries[rc.name][0]
        if rc.name in self.known and not self.make_room(self.known[rc.name], protected, reserve):
            return None
        entry, nbytes = self.build(rc)
        self.builds += 1
        self.known[rc.name] = int(nbytes)
        if not self.make_room(nbytes, protected, reserve):
            self._release(entry)
            return None
        self.entries[rc.name] = (entry, int(nbytes))
        self.bytes += int(nbytes)
        return entry

    @staticmethod
    def _release(entry):
        close = getattr(entry, "close", None)
        if close:
            close()


class Server:
    """Continuous-batching scheduler with one FIFO per lane; the executor runs the steps."""

    def __init__(self, classes: Dict[str, RequestClass], executor, hbm_budget: int, max_step_dofs: int = 1 << 28,
                 max_inflight: int = 2, max_wait: Optional[float] = None):
        self.max_inflight = int(max_inflight)
        self.max_wait = None if max_wait is None else float(max_wait)
        self.rejected: List[Request] = []
        self.classes = classes
        self.ex = executor
        self.cache = PlanCache(executor.build, hbm_budget)
        self.budget = int(hbm_budget)
        self.max_step_dofs = int(max_step_dofs)
        self.lanes = sorted({rc.lane for rc in classes.values()})
        self.queues: Dict[int, "collections.deque[Request]"] = {l: collections.deque() for l in self.lanes}
        self.inflight: List[tuple] = []        # (handle, [requests], result bytes, lane)
        self.done: List[Request] = []
        self.steps = 0
        self.waits = 0                         # steps not launched for lack of memory

    @property
    def pending(self):
        return any(self.queues.values())

    def submit(self, req: Request):
        self.queues[self.classes[req.cls].lane].append(req)

    def _inflight_io(self):
        return sum(io for _, _, io, _ in self.inflight)

    def step(self, now: Optional[float] = None):
        """Launch at most one step per lane from its admitted pending requests; returns the number launched.

        ``now`` (server seconds) is needed only with ``max_wait``: queued
        requests that arrived more than ``max_wait`` before it are rejected first.
        """
        self.collect()
        if self.max_wait is not None and now is not None:
            self._shed(now)
        launched = 0
        for lane in self.lanes:
            launched += self._step_lane(lane)
        return launched

    def _shed(self, now):
        for lane, q in self.queues.items():
            if not any(now - r.arrival > self.max_wait for r in q):
                continue
            keep = collections.deque()
            for r in q:
                if now - r.arrival > self.max_wait:
                    r.rejected = True
                    self.rejected.append(r)
                else:
                    keep.append(r)
            self.queues[lane] = keep

    def _step_lane(self, lane):
        q = self.queues[lane]
        if not q or sum(1 for s in self.inflight if s[3] == lane) >= self.max_inflight:
            return 0
        batch: List[Request] = []
        io_bytes = 0
        dofs = 0
        while q:
            req = q[0]
            rc = self.classes[req.cls]
            protected = {r.cls for _, reqs, _, _ in self.inflight for r in reqs} | {r.cls for r in batch}
            live = self._inflight_io() + io_bytes
            entry = self.cache.get(rc, protected, reserve=live)
            fits = entry is not None
            if fits:
                # room for the result too, evicting other idle classes if needed
                need = self.ex.io_bytes(entry)
                fits = self.cache.make_room(need, protected | {req.cls}, live)
            if not fits:
                if not batch and not self.inflight:
                    # nothing else holds memory and every other class was evicted:
                    # the class and its result alone exceed the budget
                    raise RuntimeError(f"class {req.cls} does not fit the HBM budget on its own")
                if not batch:
                    self.waits += 1
                break
            if batch and dofs + entry.N > self.max_step_dofs:
                break
            q.popleft()
            req.dofs = entry.N
            batch.append(req)
            io_bytes += need
            dofs += entry.N
        if not batch:
            return 0
        handle = self.ex.launch([(self.cache.entries[r.cls][0], r) for r in batch], lane)
        self.inflight.append((handle, batch, io_bytes, lane))
        self.steps += 1
        return len(batch)

    def collect(self, wait=False):
        """Retire finished steps (all of them if ``wait``)."""
        still = []
        for item in self.inflight:
            t = self.ex.finished(item[0], wait)
            if t is None:
                still.append(item)
                continue
            for r in item[1]:
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


def run_stream(server: Server, arrivals, clock, pool_slots: Dict[str, int], idle_sleep=0.0002, keep=None):
    """Feed ``arrivals`` at their times (``clock()`` gives server seconds) and serve until all finish.

    ``keep``: optional set of request ids whose results the executor keeps
    (``executor.kept[rid]``) for checking afterwards.
    """
    reqs = []
    i = 0
    slot_next = collections.Counter()
    if keep is not None:
        server.ex.keep = set(keep)
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
        launched = server.step(clock())
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
    return {"requests": int(lat.size), "rejected": sum(1 for r in reqs if r.rejected), "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "dof_per_s": dofs / max(span, 1e-9),
            "per_class": {k: {"n": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3),
                              "p99_ms": float(np.percentile(v, 99) * 1e3)} for k, v in by_cls.items()}}


class ServedClass:
    """Device state of a cached class: its block preconditioner and its residual pool."""

    def __init__(self, pc, pool):
        self.pc = pc
        self.pool = pool
        self.N = pc.N

    def close(self):
        self.pc.close()
        self.pool = None


class GpuExecutor:
    """Runs a step as one fd_apply_batched call on its lane's HIP stream; completion from a HIP event.

    Residuals come from a device pool per class (``slots`` vectors each,
    drawn from seeded generators when the class is built, freed with it);
    each request writes its own result buffer.
    """

    def __init__(self, classes: Dict[str, RequestClass], slots: int = 4, seed: int = 4, t0: Optional[float] = None):
        import torch
        from . import fd
        self.torch = torch
        self.fd = fd
        self.classes = classes
        self.slots = slots
        self.seed = seed
        self.streams = {}
        self.t0 = time.perf_counter() if t0 is None else t0
        self.ev_ref = None
        self.keep = set()
        self.kept = {}

    def stream(self, lane):
        if lane not in self.streams:
            self.streams[lane] = self.torch.cuda.Stream()   # default priority
        return self.streams[lane]

    def pool_residuals(self, rc: RequestClass, N: int):
        """The host residuals of a class's pool (seeded by the executor seed and the class)."""
        from . import workloads
        cls_idx = sorted(self.classes).index(rc.name)
        return workloads.residuals(self.seed * 1000 + cls_idx, self.slots, N)

    def build(self, rc: RequestClass):
        from .precond import BlockPreconditioner
        pc = BlockPreconditioner(rc.problem_factory(), precision=rc.precision)
        dt = self.torch.float64 if pc.io_dtype == "float64" else self.torch.float32
        pool = self.torch.from_numpy(self.pool_residuals(rc, pc.N)).to(dt).cuda()
        nbytes = sum(p.device_bytes for p in pc.plans) + pool.numel() * pool.element_size()
        return ServedClass(pc, pool), nbytes

    def io_bytes(self, entry):
        # the request's result vector plus what the library reports it needs per apply
        pc = entry.pc
        return pc.N * (8 if pc.io_dtype == "float64" else 4) + sum(p.workspace_bytes(1) for p in pc.plans)

    def launch(self, items, lane=0):
        torch = self.torch
        works, outs = [], []
        s = self.stream(lane)
        if self.ev_ref is None:
            # clock origin of the device timeline: recorded on an idle stream
            self.ev_ref = torch.cuda.Event(enable_timing=True)
            self.ev_ref.record(s)
            self.ref_host = time.perf_counter() - self.t0
        with torch.cuda.stream(s):
            for entry, req in items:
                r = entry.pool[req.slot]
                z = torch.empty_like(r)
                outs.append(z)
                works += entry.pc.works(r.data_ptr(), z.data_ptr(), 1)
            self.fd.apply_batched(works, s)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        for (entry, req), z in zip(items, outs):
            if req.rid in self.keep:
                self.kept[req.rid] = z
        return (ev, outs, [r for _, r in items])

    def finished(self, handle, wait):
        ev, outs, reqs = handle
        if not wait and not ev.query():
            return None
        ev.synchronize()
        # completion on the server clock: the event's time after the reference event
        return self.ref_host + self.ev_ref.elapsed_time(ev) * 1e-3

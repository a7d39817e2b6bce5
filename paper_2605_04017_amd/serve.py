"""Continuous-batching request loop for lens transport queries.

Requests (lens id, a batch of sensor-side rays, arrival time) arrive over
time.  The scheduler keeps every lens and map resident, admits requests as
long as the device-memory budget for in-flight requests allows, splits large
requests into chunks, and launches chunks on a pool of HIP streams as soon
as a stream slot is free, so requests that arrive while others run overlap
with them on the device.  Latency is arrival -> completion of the request's
last chunk.

Scheduling policy (deterministic): waiting requests are served in arrival
order; a request is admitted when its memory fits the remaining budget (a
request larger than the whole budget is rejected); admitted requests feed
chunks to free slots round-robin, so a long request does not block short
ones behind it.

Two implementations share this policy.  `NativeScheduler` drives the
native loop of liblt.so (lt_server_*: admission, chunking, stream slots and
completion events in C++); it is what serving uses.  `Scheduler` is the same
policy in Python over an executor with three operations (launch a chunk on a
slot, ask whether a slot's work is done, read completion times):
`GpuExecutor` runs lt_map_eval / lt_trace on HIP streams, and the policy
tests use a simulated executor.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import time
from typing import Callable, Dict, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    lens: int
    n: int
    arrival: float                 # seconds, on the scheduler's clock
    payload: object = None         # executor-specific (e.g. device ray tensors)
    prepared: object = None        # marshalled launch arguments (native loop)
    # filled by the scheduler
    admitted: float = -1.0
    done: float = -1.0
    chunks_left: int = 0
    next_offset: int = 0
    rejected: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Continuous batching over `executor.n_slots` concurrent slots."""

    def __init__(self, executor, mem_budget_bytes: int, bytes_per_ray: int, chunk: int = 262144):
        self.ex = executor
        self.budget = int(mem_budget_bytes)
        self.bpr = int(bytes_per_ray)
        self.chunk = int(chunk)
        self.in_use = 0
        self.waiting: collections.deque = collections.deque()
        self.active: List[Request] = []
        self.slot_req: Dict[int, Request] = {}
        self.free_slots = list(range(executor.n_slots))
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self._rr = 0

    def mem_of(self, r: Request) -> int:
        return r.n * self.bpr

    def submit(self, r: Request):
        if self.mem_of(r) > self.budget:
            r.rejected = True
            self.rejected.append(r)
            return
        r.chunks_left = max(1, -(-r.n // self.chunk))
        self.waiting.append(r)

    def _admit(self, now: float):
        while self.waiting and self.in_use + self.mem_of(self.waiting[0]) <= self.budget:
            r = self.waiting.popleft()
            r.admitted = now
            self.in_use += self.mem_of(r)
            self.active.append(r)

    def _launch(self):
        while self.free_slots and any(r.next_offset < r.n for r in self.active):
            # round-robin over admitted requests that still have chunks to start
            cands = [r for r in self.active if r.next_offset < r.n]
            r = cands[self._rr % len(cands)]
            self._rr += 1
            slot = self.free_slots.pop()
            lo = r.next_offset
            hi = min(r.n, lo + self.chunk)
            r.next_offset = hi
            self.slot_req[slot] = r
            self.ex.launch(slot, r, lo, hi)

    def _reap(self):
        for slot in list(self.slot_req):
            if self.ex.done(slot):
                r = self.slot_req.pop(slot)
                self.free_slots.append(slot)
                r.chunks_left -= 1
                if r.chunks_left == 0:
                    r.done = self.ex.finish_time(slot)
                    self.in_use -= self.mem_of(r)
                    self.active.remove(r)
                    self.finished.append(r)

    def step(self, now: float):
        self._reap()
        self._admit(now)
        self._launch()

    @property
    def idle(self) -> bool:
        return not self.waiting and not self.active


class NativeScheduler:
    """The native request loop (lt_server_*) behind the interface run_trace
    uses.  ``r.payload`` holds (rays, out): the request's device ray tensors
    and its preallocated outputs (empty_map_out(1, n) or empty_exit(n)).
    Completion times are device times after the server's start event, so the
    clock to replay arrivals against is ``clock`` (host seconds since the
    server was created)."""

    def __init__(self, server, lenses, maps, mode: str = "map", dtype: int = 1,
                 path=(0, 0, 0)):
        self.server = server
        self.t0 = time.perf_counter()
        self.lenses, self.maps, self.mode, self.dtype, self.path = lenses, maps, mode, dtype, path
        self.reqs: Dict[int, Request] = {}
        self.finished: List[Request] = []
        self.rejected: List[Request] = []

    def clock(self) -> float:
        return time.perf_counter() - self.t0

    def prepare(self, r: Request):
        """Marshal the request's launch arguments ahead of its arrival (what
        a client library does when it builds a request)."""
        import paper_2605_04017_amd as lt
        rays, out = r.payload
        if self.mode == "map":
            r.prepared = lt.Server.prepare_map(self.maps[r.lens], self.dtype, rays, out, r.n)
        else:
            r.prepared = lt.Server.prepare_trace(self.lenses[r.lens], self.path, rays, out, r.n)

    def submit(self, r: Request):
        import paper_2605_04017_amd as lt
        if getattr(r, "prepared", None) is None:
            self.prepare(r)
        try:
            self.server.submit(r.prepared, r.rid)
        except lt.LtError as e:
            if e.status != lt.LT_ERR_ARG:
                raise
            r.rejected = True
            self.rejected.append(r)
            return
        self.reqs[r.rid] = r

    def step(self, now: float):
        done, _ = self.server.poll()
        for tag, done_s, status in done:
            r = self.reqs.pop(tag)
            if status != 0:
                raise RuntimeError(f"request {tag} failed with status {status}")
            r.done = done_s
            self.finished.append(r)

    @property
    def idle(self) -> bool:
        return not self.reqs


def run_trace(sched: Scheduler, requests: List[Request], clock: Callable[[], float],
              wait: Optional[Callable[[float], None]] = None) -> List[Request]:
    """Replay `requests` (sorted by arrival) against the scheduler's clock."""
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    i = 0
    while i < len(pending) or not sched.idle:
        now = clock()
        k = 0
        while i < len(pending) and pending[i].arrival <= now:
            sched.submit(pending[i])
            i += 1
            k += 1
            if k % 16 == 0:   # keep the device fed while a burst is being queued
                sched.step(now)
        sched.step(now)
        if wait is not None:
            nxt = pending[i].arrival if i < len(pending) else None
            wait(nxt)
    return sched.finished


# ---------------------------------------------------------------- executors

class SimExecutor:
    """Simulated device for scheduler tests: each slot runs one chunk at a
    time; a chunk of k rays takes overhead + k / rate seconds of simulated
    time; slots run concurrently (rate is per slot)."""

    def __init__(self, n_slots: int, rate_rays_per_s: float, overhead_s: float = 10e-6):
        self.n_slots = n_slots
        self.rate = rate_rays_per_s
        self.overhead = overhead_s
        self.now = 0.0
        self.busy_until: Dict[int, float] = {}
        self.log: List[tuple] = []

    def clock(self) -> float:
        return self.now

    def launch(self, slot, r, lo, hi):
        start = self.now
        end = start + self.overhead + (hi - lo) / self.rate
        self.busy_until[slot] = end
        self.log.append((slot, r.rid, lo, hi, start, end))

    def done(self, slot) -> bool:
        return self.busy_until.get(slot, 0.0) <= self.now

    def finish_time(self, slot) -> float:
        return self.busy_until[slot]

    def wait(self, next_arrival: Optional[float]):
        """Advance simulated time to the next event."""
        events = [t for t in self.busy_until.values() if t > self.now]
        if next_arrival is not None:
            events.append(next_arrival)
        if events:
            self.now = max(self.now, min(events))


class GpuExecutor:
    """Launches lt_map_eval (or lt_trace) for request chunks on HIP streams."""

    def __init__(self, n_slots: int, lenses, maps, mode: str = "map", dtype: int = 1,
                 outputs: Optional[Dict[int, Dict]] = None):
        import torch
        self.torch = torch
        self.n_slots = n_slots
        # all streams at the default priority
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.events = [None] * n_slots
        self.lenses, self.maps = lenses, maps
        self.mode, self.dtype = mode, dtype
        if mode == "map":
            # packed weights built once, before chunks of one map run on several streams
            import paper_2605_04017_amd as lt
            for m in maps:
                lt.lt_map_quantize(m, dtype)
            torch.cuda.synchronize()
        self.outputs = outputs if outputs is not None else {}
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_host = None

    def start_clock(self):
        self.torch.cuda.synchronize()
        self.t0_event.record(self.torch.cuda.current_stream())
        self.torch.cuda.synchronize()
        self.t0_host = time.perf_counter()

    def clock(self) -> float:
        return time.perf_counter() - self.t0_host

    def launch(self, slot, r, lo, hi):
        import paper_2605_04017_amd as lt
        s = self.streams[slot]
        rays = {k: v[lo:hi] for k, v in r.payload.items()}
        out = self.outputs.get(r.rid)
        with self.torch.cuda.stream(s):
            if self.mode == "map":
                o = lt.lt_map_eval(self.maps[r.lens], self.dtype, rays, None, hi - lo, s)
            else:
                o = lt.lt_trace(self.lenses[r.lens], (0, 0, 0), rays, None, hi - lo, s)
            ev = self.torch.cuda.Event(enable_timing=True)
            ev.record(s)
        if out is not None:
            out.append((lo, hi, o))
        self.events[slot] = ev

    def done(self, slot) -> bool:
        ev = self.events[slot]
        return ev is None or ev.query()

    def finish_time(self, slot) -> float:
        return self.t0_event.elapsed_time(self.events[slot]) * 1e-3

    def wait(self, next_arrival):
        pass


def poisson_requests(n_req: int, rate_per_s: float, n_lenses: int, seed: int,
                     min_rays: int = 1000, max_rays: int = 1000000) -> List[Request]:
    """Poisson arrivals; sizes log-uniform in [min_rays, max_rays]; lens
    uniform.  Deterministic for a seed."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, n_req)
    t = np.cumsum(gaps)
    sizes = np.round(np.exp(rng.uniform(np.log(min_rays), np.log(max_rays), n_req))).astype(int)
    lens = rng.integers(0, n_lenses, n_req)
    return [Request(i, int(lens[i]), int(sizes[i]), float(t[i])) for i in range(n_req)]


def latency_stats(done: List[Request]) -> Dict[str, float]:
    import numpy as np
    lat = np.array([r.latency for r in done])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "n": len(done)}

"""Continuous-batching trace server over several resident scenes.

Scenes (surfels + their BVHs) stay resident on the device.  Requests -- a
scene index plus a batch of rays already on the device, of any size -- arrive
at any time.  The loop

  * admits queued requests in arrival order while the output memory they need
    fits the budget (a fixed byte count or a fraction of free device memory)
    and a launch slot is free; a request that could never fit is rejected;
  * packs every admitted request into one persistent launch
    (``irgs_trace_packed``: all requests' rays, across scenes, drained by one
    grid), alternating two streams so that a launch can start while the
    previous one is still finishing -- requests that arrive while others are
    on the device join the next launch instead of waiting for the whole queue;
  * polls launch events without blocking, completes requests, frees their
    budget and records arrival -> completion latency.

The packed kernel runs each ray through exactly the same code as a single
trace, so a request's result is bit-identical alone or in any mix.

``Scheduler`` holds the host-side policy (admission, budget, bookkeeping)
and is independent of the GPU; ``Server`` drives it with device launches.
"""
from __future__ import annotations

import collections
import dataclasses
import itertools
import time
from typing import Callable, Deque, List, Optional, Sequence

QUEUED, ADMITTED, RUNNING, DONE, REJECTED, CANCELLED = ("queued", "admitted", "running", "done", "rejected",
                                                       "cancelled")


@dataclasses.dataclass(eq=False)
class Request:
    id: int
    scene: int
    n_rays: int
    ro: object = None
    rd: object = None
    arrival: float = 0.0
    admitted_at: Optional[float] = None
    launched_at: Optional[float] = None
    done_at: Optional[float] = None
    status: str = QUEUED
    error: Optional[str] = None
    result: object = None
    nbytes: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_at is None else self.done_at - self.arrival


class Scheduler:
    """Admission and budget bookkeeping (no device work).

    budget_bytes  -- bytes of outputs the admitted and running requests may
                     hold at once
    bytes_per_ray -- output bytes one ray needs
    max_launch_rays -- cap on the rays of one packed launch
    """

    def __init__(self, n_scenes: int, budget_bytes: int, bytes_per_ray: int, max_launch_rays: int = 1 << 25):
        if budget_bytes <= 0 or bytes_per_ray <= 0:
            raise ValueError("budget_bytes and bytes_per_ray must be positive")
        self.n_scenes = n_scenes
        self.budget = int(budget_bytes)
        self.bytes_per_ray = int(bytes_per_ray)
        self.max_launch_rays = int(max_launch_rays)
        self.used = 0
        self.peak_used = 0
        self.queue: Deque[Request] = collections.deque()
        self._ids = itertools.count()

    def new_request(self, scene: int, n_rays: int, ro=None, rd=None, arrival: Optional[float] = None) -> Request:
        r = Request(next(self._ids), int(scene), int(n_rays), ro, rd,
                    time.perf_counter() if arrival is None else arrival)
        r.nbytes = r.n_rays * self.bytes_per_ray
        if not (0 <= r.scene < self.n_scenes):
            r.status, r.error = REJECTED, f"unknown scene {scene}"
        elif r.n_rays < 0:
            r.status, r.error = REJECTED, "negative ray count"
        elif r.nbytes > self.budget or r.n_rays > self.max_launch_rays:
            r.status, r.error = REJECTED, "request larger than the memory budget or launch cap"
        else:
            self.queue.append(r)
        return r

    def cancel(self, r: Request) -> bool:
        if r.status == QUEUED:
            self.queue.remove(r)
            r.status = CANCELLED
            return True
        return False

    def admit(self, now: float) -> List[Request]:
        """Admit requests in arrival order while they fit (budget and launch
        cap); the first that does not fit stops admission (no overtaking, so
        a large request is never starved)."""
        out, rays = [], 0
        while self.queue:
            r = self.queue[0]
            if self.used + r.nbytes > self.budget or rays + r.n_rays > self.max_launch_rays:
                break
            self.queue.popleft()
            self.used += r.nbytes
            self.peak_used = max(self.peak_used, self.used)
            rays += r.n_rays
            r.status, r.admitted_at = ADMITTED, now
            out.append(r)
        return out

    def release(self, r: Request) -> None:
        self.used -= r.nbytes
        assert self.used >= 0


class Server:
    """Device side: resident scenes, packed launches on alternating streams.

    scenes        -- list of built ``Scene`` objects (same alpha_min/sigma)
    budget_bytes  -- output-memory budget; default `budget_frac` of the free
                     device memory at construction
    executor      -- optional callable(requests, stream) that launches them
                     (for tests); the default uses ``trace_packed``
    """

    def __init__(self, scenes: Sequence, cfg=None, budget_bytes: Optional[int] = None, budget_frac: float = 0.5,
                 max_inflight: int = 2, max_launch_rays: int = 1 << 25,
                 executor: Optional[Callable] = None):
        import torch
        from .tracer import TraceConfig
        self.torch = torch
        self.scenes = list(scenes)
        if not self.scenes:
            raise ValueError("no scenes")
        self.cfg = cfg or TraceConfig()
        self.F = max(s.F for s in self.scenes)
        self.device = self.scenes[0].device
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(free * budget_frac)
        self.sched = Scheduler(len(self.scenes), budget_bytes, 4 * (self.F + 4), max_launch_rays)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(max_inflight)]
        self.max_inflight = max_inflight
        self.inflight: Deque = collections.deque()  # (event, requests, stream index)
        self._next_stream = 0
        self.executor = executor or self._launch_packed
        self.completed: List[Request] = []
        self.launches = 0

    # ---------------------------------------------------------------- API
    def submit(self, scene: int, ro, rd, arrival: Optional[float] = None) -> Request:
        n = int(ro.shape[0]) if ro is not None else 0
        r = self.sched.new_request(scene, n, ro, rd, arrival)
        if r.status == QUEUED:
            err = self._check_rays(r)
            if err:
                self.sched.queue.remove(r)
                r.status, r.error = REJECTED, err
        if r.status == REJECTED:
            r.done_at = time.perf_counter()
            self.completed.append(r)
        return r

    def cancel(self, r: Request) -> bool:
        return self.sched.cancel(r)

    def poll(self) -> int:
        """One non-blocking turn of the loop: retire finished launches, admit,
        launch.  Returns the number of requests completed in this turn."""
        done = 0
        while self.inflight and self.inflight[0][0].query():
            _, reqs, _ = self.inflight.popleft()
            now = time.perf_counter()
            for r in reqs:
                r.status, r.done_at = DONE, now
                self.sched.release(r)
                self.completed.append(r)
                done += 1
        if len(self.inflight) < self.max_inflight:
            reqs = self.sched.admit(time.perf_counter())
            if reqs:
                self._launch(reqs)
        return done

    def pending(self) -> int:
        return len(self.sched.queue) + sum(len(x[1]) for x in self.inflight)

    def drain(self, timeout: float = 600.0) -> None:
        t0 = time.perf_counter()
        while self.pending():
            if not self.poll():
                time.sleep(1e-4)
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")

    # ---------------------------------------------------------------- device
    def _check_rays(self, r: Request) -> Optional[str]:
        torch = self.torch
        for t, nm in ((r.ro, "ro"), (r.rd, "rd")):
            if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float32 \
                    or t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous() or t.shape[0] != r.n_rays:
                return f"{nm} must be a contiguous (R, 3) float32 tensor on {self.device}"
        return None

    def _launch(self, reqs: List[Request]) -> None:
        torch = self.torch
        si = self._next_stream
        self._next_stream = (si + 1) % self.max_inflight
        stream = self.streams[si]
        now = time.perf_counter()
        for r in reqs:
            r.status, r.launched_at = RUNNING, now
        with torch.cuda.stream(stream):
            self.executor(reqs, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.inflight.append((ev, reqs, si))
        self.launches += 1

    def _launch_packed(self, reqs: List[Request], stream) -> None:
        from .tracer import alloc_result, trace_packed
        items = []
        for r in reqs:
            # the rays were produced on the caller's stream: order this launch after them
            r.result = alloc_result(r.n_rays, self.scenes[r.scene].F, self.device, 0)
            items.append((r.scene, r.ro, r.rd, r.result))
        stream.wait_stream(self.torch.cuda.default_stream(self.device))
        trace_packed(self.scenes, items, self.cfg)


def run_open_loop(server: Server, arrivals: Sequence[float], make_request: Callable[[int], tuple],
                  poll_sleep: float = 5e-5) -> List[Request]:
    """Submit request i at time arrivals[i] (seconds after start; open loop),
    polling the server in between; returns the requests in submission order."""
    t0 = time.perf_counter()
    reqs = []
    i = 0
    n = len(arrivals)
    while i < n or server.pending():
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            scene, ro, rd = make_request(i)
            reqs.append(server.submit(scene, ro, rd, arrival=t0 + arrivals[i]))
            i += 1
        if not server.poll():
            time.sleep(poll_sleep)
    return reqs


def run_per_request(scenes: Sequence, cfg, arrivals: Sequence[float], make_request: Callable[[int], tuple],
                    poll_sleep: float = 5e-5) -> List[Request]:
    """Baseline: one plain trace launch per request, FIFO on one stream, the
    same open-loop arrivals."""
    import torch
    from .tracer import trace
    dev = scenes[0].device
    stream = torch.cuda.Stream(dev)
    t0 = time.perf_counter()
    reqs: List[Request] = []
    inflight: Deque = collections.deque()
    i, n = 0, len(arrivals)
    while i < n or inflight:
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            scene, ro, rd = make_request(i)
            r = Request(i, scene, int(ro.shape[0]), ro, rd, t0 + arrivals[i])
            stream.wait_stream(torch.cuda.default_stream(dev))
            with torch.cuda.stream(stream):
                r.result = trace(scenes[scene], ro, rd, cfg)
                ev = torch.cuda.Event()
                ev.record(stream)
            r.status, r.launched_at = RUNNING, time.perf_counter()
            inflight.append((ev, r))
            reqs.append(r)
            i += 1
        progressed = False
        while inflight and inflight[0][0].query():
            _, r = inflight.popleft()
            r.status, r.done_at = DONE, time.perf_counter()
            progressed = True
        if not progressed:
            time.sleep(poll_sleep)
    return reqs


def latency_stats(reqs: Sequence[Request]) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in reqs if r.status == DONE])
    done = [r for r in reqs if r.status == DONE]
    if not len(lat):
        return dict(n=0)
    span = max(r.done_at for r in done) - min(r.arrival for r in done)
    rays = sum(r.n_rays for r in done)
    return dict(n=len(lat), p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3), rays=int(rays), span_s=float(span),
                mrays_s=float(rays / span / 1e6))

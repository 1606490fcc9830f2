"""Continuous-batching trace server over several resident scenes.

Scenes (surfels + their BVHs) stay resident on the device.  Requests -- a
scene index plus a batch of rays already on the device, of any size -- arrive
at any time.  The loop

  * admits queued requests in arrival order while the output memory they
    need fits the budget; the budget first sets aside the scratch of every
    launch that may be in flight (the packed launch's per-thread stack
    overflow and deferred lists, ``irgs_trace_bytes``); a request that could
    never fit is rejected;
  * splits every admitted request into work items of at most ``chunk_rays``
    rays and builds each launch from the items of all admitted requests in
    turn (one item per request per turn), up to ``max_launch_rays``, so that
    a small request that arrives while a large one is being traced rides in
    the next launch instead of waiting for the large one to finish;
  * runs each launch as one persistent packed trace (``irgs_trace_packed``:
    items of different requests and scenes drained by one grid) on
    alternating streams, so that one launch starts while the previous one is
    still draining its last rays;
  * polls launch events without blocking: a request completes when the
    launches holding all of its items have finished (not the launches of
    other requests), frees its budget and records arrival -> completion
    latency.

The packed kernel runs each ray through exactly the same code as a single
trace, so a request's result is bit-identical alone or in any mix, whatever
its split into items.

``Scheduler`` holds the host-side policy (admission, budget, splitting,
turn order, bookkeeping) and is independent of the GPU; ``Server`` drives it
with device launches.
"""
from __future__ import annotations

import collections
import dataclasses
import itertools
import time
from typing import Callable, Deque, List, Optional, Sequence, Tuple

QUEUED, ADMITTED, RUNNING, DONE, REJECTED, CANCELLED = ("queued", "admitted", "running", "done", "rejected",
                                                       "cancelled")

CHUNK_RAYS = 65536          # rays per work item
MAX_LAUNCH_RAYS = 1 << 21   # rays per packed launch


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
    next_ray: int = 0        # first ray not yet placed in a launch
    rays_left: int = 0       # rays whose launch has not finished yet
    launches: int = 0        # launches that carried items of this request

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_at is None else self.done_at - self.arrival


# One work item: rays [begin, begin + count) of a request.
Item = Tuple[Request, int, int]


class Scheduler:
    """Admission, splitting and bookkeeping (no device work).

    budget_bytes    -- bytes of outputs the admitted and running requests may
                       hold at once
    bytes_per_ray   -- output bytes one ray needs
    chunk_rays      -- rays per work item
    max_launch_rays -- cap on the rays of one launch
    """

    def __init__(self, n_scenes: int, budget_bytes: int, bytes_per_ray: int, chunk_rays: int = CHUNK_RAYS,
                 max_launch_rays: int = MAX_LAUNCH_RAYS):
        if budget_bytes <= 0 or bytes_per_ray <= 0:
            raise ValueError("budget_bytes and bytes_per_ray must be positive")
        if chunk_rays <= 0 or max_launch_rays <= 0:
            raise ValueError("chunk_rays and max_launch_rays must be positive")
        self.n_scenes = n_scenes
        self.budget = int(budget_bytes)
        self.bytes_per_ray = int(bytes_per_ray)
        self.chunk_rays = int(chunk_rays)
        self.max_launch_rays = int(max_launch_rays)
        self.used = 0
        self.peak_used = 0
        self.queue: Deque[Request] = collections.deque()   # waiting for admission
        self.active: Deque[Request] = collections.deque()  # admitted, with rays not yet in a launch
        self._ids = itertools.count()

    def new_request(self, scene: int, n_rays: int, ro=None, rd=None, arrival: Optional[float] = None) -> Request:
        r = Request(next(self._ids), int(scene), int(n_rays), ro, rd,
                    time.perf_counter() if arrival is None else arrival)
        r.nbytes = max(r.n_rays, 0) * self.bytes_per_ray
        r.rays_left = max(r.n_rays, 0)
        if not (0 <= r.scene < self.n_scenes):
            r.status, r.error = REJECTED, f"unknown scene {scene}"
        elif r.n_rays < 0:
            r.status, r.error = REJECTED, "negative ray count"
        elif r.nbytes > self.budget:
            r.status, r.error = REJECTED, "request larger than the memory budget"
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
        """Admit requests in arrival order while their outputs fit the budget;
        the first that does not fit stops admission (no overtaking, so a
        large request is never starved)."""
        out = []
        while self.queue:
            r = self.queue[0]
            if self.used + r.nbytes > self.budget:
                break
            self.queue.popleft()
            self.used += r.nbytes
            self.peak_used = max(self.peak_used, self.used)
            r.status, r.admitted_at = ADMITTED, now
            self.active.append(r)
            out.append(r)
        return out

    def next_launch(self) -> List[Item]:
        """Work items of the next launch: one item (up to chunk_rays rays) from
        each active request in turn, until the launch holds max_launch_rays
        rays or no rays are left.  The turn order carries over between
        launches; a request leaves it once all its rays are placed."""
        items: List[Item] = []
        rays = 0
        while self.active and rays < self.max_launch_rays:
            r = self.active.popleft()
            n = min(self.chunk_rays, r.n_rays - r.next_ray, self.max_launch_rays - rays)
            if n > 0 or r.n_rays == 0:
                items.append((r, r.next_ray, n))
                r.next_ray += n
                rays += n
            if r.next_ray < r.n_rays:
                self.active.append(r)
        return items

    def item_done(self, r: Request, count: int) -> bool:
        """Account a finished item; True when it was the request's last."""
        r.rays_left -= count
        assert r.rays_left >= 0
        return r.rays_left == 0 and r.next_ray >= r.n_rays

    def release(self, r: Request) -> None:
        self.used -= r.nbytes
        assert self.used >= 0


class Server:
    """Device side: resident scenes, packed launches on alternating streams.

    scenes          -- list of built ``Scene`` objects (same alpha_min/sigma)
    budget_bytes    -- device bytes for outputs and launch scratch; default
                       `budget_frac` of the free device memory at
                       construction
    chunk_rays, max_launch_rays -- work-item and launch sizes
    hit_cap         -- also keep each ray's first hit_cap hit ids and the
                       transmittance before each (0: none)
    executor        -- optional callable(items, stream) that launches them
                       (for tests); the default uses ``trace_packed``
    """

    def __init__(self, scenes: Sequence, cfg=None, budget_bytes: Optional[int] = None, budget_frac: float = 0.5,
                 max_inflight: int = 2, chunk_rays: int = CHUNK_RAYS, max_launch_rays: int = MAX_LAUNCH_RAYS,
                 hit_cap: int = 0, executor: Optional[Callable] = None):
        import torch
        from . import _lib
        from .tracer import TraceConfig
        self.torch = torch
        self.scenes = list(scenes)
        if not self.scenes:
            raise ValueError("no scenes")
        self.cfg = cfg or TraceConfig()
        self.F = max(s.F for s in self.scenes)
        self.device = self.scenes[0].device
        self.hit_cap = int(hit_cap)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(free * budget_frac)
        # every launch in flight holds the packed launch's scratch (sized for
        # its grid, at most that of a max_launch_rays launch)
        self.scratch_bytes = max_inflight * int(_lib.lib().irgs_trace_bytes(int(max_launch_rays), self.F, 0))
        out_budget = int(budget_bytes) - self.scratch_bytes
        if out_budget <= 0:
            raise ValueError(f"budget of {budget_bytes} bytes does not cover the launch scratch "
                             f"({self.scratch_bytes} bytes for {max_inflight} launches in flight)")
        bytes_per_ray = 4 * (self.F + 4) + 8 * self.hit_cap
        self.sched = Scheduler(len(self.scenes), out_budget, bytes_per_ray, chunk_rays, max_launch_rays)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(max_inflight)]
        self.max_inflight = max_inflight
        self.inflight: Deque = collections.deque()  # (event, items)
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
        """One non-blocking turn of the loop: retire finished launches
        (completing the requests whose last items they held), admit, launch.
        Returns the number of requests completed in this turn."""
        done = 0
        while self.inflight and self.inflight[0][0].query():
            _, items = self.inflight.popleft()
            now = time.perf_counter()
            for r, _, n in items:
                if self.sched.item_done(r, n):
                    r.status, r.done_at = DONE, now
                    self.sched.release(r)
                    self.completed.append(r)
                    done += 1
        if len(self.inflight) < self.max_inflight:
            for r in self.sched.admit(time.perf_counter()):
                self._alloc(r)
            items = self.sched.next_launch()
            if items:
                self._launch(items)
        return done

    def pending(self) -> int:
        return len(self.sched.queue) + len(self.sched.active) + sum(len(x[1]) for x in self.inflight)

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

    def _alloc(self, r: Request) -> None:
        from .tracer import alloc_result
        r.result = alloc_result(r.n_rays, self.scenes[r.scene].F, self.device, self.hit_cap)

    def _launch(self, items: List[Item]) -> None:
        torch = self.torch
        si = self._next_stream
        self._next_stream = (si + 1) % self.max_inflight
        stream = self.streams[si]
        now = time.perf_counter()
        for r, _, _ in items:
            if r.status == ADMITTED:
                r.status, r.launched_at = RUNNING, now
            r.launches += 1
        # the rays and the outputs were made on the caller's stream: order
        # this launch after them
        stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(stream):
            self.executor(items, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.inflight.append((ev, items))
        self.launches += 1

    def _launch_packed(self, items: List[Item], stream) -> None:
        from .tracer import trace_packed
        trace_packed(self.scenes, [(r.scene, r.ro, r.rd, r.result, b, n) for r, b, n in items], self.cfg)


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

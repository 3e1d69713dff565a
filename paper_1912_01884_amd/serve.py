"""Continuous-batching detection server on one GPU.

Requests (a device image, k and a bend restriction) arrive at any time.  The
server owns one device arena, sized at start from the free HBM the device
reports, and a few streams.  Each call of ``poll``

  1. retires every in-flight group whose completion event has fired, which
     frees its arena block and stream;
  2. admits waiting requests in arrival order into one group, as many as fit
     the largest free arena block (their band tables, DP planes and
     back-pointers stay resident there until the group retires) and the group
     size limit;
  3. launches that group as ONE batched detection (fhtp_detect_batch) on a
     free stream and records its completion event.

So requests that arrive while others run are admitted as soon as a stream
and memory free up, and groups on different streams overlap on the device.
Admission is first come, first served: a request that does not fit waits
(backpressure) and holds back those behind it; a request larger than the
whole arena is rejected at submit.  Results are the library's, bit for bit:
batching changes which launches an image shares, not its arithmetic.

The scheduling logic is independent of the GPU: ``Server`` talks to a
backend with four methods (request_bytes, launch, done, capacity), so the
tests drive it on the CPU with a simulated backend.  ``FhtpBackend`` is the
real one; ``PlainServer`` is the one-request-at-a-time reference path.
"""

from __future__ import annotations

import bisect
import collections
import ctypes as C
import gc
import math
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, List, Optional, Tuple

ALIGN = 256


def align_up(v: int) -> int:
    return (v + ALIGN - 1) // ALIGN * ALIGN


@dataclass
class Request:
    """One detection: inputs and preallocated outputs are device tensors."""

    img: Any                      # device [h][w] uint8 / uint16
    k: int
    bend: Optional[int] = None    # shift bound (mode 0) ...
    gamma: Optional[float] = None  # ... or angle bound (mode 1)
    score: Any = None             # device int32[1], written by the detection
    xs: Any = None                # device int32[k+1]
    rid: int = -1
    arrival: float = math.nan     # seconds on the load generator's clock
    admitted: float = math.nan
    done: float = math.nan
    nbytes: int = 0               # arena bytes while in flight
    error: Optional[str] = None
    producer: Any = None          # stream current at submit (GPU backends), waited on at launch

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Arena:
    """First-fit allocator of 256-byte aligned blocks in [0, capacity)."""

    def __init__(self, capacity: int):
        self.capacity = capacity - capacity % ALIGN
        self._starts: List[int] = [0] if self.capacity > 0 else []
        self._sizes: List[int] = [self.capacity] if self.capacity > 0 else []
        self.used = 0

    def largest_free(self) -> int:
        return max(self._sizes, default=0)

    def alloc(self, nbytes: int) -> Optional[int]:
        n = align_up(max(nbytes, 1))
        for i, sz in enumerate(self._sizes):
            if sz >= n:
                off = self._starts[i]
                if sz == n:
                    del self._starts[i]
                    del self._sizes[i]
                else:
                    self._starts[i] += n
                    self._sizes[i] -= n
                self.used += n
                return off
        return None

    def free(self, off: int, nbytes: int) -> None:
        n = align_up(max(nbytes, 1))
        i = bisect.bisect_left(self._starts, off)
        if i < len(self._starts) and self._starts[i] < off + n:
            raise ValueError("double free or overlap in arena")
        if i > 0 and self._starts[i - 1] + self._sizes[i - 1] > off:
            raise ValueError("double free or overlap in arena")
        self._starts.insert(i, off)
        self._sizes.insert(i, n)
        self.used -= n
        # coalesce with the right, then the left neighbour
        if i + 1 < len(self._starts) and self._starts[i] + self._sizes[i] == self._starts[i + 1]:
            self._sizes[i] += self._sizes.pop(i + 1)
            self._starts.pop(i + 1)
        if i > 0 and self._starts[i - 1] + self._sizes[i - 1] == self._starts[i]:
            self._sizes[i - 1] += self._sizes.pop(i)
            self._starts.pop(i)

    def free_blocks(self) -> List[Tuple[int, int]]:
        return list(zip(self._starts, self._sizes))


@dataclass
class _Group:
    reqs: List[Request]
    offset: int
    nbytes: int
    stream: int
    handle: Any


class Server:
    """Continuous batching over a backend (see the module docstring)."""

    def __init__(self, backend, streams: int = 4, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter):
        if streams < 1 or max_batch < 1:
            raise ValueError("need at least one stream and a group size of at least one")
        self.backend = backend
        self.arena = Arena(backend.capacity())
        self.n_streams = streams
        self.max_batch = max_batch
        self.clock = clock
        self.waiting: Deque[Request] = collections.deque()
        self.inflight: List[_Group] = []
        self._free_streams = list(range(streams))
        self.groups_launched = 0
        self.rejected = 0

    def submit(self, req: Request) -> bool:
        """Queue a request; False (with req.error set) if it can never fit the arena."""
        req.nbytes = align_up(self.backend.request_bytes(req))
        if req.nbytes > self.arena.capacity:
            req.error = (f"request needs {req.nbytes} bytes of device memory, the arena holds "
                         f"{self.arena.capacity}")
            self.rejected += 1
            return False
        on_submit = getattr(self.backend, "on_submit", None)
        if on_submit is not None:
            on_submit(req)
        self.waiting.append(req)
        return True

    def idle(self) -> bool:
        return not self.waiting and not self.inflight

    def poll(self) -> List[Request]:
        """Retire finished groups, then admit and launch; returns the requests finished now."""
        finished: List[Request] = []
        still = []
        for g in self.inflight:
            if self.backend.done(g.handle):
                now = self.clock()
                self.arena.free(g.offset, g.nbytes)
                self._free_streams.append(g.stream)
                for r in g.reqs:
                    r.done = now
                finished.extend(g.reqs)
            else:
                still.append(g)
        self.inflight = still
        while self.waiting and self._free_streams:
            if not self._launch_one():
                break
        return finished

    def _launch_one(self) -> bool:
        room = self.arena.largest_free()
        take: List[Request] = []
        total = 0
        for r in self.waiting:
            if len(take) == self.max_batch or total + r.nbytes > room:
                break
            take.append(r)
            total += r.nbytes
        if not take:
            return False  # the head waits for memory (backpressure)
        for _ in take:
            self.waiting.popleft()
        off = self.arena.alloc(total)
        assert off is not None
        stream = self._free_streams.pop(0)
        now = self.clock()
        for r in take:
            r.admitted = now
        try:
            handle = self.backend.launch(take, off, total, stream)
        except BaseException:
            # nothing of the group runs: give back its memory and stream and
            # put its requests back at the head of the queue, in order
            self.arena.free(off, total)
            self._free_streams.insert(0, stream)
            for r in reversed(take):
                r.admitted = math.nan
                self.waiting.appendleft(r)
            raise
        self.inflight.append(_Group(take, off, total, stream, handle))
        self.groups_launched += 1
        return True

    def drain(self, timeout: float = 60.0) -> List[Request]:
        """Poll until nothing waits or runs."""
        out: List[Request] = []
        t_end = self.clock() + timeout
        while not self.idle():
            out.extend(self.poll())
            if self.clock() > t_end:
                raise TimeoutError("server did not drain in time")
        return out


# ---- the GPU backend ---------------------------------------------------------

def request_bytes_cached(F, cache: dict, r: Request) -> int:
    """fhtp_detect_workspace_bytes of a request, looked up once per shape
    (pixel type, h, w, k, bend restriction)."""
    h, w = r.img.shape
    key = (r.img.dtype, h, w, r.k, r.bend, r.gamma)
    n = cache.get(key)
    if n is None:
        n = F.detect_workspace_bytes(F._dtype_code(r.img), h, w, r.k, F.make_bend(r.bend, r.gamma))
        cache[key] = n
    return n


def order_after_submitter(torch, s, reqs: List[Request], device) -> None:
    """Order the detections on stream `s` after the request tensors' producers.

    The images, scores and vertex buffers may have been filled or allocated
    asynchronously on the stream that was current when the request was
    submitted (`Request.producer`): `s` waits for each such stream that still
    has work queued, once per distinct stream (without a recorded producer,
    for the stream current now).
    The tensors themselves cannot be freed while the detection runs: the
    server holds its requests until their completion event has fired.
    """
    seen = set()
    for r in reqs:
        p = r.producer if r.producer is not None else torch.cuda.current_stream(device)
        if p.cuda_stream not in seen:
            seen.add(p.cuda_stream)
            # a producer with nothing left to run has finished every tensor
            # submitted before now: no event needed
            if not p.query():
                s.wait_stream(p)


class FhtpBackend:
    """Arena in device memory, streams and events; groups run fhtp_detect_batch."""

    def __init__(self, device=None, arena_bytes: Optional[int] = None, streams: int = 4,
                 free_fraction: float = 0.5, warmup: bool = True):
        import torch

        from . import fhtp
        self.torch = torch
        self.fhtp = fhtp
        self.L = fhtp.lib()
        self.device = torch.device("cuda:0") if device is None else torch.device(device)
        free, _total = torch.cuda.mem_get_info(self.device)
        budget = int(free * free_fraction)
        size = budget if arena_bytes is None else min(int(arena_bytes), budget)
        size -= size % ALIGN
        if size <= 0:
            raise RuntimeError("no device memory available for the arena")
        self.arena = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.base = self.arena.data_ptr()
        self._bytes: dict = {}  # workspace bytes per request shape
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        # one completion event per stream: a stream carries one group at a time
        # (the server frees it only after its group's event has fired), so the
        # event is re-recorded for each group instead of created anew
        self.events = [torch.cuda.Event() for _ in range(streams)]
        # the arena's allocation is ordered before any group on any stream
        torch.cuda.synchronize(self.device)
        if warmup:
            self.warmup()

    def warmup(self) -> None:
        """Run one tiny batch on every stream before serving.

        The batch mixes an image whose bands take the second-stream path (256
        rows) with one that does not (64 rows), so the library creates the
        second stream it keeps for each of this backend's streams now, and
        loads its kernels, instead of during the first groups served (each
        such first use stalls the host for milliseconds).
        """
        torch, F = self.torch, self.fhtp
        imgs = [torch.zeros((256, 1), dtype=torch.uint8, device=self.device),
                torch.zeros((64, 1), dtype=torch.uint8, device=self.device)]
        scores = [torch.zeros(1, dtype=torch.int32, device=self.device) for _ in imgs]
        xss = [torch.zeros(2, dtype=torch.int32, device=self.device) for _ in imgs]
        jobs, _keep = F.make_jobs(imgs, [1, 1], bends=[0, 0], scores=scores, xss=xss)
        nbytes = F.batch_workspace_bytes(jobs)
        if nbytes > self.arena.numel():
            return
        arr = (F.Job * len(jobs))(*jobs)
        for s in self.streams:
            rc = self.L.fhtp_detect_batch(arr, len(jobs), C.c_void_p(self.base), nbytes,
                                          C.c_void_p(s.cuda_stream))
            F._check(rc, "detect_batch")
            # the next stream's batch reuses the same arena bytes
            s.synchronize()
        torch.cuda.synchronize(self.device)

    def capacity(self) -> int:
        return self.arena.numel()

    def on_submit(self, r: Request) -> None:
        r.producer = self.torch.cuda.current_stream(self.device)

    def _job(self, r: Request):
        F = self.fhtp
        h, w = r.img.shape
        b = F.make_bend(r.bend, r.gamma)
        return F.Job(r.img.data_ptr(), F._dtype_code(r.img), h, w, r.k, b, r.score.data_ptr(),
                     r.xs.data_ptr())

    def request_bytes(self, r: Request) -> int:
        return request_bytes_cached(self.fhtp, self._bytes, r)

    def launch(self, reqs: List[Request], offset: int, nbytes: int, stream: int):
        jobs = [self._job(r) for r in reqs]
        arr = (self.fhtp.Job * len(jobs))(*jobs)
        s = self.streams[stream]
        order_after_submitter(self.torch, s, reqs, self.device)
        rc = self.L.fhtp_detect_batch(arr, len(jobs), C.c_void_p(self.base + offset), nbytes,
                                      C.c_void_p(s.cuda_stream))
        self.fhtp._check(rc, "detect_batch")
        ev = self.events[stream]
        ev.record(s)
        return ev

    def done(self, handle) -> bool:
        return handle.query()


class PlainServer:
    """Reference path: one request at a time with fhtp_detect_polyline, in arrival order."""

    def __init__(self, device=None, max_request_bytes: int = 0,
                 clock: Callable[[], float] = time.perf_counter):
        import torch

        from . import fhtp
        self.torch = torch
        self.fhtp = fhtp
        self.L = fhtp.lib()
        self.device = torch.device("cuda:0") if device is None else torch.device(device)
        self.ws = torch.empty(max(align_up(max_request_bytes), ALIGN), dtype=torch.uint8,
                              device=self.device)
        self.stream = torch.cuda.Stream(self.device)
        self.event = torch.cuda.Event()
        self._bytes: dict = {}  # workspace bytes per request shape
        self.clock = clock
        self.waiting: Deque[Request] = collections.deque()
        self.current: Optional[Tuple[Request, Any]] = None
        torch.cuda.synchronize(self.device)

    def submit(self, req: Request) -> bool:
        req.nbytes = request_bytes_cached(self.fhtp, self._bytes, req)
        if req.nbytes > self.ws.numel():
            req.error = "request larger than the workspace"
            return False
        req.producer = self.torch.cuda.current_stream(self.device)
        self.waiting.append(req)
        return True

    def idle(self) -> bool:
        return not self.waiting and self.current is None

    def poll(self) -> List[Request]:
        out = []
        if self.current is not None and self.current[1].query():
            r = self.current[0]
            r.done = self.clock()
            out.append(r)
            self.current = None
        if self.current is None and self.waiting:
            r = self.waiting.popleft()
            r.admitted = self.clock()
            F = self.fhtp
            h, w = r.img.shape
            order_after_submitter(self.torch, self.stream, [r], self.device)
            rc = self.L.fhtp_detect_polyline(
                C.c_void_p(r.img.data_ptr()), F._dtype_code(r.img), h, w, r.k,
                F.make_bend(r.bend, r.gamma), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                C.c_void_p(r.score.data_ptr()), C.c_void_p(r.xs.data_ptr()),
                C.c_void_p(self.stream.cuda_stream))
            F._check(rc, "detect_polyline")
            self.event.record(self.stream)  # one request in flight at a time
            self.current = (r, self.event)
        return out

    def drain(self, timeout: float = 60.0) -> List[Request]:
        out: List[Request] = []
        t_end = self.clock() + timeout
        while not self.idle():
            out.extend(self.poll())
            if self.clock() > t_end:
                raise TimeoutError("plain server did not drain in time")
        return out


# ---- open-loop driver ----------------------------------------------------------

def poisson_arrivals(rate: float, count: int, seed) -> List[float]:
    """Arrival times (s) of a Poisson stream: exponential gaps of mean 1/rate."""
    import numpy as np
    rng = np.random.default_rng(seed)
    if math.isinf(rate):
        return [0.0] * count
    return np.cumsum(rng.exponential(1.0 / rate, size=count)).tolist()


def run_open_loop(server, requests: List[Request], arrivals: List[float],
                  timeout: float = 120.0) -> dict:
    """Submit each request at its arrival time (relative to now) and poll until all finish.

    Latency is completion (observed by the host) minus the scheduled arrival,
    so any lag of the loop itself counts against the server.  Python's cyclic
    garbage collector is paused for the run (its pauses would land in the
    tail of whichever request was in flight); it runs again afterwards.
    """
    enabled = gc.isenabled()
    gc.disable()
    try:
        return _open_loop(server, requests, arrivals, timeout)
    finally:
        if enabled:
            gc.enable()


def _open_loop(server, requests: List[Request], arrivals: List[float], timeout: float) -> dict:
    clock = server.clock
    t0 = clock()
    order = sorted(range(len(requests)), key=lambda i: arrivals[i])
    i = 0
    finished = 0
    n = len(requests)
    rejected = 0
    while finished + rejected < n:
        now = clock()
        while i < n and arrivals[order[i]] <= now - t0:
            r = requests[order[i]]
            r.arrival = t0 + arrivals[order[i]]
            if not server.submit(r):
                rejected += 1
            i += 1
        finished += len(server.poll())
        if now - t0 > timeout:
            raise TimeoutError("open-loop run did not finish in time")
    t_end = max((r.done for r in requests if r.error is None), default=t0)
    lat = sorted(r.latency for r in requests if r.error is None)
    return summarize(lat, finished, t_end - t0, rejected)


def summarize(lat: List[float], finished: int, span: float, rejected: int = 0) -> dict:
    def pct(p):
        if not lat:
            return math.nan
        idx = min(len(lat) - 1, max(0, math.ceil(p / 100.0 * len(lat)) - 1))
        return lat[idx]
    return {"requests": finished, "rejected": rejected,
            "p50_ms": round(pct(50) * 1e3, 4), "p99_ms": round(pct(99) * 1e3, 4),
            "max_ms": round((lat[-1] if lat else math.nan) * 1e3, 4),
            "images_per_s": round(finished / span, 1) if span > 0 else math.nan,
            "span_s": round(span, 4)}

"""CPU tests of the serving loop's scheduling: arena, admission, backpressure, overlap.

The server is driven with a simulated backend and a simulated clock, so no
GPU is involved: launches finish after a set time, and every check is about
which requests run together, where their memory sits and when they finish.
"""

import math
import random
from types import SimpleNamespace

import pytest

from paper_1912_01884_amd.serve import (ALIGN, Arena, Request, Server, poisson_arrivals,
                                        run_open_loop, summarize)


class Clock:
    def __init__(self, step=0.0):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t


class SimBackend:
    """Groups take `per_group + per_request * len` seconds; checks arena and stream use."""

    def __init__(self, clock, capacity, per_group=1e-3, per_request=1e-4):
        self.clock = clock
        self.cap = capacity
        self.per_group = per_group
        self.per_request = per_request
        self.live = {}  # stream -> (offset, nbytes)
        self.launches = []
        self.max_concurrent = 0

    def capacity(self):
        return self.cap

    def request_bytes(self, r):
        return r.img.nbytes

    def launch(self, reqs, offset, nbytes, stream):
        assert stream not in self.live, "stream reused while busy"
        for s, (o, n) in self.live.items():
            assert offset + nbytes <= o or o + n <= offset, "arena blocks overlap"
        assert offset % ALIGN == 0 and offset + nbytes <= self.cap
        assert nbytes == sum(r.nbytes for r in reqs)
        self.live[stream] = (offset, nbytes)
        self.max_concurrent = max(self.max_concurrent, len(self.live))
        t_done = self.clock.t + self.per_group + self.per_request * len(reqs)
        self.launches.append([r.rid for r in reqs])
        return SimpleNamespace(t=t_done, stream=stream)

    def done(self, h):
        if self.clock.t >= h.t:
            self.live.pop(h.stream, None)
            return True
        return False


def _req(rid, nbytes):
    return Request(img=SimpleNamespace(nbytes=nbytes), k=4, bend=1, rid=rid)


# ---- arena ---------------------------------------------------------------------

def test_arena_first_fit_and_coalescing():
    a = Arena(10 * ALIGN + 17)
    assert a.capacity == 10 * ALIGN
    x = a.alloc(1)
    y = a.alloc(2 * ALIGN)
    z = a.alloc(ALIGN + 1)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert a.largest_free() == 5 * ALIGN
    a.free(y, 2 * ALIGN)
    assert a.alloc(ALIGN) == ALIGN  # first fit reuses the hole
    a.free(ALIGN, ALIGN)
    a.free(x, 1)
    a.free(z, ALIGN + 1)
    assert a.free_blocks() == [(0, 10 * ALIGN)] and a.used == 0
    assert a.alloc(11 * ALIGN) is None


def test_arena_rejects_double_free():
    a = Arena(4 * ALIGN)
    o = a.alloc(ALIGN)
    a.free(o, ALIGN)
    with pytest.raises(ValueError):
        a.free(o, ALIGN)


def test_arena_random_against_bitmap():
    rnd = random.Random(5)
    units = 64
    a = Arena(units * ALIGN)
    used = [False] * units
    live = []
    for _ in range(2000):
        if live and rnd.random() < 0.45:
            off, n = live.pop(rnd.randrange(len(live)))
            a.free(off, n)
            for u in range(off // ALIGN, (off + n) // ALIGN):
                used[u] = False
        else:
            n = rnd.randint(1, 8) * ALIGN
            off = a.alloc(n)
            # first fit: the lowest run of free units that is long enough
            want = None
            for s in range(units - n // ALIGN + 1):
                if not any(used[s:s + n // ALIGN]):
                    want = s * ALIGN
                    break
            assert off == want
            if off is not None:
                for u in range(off // ALIGN, (off + n) // ALIGN):
                    used[u] = True
                live.append((off, n))
        assert a.used == sum(used) * ALIGN


# ---- server --------------------------------------------------------------------

def test_everything_finishes_in_fifo_groups():
    clock = Clock()
    be = SimBackend(clock, capacity=1 << 20)
    srv = Server(be, streams=2, max_batch=4, clock=clock)
    reqs = [_req(i, 1000 + 37 * i) for i in range(10)]
    for r in reqs:
        assert srv.submit(r)
    done = []
    while not srv.idle():
        done += srv.poll()
        clock.t += 1e-4
    assert sorted(r.rid for r in done) == list(range(10))
    flat = [rid for g in be.launches for rid in g]
    assert flat == list(range(10))  # admission in arrival order
    assert max(len(g) for g in be.launches) <= 4
    assert be.max_concurrent == 2  # two groups overlapped
    assert all(r.admitted <= r.done for r in reqs)
    assert srv.arena.used == 0


def test_backpressure_holds_the_head_and_keeps_order():
    clock = Clock()
    cap = 10 * ALIGN
    be = SimBackend(clock, capacity=cap)
    srv = Server(be, streams=4, max_batch=8, clock=clock)
    sizes = [6, 6, 2, 9, 1]
    reqs = [_req(i, s * ALIGN) for i, s in enumerate(sizes)]
    for r in reqs:
        srv.submit(r)
    srv.poll()
    # request 0 runs; request 1 (6 units) does not fit beside it, and 2 may not overtake it
    assert be.launches == [[0]]
    assert [r.rid for r in srv.waiting] == [1, 2, 3, 4]
    order = []
    while not srv.idle():
        order += [r.rid for r in srv.poll()]
        clock.t += 1e-4
    flat = [rid for g in be.launches for rid in g]
    assert flat == [0, 1, 2, 3, 4]
    assert order == [0, 1, 2, 3, 4]


def test_oversized_request_is_rejected_at_submit():
    clock = Clock()
    be = SimBackend(clock, capacity=4 * ALIGN)
    srv = Server(be, clock=clock)
    big = _req(0, 5 * ALIGN)
    assert not srv.submit(big)
    assert big.error and "arena" in big.error and srv.rejected == 1
    ok = _req(1, 4 * ALIGN)
    assert srv.submit(ok)
    while not srv.idle():
        srv.poll()
        clock.t += 1e-3
    assert ok.done >= 0


def test_arrivals_during_a_group_start_a_second_group_on_another_stream():
    clock = Clock()
    be = SimBackend(clock, capacity=1 << 20, per_group=1.0)
    srv = Server(be, streams=2, clock=clock)
    srv.submit(_req(0, 100))
    srv.poll()
    clock.t = 0.1
    srv.submit(_req(1, 100))
    srv.submit(_req(2, 100))
    srv.poll()
    assert be.launches == [[0], [1, 2]]  # admitted while group 0 still runs
    assert be.max_concurrent == 2
    clock.t = 0.2
    srv.submit(_req(3, 100))
    srv.poll()
    assert be.launches == [[0], [1, 2]]  # no free stream yet: it waits
    clock.t = 1.05
    fin = srv.poll()
    assert [r.rid for r in fin] == [0]
    assert be.launches[-1] == [3]  # the freed stream takes the waiting request at once


def test_open_loop_driver_and_latency_summary():
    clock = Clock(step=1e-5)
    be = SimBackend(clock, capacity=1 << 24, per_group=2e-3, per_request=1e-4)
    srv = Server(be, streams=3, max_batch=16, clock=clock)
    arr = poisson_arrivals(2000.0, 300, [191201884, 5, 999])
    assert all(b >= a for a, b in zip(arr, arr[1:]))
    reqs = [_req(i, 4096) for i in range(300)]
    res = run_open_loop(srv, reqs, arr)
    assert res["requests"] == 300 and res["rejected"] == 0
    lat = sorted(r.latency for r in reqs)
    assert lat[0] >= 2e-3  # at least one group's duration
    assert res["p50_ms"] <= res["p99_ms"] <= res["max_ms"]
    assert res["images_per_s"] > 0
    # under load the server batches: fewer groups than requests
    assert len(be.launches) < 300


def test_summary_percentiles():
    lat = [i / 1000 for i in range(1, 101)]  # 1..100 ms
    s = summarize(lat, 100, 2.0)
    assert s["p50_ms"] == 50.0 and s["p99_ms"] == 99.0 and s["max_ms"] == 100.0
    assert s["images_per_s"] == 50.0
    e = summarize([], 0, 0.0)
    assert math.isnan(e["p50_ms"])


def test_poisson_rate():
    arr = poisson_arrivals(1000.0, 20000, 3)
    assert abs(arr[-1] - 20.0) < 0.6  # mean gap 1 ms
    assert poisson_arrivals(float("inf"), 5, 3) == [0.0] * 5


def test_failed_launch_gives_back_memory_and_stream_and_requeues():
    """A backend launch that raises leaves the server as it was before admission."""

    class Flaky(SimBackend):
        def __init__(self, *a, fail=1, **kw):
            super().__init__(*a, **kw)
            self.fail = fail

        def launch(self, reqs, offset, nbytes, stream):
            if self.fail > 0:
                self.fail -= 1
                raise RuntimeError("launch refused")
            return super().launch(reqs, offset, nbytes, stream)

    clock = Clock()
    be = Flaky(clock, capacity=1 << 20)
    srv = Server(be, streams=2, max_batch=4, clock=clock)
    reqs = [_req(i, 1000) for i in range(6)]
    for r in reqs:
        srv.submit(r)
    with pytest.raises(RuntimeError, match="launch refused"):
        srv.poll()
    assert srv.arena.used == 0 and srv.arena.free_blocks() == [(0, srv.arena.capacity)]
    assert sorted(srv._free_streams) == [0, 1]
    assert [r.rid for r in srv.waiting] == list(range(6))  # back at the head, in order
    assert all(math.isnan(r.admitted) for r in reqs)
    done = []
    while not srv.idle():
        done += srv.poll()
        clock.t += 1e-4
    assert sorted(r.rid for r in done) == list(range(6))
    assert [rid for g in be.launches for rid in g] == list(range(6))
    assert srv.arena.used == 0

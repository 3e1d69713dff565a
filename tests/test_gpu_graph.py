"""A detection captured in a HIP graph gives the eager result on every replay.

Each replay is separated by eager work of its own (another detection on a
different image and a host synchronisation), and every replay's outputs are
compared with the eager call's.
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", ["64x64", "1024x1024", "4096x4096"])
def test_graph_replays_match_eager(cfg):
    from paper_1912_01884_amd import fhtp
    dev = require_gpu()
    s = synth.make_config(cfg)
    other = synth.make_config(cfg, image=1)
    img = to_device(s.image, dev)
    img2 = to_device(other.image, dev)
    dt = fhtp.FHTP_U8 if s.image.dtype == np.uint8 else fhtp.FHTP_U16
    b = fhtp.make_bend(s.bend)
    ws = torch.empty(fhtp.detect_workspace_bytes(dt, s.h, s.w, s.k, b), dtype=torch.uint8,
                     device=dev)
    score = torch.empty(1, dtype=torch.int32, device=dev)
    xs = torch.empty(s.k + 1, dtype=torch.int32, device=dev)
    announce(f"graph eager {cfg}")
    e_s, e_x = fhtp.detect_polyline(img, s.k, bend=s.bend)
    e_s, e_x = host(e_s), host(e_x)
    o_s, o_x = [host(t) for t in fhtp.detect_polyline(img2, s.k, bend=s.bend)]

    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(dev)
    cap.wait_stream(torch.cuda.current_stream(dev))
    announce(f"graph capture {cfg}")
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            fhtp.detect_polyline(img, s.k, bend=s.bend, ws=ws, score=score, xs=xs, stream=cap)
    torch.cuda.current_stream(dev).wait_stream(cap)
    torch.cuda.synchronize()
    for rep in range(4):
        score.fill_(-7)
        xs.fill_(-7)
        announce(f"graph replay {cfg} #{rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(score), e_s), rep
        assert np.array_equal(host(xs), e_x), rep
        # eager work between replays, sharing nothing with the graph's buffers
        g_s, g_x = fhtp.detect_polyline(img2, s.k, bend=s.bend)
        torch.cuda.synchronize()
        assert np.array_equal(host(g_s), o_s) and np.array_equal(host(g_x), o_x)


def test_graph_replays_batch_and_options():
    """A batched call and a smoothed, pinned, horizontal call captured together."""
    from paper_1912_01884_amd import fhtp
    dev = require_gpu()
    batch = synth.make_mixed_batch(24)
    imgs = [to_device(s.image, dev) for s in batch]
    ks = [s.k for s in batch]
    bends = [s.bend for s in batch]
    ex_img = to_device(synth.make_config("1024x1024").image, dev)
    announce("graph eager batch + ex")
    eager = [(host(a), host(b)) for a, b in fhtp.detect_batch(imgs, ks, bends=bends)]
    e_s, e_x = [host(t) for t in fhtp.detect_polyline_ex(ex_img, 16, bend=4, smooth_radius=2,
                                                          horizontal=True, pin=(8, 300))]
    jobs, keep = fhtp.make_jobs(imgs, ks, bends=bends)
    nb = fhtp.batch_workspace_bytes(jobs)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    b = fhtp.make_bend(4)
    opt = fhtp.make_options(2, True, (8, 300))
    ws2 = torch.empty(fhtp.detect_ex_workspace_bytes(fhtp.FHTP_U8, 1024, 1024, 16, b, opt),
                      dtype=torch.uint8, device=dev)
    sc2 = torch.empty(1, dtype=torch.int32, device=dev)
    xs2 = torch.empty(17, dtype=torch.int32, device=dev)
    import ctypes as C
    arr = (fhtp.Job * len(jobs))(*jobs)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream(dev)
    cap.wait_stream(torch.cuda.current_stream(dev))
    announce("graph capture batch + ex")
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            rc = fhtp.lib().fhtp_detect_batch(arr, len(jobs), C.c_void_p(ws.data_ptr()), nb,
                                             C.c_void_p(cap.cuda_stream))
            assert rc == 0
            fhtp.detect_polyline_ex(ex_img, 16, bend=4, smooth_radius=2, horizontal=True,
                                    pin=(8, 300), ws=ws2, score=sc2, xs=xs2, stream=cap)
    torch.cuda.current_stream(dev).wait_stream(cap)
    torch.cuda.synchronize()
    for rep in range(3):
        for sc, x in keep:
            sc.fill_(-7)
            x.fill_(-7)
        sc2.fill_(-7)
        announce(f"graph replay batch + ex #{rep}")
        graph.replay()
        torch.cuda.synchronize()
        for (sc, x), (w_s, w_x) in zip(keep, eager):
            assert np.array_equal(host(sc), w_s) and np.array_equal(host(x), w_x), rep
        assert np.array_equal(host(sc2), e_s) and np.array_equal(host(xs2), e_x), rep
        # eager work between replays
        fhtp.detect_polyline(imgs[0], ks[0], bend=bends[0])
        torch.cuda.synchronize()


def test_plan_replays_match_direct_calls(orc):
    """fhtp_plan_*: one 4096x4096 job and a mixed batch, each recorded once and
    replayed; images refilled in place between replays; eager work between."""
    from paper_1912_01884_amd import fhtp
    dev = require_gpu()
    big = synth.make_config("4096x4096")
    img = to_device(big.image, dev)
    announce("plan 4096x4096: eager")
    e_s, e_x = [host(t) for t in fhtp.detect_polyline(img, big.k, bend=big.bend)]
    plan = fhtp.Plan([img], [big.k], bends=[big.bend])
    (sc, xs), = plan.results
    for rep in range(3):
        sc.fill_(-7)
        xs.fill_(-7)
        announce(f"plan 4096x4096: replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(sc), e_s) and np.array_equal(host(xs), e_x), rep
        fhtp.detect_polyline(img, big.k, bend=big.bend + 1)  # eager work between replays
        torch.cuda.synchronize()
    # new contents in the same buffer: the next replay reads them
    flipped = np.ascontiguousarray(big.image[::-1])
    img.copy_(torch.from_numpy(flipped).to(dev))
    f_s, f_x = [host(t) for t in fhtp.detect_polyline(img, big.k, bend=big.bend)]
    announce("plan 4096x4096: replay on refilled image")
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(host(sc), f_s) and np.array_equal(host(xs), f_x)
    plan.destroy()

    batch = synth.make_mixed_batch(32)
    imgs = [to_device(s.image, dev) for s in batch]
    ks = [s.k for s in batch]
    bends = [s.bend for s in batch]
    announce("plan mixed batch: eager")
    eager = [(host(a), host(b)) for a, b in fhtp.detect_batch(imgs, ks, bends=bends)]
    bplan = fhtp.Plan(imgs, ks, bends=bends)
    for rep in range(3):
        for a, b in bplan.results:
            a.fill_(-7)
            b.fill_(-7)
        announce(f"plan mixed batch: replay {rep}")
        bplan.launch()
        torch.cuda.synchronize()
        for (a, b), (w_s, w_x) in zip(bplan.results, eager):
            assert np.array_equal(host(a), w_s) and np.array_equal(host(b), w_x), rep
        fhtp.detect_polyline(imgs[0], ks[0], bend=bends[0])
        torch.cuda.synchronize()
    bplan.destroy()

    # a small plan against the oracle itself
    small = synth.make_config("64x64")
    want_s, want_x = orc.detect_polyline(small.image, small.k, bend=small.bend)
    splan = fhtp.Plan([to_device(small.image, dev)], [small.k], bends=[small.bend])
    announce("plan 64x64 vs oracle")
    splan.launch()
    torch.cuda.synchronize()
    (a, b), = splan.results
    assert int(host(a)[0]) == want_s and host(b).tolist() == want_x.tolist()
    splan.destroy()


def test_plan_with_scanned_windows(orc):
    """A plan whose jobs take the scanned windows (angle form, a large bound,
    no bound) and a tall two-pass band, replayed twice, against the oracle."""
    import math
    from paper_1912_01884_amd import fhtp
    dev = require_gpu()
    rng = np.random.default_rng([191201884, 77, 1])
    shapes = [(256, 300, 8), (1024, 200, 4), (512, 130, 2)]
    imgs = [rng.integers(0, 256, size=(h, w)).astype(np.uint8) for h, w, _ in shapes]
    ks = [k for _, _, k in shapes]
    gammas = [math.radians(10), None, None]
    bends = [None, 40, 1000]
    plan = fhtp.Plan([to_device(im, dev) for im in imgs], ks, bends=bends, gammas=gammas)
    want = []
    for im, k, b, g in zip(imgs, ks, bends, gammas):
        want.append(orc.detect_polyline(im, k, gamma=g) if g is not None
                    else orc.detect_polyline(im, k, bend=b))
    for rep in range(2):
        for a, b in plan.results:
            a.fill_(-7)
            b.fill_(-7)
        announce(f"plan with scanned windows: replay {rep}")
        plan.launch()
        torch.cuda.synchronize()
        for (a, b), (w_s, w_x) in zip(plan.results, want):
            assert int(host(a)[0]) == w_s, rep
            assert host(b).tolist() == w_x.tolist(), rep
    plan.destroy()


_FIRST_CALL = """
import json, sys
import torch
import synth
from paper_1912_01884_amd import fhtp
s = synth.make_config(sys.argv[1])
img = torch.from_numpy(s.image).to("cuda:0")
plan = fhtp.Plan([img], [s.k], bends=[s.bend])
plan.launch()
torch.cuda.synchronize()
(sc, xs), = plan.results
print(json.dumps([int(sc.cpu()[0]), xs.cpu().tolist()]))
"""


@pytest.mark.parametrize("cfg", ["64x64", "1024x1024"])
def test_plan_as_first_call_in_a_fresh_process(orc, cfg):
    """A plan recorded by a process that has made no other library call.  Its
    first-use set-up then runs while the capture is open: raising the
    one-workgroup kernel's LDS limit and the FHT's occupancy query, neither of
    them stream work (the plan's second stream is made before the capture)."""
    require_gpu()
    s = synth.make_config(cfg)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    announce(f"plan as a fresh process's first call: {cfg}")
    r = subprocess.run([sys.executable, "-c", _FIRST_CALL, cfg], cwd=root, capture_output=True,
                       text=True, timeout=180, env=dict(os.environ, PYTHONPATH=root))
    assert r.returncode == 0, r.stdout + r.stderr
    got_s, got_x = json.loads(r.stdout.strip().splitlines()[-1])
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=s.bend)
    assert got_s == want_s and got_x == want_x.tolist()

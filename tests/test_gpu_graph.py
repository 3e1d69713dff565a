"""A detection captured in a HIP graph gives the eager result on every replay.

Each replay is separated by eager work of its own (another detection on a
different image and a host synchronisation), and every replay's outputs are
compared with the eager call's.
"""

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3"])
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

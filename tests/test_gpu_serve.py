"""GPU tests of the serving loop: each result is the same alone and in the mix.

Requests from the mixed-size workload (heights 128..2048, widths 256..2048,
k in {4, 8, 16}) go through the continuous-batching server while earlier
groups still run; every score and vertex list must equal the plain
one-image call on the same input, and a sample is checked against the oracle.
"""

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def mix(dev):
    batch = synth.make_mixed_batch(48)
    return batch, [to_device(s.image, dev) for s in batch]


def _requests(batch, imgs, dev, order):
    from paper_1912_01884_amd.serve import Request
    out = []
    for rid, q in enumerate(order):
        s = batch[q]
        out.append(Request(img=imgs[q], k=s.k, bend=s.bend,
                           score=torch.full((1,), -7, dtype=torch.int32, device=dev),
                           xs=torch.full((s.k + 1,), -7, dtype=torch.int32, device=dev), rid=rid))
    return out


def _alone(batch, imgs):
    from paper_1912_01884_amd import fhtp
    res = []
    for s, im in zip(batch, imgs):
        sc, xs = fhtp.detect_polyline(im, s.k, bend=s.bend)
        res.append((sc, xs))
    torch.cuda.synchronize()
    return [(int(host(a)[0]), host(b).tolist()) for a, b in res]


def _drive_in_waves(srv, reqs, wave):
    """Submit `wave` requests, poll once (groups start), repeat, then drain."""
    for i in range(0, len(reqs), wave):
        for r in reqs[i:i + wave]:
            assert srv.submit(r), r.error
        srv.poll()
    srv.drain(timeout=60)


def test_served_results_equal_alone(dev, mix, orc):
    from paper_1912_01884_amd.serve import FhtpBackend, Server
    batch, imgs = mix
    alone = _alone(batch, imgs)
    order = list(np.random.default_rng([191201884, 5, 7]).permutation(len(batch)))
    reqs = _requests(batch, imgs, dev, order)
    announce("serve 48 mixed requests, 3 streams, waves of 5")
    srv = Server(FhtpBackend(dev, arena_bytes=2 << 30, streams=3), streams=3, max_batch=16)
    _drive_in_waves(srv, reqs, 5)
    assert srv.groups_launched < len(reqs)  # requests really were grouped
    for r, q in zip(reqs, order):
        assert (int(host(r.score)[0]), host(r.xs).tolist()) == alone[q], (r.rid, q)
    # and the plain path itself against the oracle on the smaller images
    small = sorted(range(len(batch)), key=lambda q: batch[q].h * batch[q].w)[:6]
    for q in small:
        s = batch[q]
        assert orc.detect_polyline(s.image, s.k, bend=s.bend)[0] == alone[q][0]
        assert orc.detect_polyline(s.image, s.k, bend=s.bend)[1].tolist() == alone[q][1]


def test_tight_arena_backpressure_keeps_results(dev, mix):
    from paper_1912_01884_amd import fhtp
    from paper_1912_01884_amd.serve import FhtpBackend, Server, align_up
    batch, imgs = mix
    alone = _alone(batch, imgs)
    need = [align_up(fhtp.detect_workspace_bytes(s.dtype_code, s.h, s.w, s.k,
                                                 fhtp.make_bend(s.bend))) for s in batch]
    cap = max(need) + max(need) // 2  # the largest request plus a little: groups stay small
    reqs = _requests(batch, imgs, dev, range(len(batch)))
    announce(f"serve 48 mixed requests in a {cap} byte arena")
    srv = Server(FhtpBackend(dev, arena_bytes=cap, streams=4), streams=4, max_batch=64)
    _drive_in_waves(srv, reqs, 48)
    for r in reqs:
        assert (int(host(r.score)[0]), host(r.xs).tolist()) == alone[r.rid]
    assert srv.arena.used == 0


def test_open_loop_server_and_plain_agree(dev, mix):
    from paper_1912_01884_amd.serve import (FhtpBackend, PlainServer, Server, poisson_arrivals,
                                            run_open_loop)
    batch, imgs = mix
    alone = _alone(batch, imgs)
    arr = poisson_arrivals(5000.0, len(batch), [191201884, 5, 999])
    announce("open loop 48 requests at 5000/s: server")
    reqs = _requests(batch, imgs, dev, range(len(batch)))
    srv = Server(FhtpBackend(dev, arena_bytes=2 << 30, streams=4), streams=4)
    res = run_open_loop(srv, reqs, arr, timeout=60)
    assert res["requests"] == len(batch)
    srv_reqs = reqs
    for r in reqs:
        assert (int(host(r.score)[0]), host(r.xs).tolist()) == alone[r.rid]
    announce("open loop 48 requests at 5000/s: plain")
    reqs = _requests(batch, imgs, dev, range(len(batch)))
    plain = PlainServer(dev, max_request_bytes=max(r.nbytes for r in srv_reqs))
    res_p = run_open_loop(plain, reqs, arr, timeout=60)
    assert res_p["requests"] == len(batch)
    for r in reqs:
        assert (int(host(r.score)[0]), host(r.xs).tolist()) == alone[r.rid]



def test_requests_made_on_a_side_stream_after_the_server_starts(dev, mix):
    """Inputs and outputs produced asynchronously on the submitting stream are waited for."""
    from paper_1912_01884_amd.serve import FhtpBackend, PlainServer, Request, Server
    batch, imgs = mix
    alone = _alone(batch, imgs)
    srv = Server(FhtpBackend(dev, arena_bytes=2 << 30, streams=3), streams=3, max_batch=8)
    plain = PlainServer(dev, max_request_bytes=1 << 28)
    side = torch.cuda.Stream(dev)
    announce("serve 12 requests whose tensors are filled on a side stream")
    for server in (srv, plain):
        reqs = []
        with torch.cuda.stream(side):
            # a long kernel first, so that the copies really are still pending at submit
            junk = torch.empty(1 << 28, dtype=torch.uint8, device=dev)
            junk.fill_(3)
            for rid, q in enumerate(range(12)):
                s = batch[q]
                img = torch.empty_like(imgs[q])
                img.copy_(imgs[q])
                reqs.append(Request(img=img, k=s.k, bend=s.bend,
                                    score=torch.full((1,), -7, dtype=torch.int32, device=dev),
                                    xs=torch.full((s.k + 1,), -7, dtype=torch.int32, device=dev),
                                    rid=rid))
            for r in reqs:
                assert server.submit(r), r.error
            server.poll()
        server.drain(timeout=60)
        torch.cuda.synchronize()
        del junk
        for r in reqs:
            assert (int(host(r.score)[0]), host(r.xs).tolist()) == alone[r.rid], r.rid

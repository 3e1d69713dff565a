"""The allocation-free entry point against fhtp_detect_polyline (GPU).

fhtp_detect_polyline_noalloc keeps its scratch in a device array built into
the library instead of a caller workspace.  Two calls in a row (the second on
a smaller image, so that it runs over what the first left in the array) must
each equal the workspace entry point and the oracle, and a request larger
than the array is refused before anything is enqueued.
"""

import ctypes as C

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _call_noalloc(L, fhtp, img, k, bend, score, xs, stream):
    h, w = img.shape
    return L.fhtp_detect_polyline_noalloc(C.c_void_p(img.data_ptr()), fhtp._dtype_code(img), h, w,
                                          k, fhtp.make_bend(bend), C.c_void_p(score.data_ptr()),
                                          C.c_void_p(xs.data_ptr()), C.c_void_p(stream.cuda_stream))


def test_noalloc_matches_workspace_entry_point_twice(dev, orc):
    from paper_1912_01884_amd import fhtp
    L = fhtp.lib()
    stream = torch.cuda.current_stream(dev)
    cases = [synth.make_medium(), synth.make_small()]  # 1024x1024 k=16, then 64x64 k=4
    for s in cases:
        need = fhtp.detect_workspace_bytes(s.dtype_code, s.h, s.w, s.k, fhtp.make_bend(s.bend))
        assert need <= fhtp.noalloc_scratch_bytes()
    outs = []
    for s in cases:
        img = to_device(s.image, dev)
        announce(f"detect_polyline_noalloc {s.h}x{s.w} k={s.k} bend={s.bend}")
        score = torch.full((1,), -7, dtype=torch.int32, device=dev)
        xs = torch.full((s.k + 1,), -7, dtype=torch.int32, device=dev)
        assert _call_noalloc(L, fhtp, img, s.k, s.bend, score, xs, stream) == fhtp.OK
        torch.cuda.synchronize()
        outs.append((s, img, int(host(score)[0]), host(xs).copy()))
    for s, img, got_s, got_x in outs:
        ref_s, ref_x = fhtp.detect_polyline(img, s.k, bend=s.bend)
        torch.cuda.synchronize()
        assert got_s == int(host(ref_s)[0]) and np.array_equal(got_x, host(ref_x)), (s.h, s.w)
        want = orc.detect_polyline(s.image, s.k, bend=s.bend)
        assert got_s == want[0] and np.array_equal(got_x, want[1]), (s.h, s.w)


def test_noalloc_refuses_requests_beyond_its_array(dev):
    from paper_1912_01884_amd import fhtp
    L = fhtp.lib()
    stream = torch.cuda.current_stream(dev)
    img = torch.zeros((4096, 4096), dtype=torch.uint16, device=dev)
    score = torch.full((1,), -7, dtype=torch.int32, device=dev)
    xs = torch.full((33,), -7, dtype=torch.int32, device=dev)
    assert fhtp.detect_workspace_bytes(fhtp.FHTP_U16, 4096, 4096, 32, fhtp.make_bend(8)) > \
        fhtp.noalloc_scratch_bytes()
    announce("detect_polyline_noalloc 4096x4096: refused, nothing enqueued")
    assert _call_noalloc(L, fhtp, img, 32, 8, score, xs, stream) == fhtp.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int(host(score)[0]) == -7 and (host(xs) == -7).all()

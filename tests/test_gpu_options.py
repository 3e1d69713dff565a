"""GPU parity of the optional steps against the CPU oracle, bit for bit.

Through-point queries pin one vertex (every boundary j = 0..k, columns at the
edges and inside, every kind of bend window, one- and two-band images where
the pin falls on the table read directly); row smoothing and the transpose of
mostly horizontal curves are checked as images (fhtp_prepare_image against
the oracle's smoothing and numpy's transpose) and through the whole detector.
"""

import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside per-test time limits)

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def F():
    from paper_1912_01884_amd import fhtp
    return fhtp


def _rng(seed):
    return np.random.default_rng([191201884, 98, seed])


def _run(F, orc, dev, img, k, bend=None, gamma=None, smooth_radius=0, horizontal=False,
         pin=None):
    want_s, want_x = orc.detect_ex(img, k, bend=bend, gamma=gamma, smooth_radius=smooth_radius,
                                   horizontal=horizontal, pin=pin)
    s, xs = F.detect_polyline_ex(to_device(img, dev), k, bend=bend, gamma=gamma,
                                 smooth_radius=smooth_radius, horizontal=horizontal, pin=pin)
    torch.cuda.synchronize()
    assert int(host(s)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()
    return want_s, want_x


def _pins(k, w, rng):
    js = sorted({0, 1, k // 2, k - 2, k - 1, k} & set(range(k + 1)))
    out = []
    for j in js:
        for x in sorted({0, w - 1, int(rng.integers(0, w))}):
            out.append((j, x))
    return out


PIN_CASES = [
    # (h, w, k, dtype, bend kwargs)
    (64, 64, 4, np.uint8, dict(bend=1)),              # 64x64 k=4 configuration shape
    (64, 77, 1, np.uint8, dict(bend=1)),              # k = 1: argmax of one table
    (64, 90, 2, np.uint16, dict(bend=3)),             # k = 2: the walk reads the table
    (96, 130, 3, np.uint8, dict(bend=2)),             # ragged tiles
    (256, 200, 8, np.uint8, dict(bend=20)),           # scanning kernel (B > 16)
    (256, 150, 4, np.uint8, dict(bend=126)),          # unbounded: whole-column maximum
    (128, 140, 4, np.uint16, dict(gamma=0.3)),        # angle windows
    (512, 300, 2, np.uint8, dict(bend=4)),            # n = 256: 16-bit back-pointers, 2 passes
    (1024, 1024, 16, np.uint8, dict(bend=4)),         # 1024^2 k=16 configuration shape
    # two steps per launch with the pin inside a pair, on the table the first
    # pair reads, on an odd top band stepped alone, and with 16-bit pointers
    (80, 150, 5, np.uint8, dict(bend=3)),             # k = 5: top band alone, one pair
    (144, 200, 9, np.uint16, dict(bend=8)),           # k = 9: top band alone, three pairs
    (192, 110, 6, np.uint8, dict(bend=0)),            # k = 6: two pairs, straight lines
    (1024, 120, 4, np.uint8, dict(bend=5)),           # n = 256, 16-bit back-pointers, one pair
]


@pytest.mark.parametrize("h,w,k,dtype,bk", PIN_CASES,
                         ids=[f"{c[0]}x{c[1]}k{c[2]}{np.dtype(c[3]).name}-" +
                              "-".join(f"{a}{b}" for a, b in c[4].items()) for c in PIN_CASES])
def test_through_point_matches_oracle(F, orc, dev, h, w, k, dtype, bk):
    rng = _rng(h * 7 + w * 3 + k)
    top = 3 if h <= 128 else np.iinfo(dtype).max  # tie-heavy for small images
    img = rng.integers(0, top + 1, size=(h, w)).astype(dtype)
    for j, x in _pins(k, w, rng):
        announce(f"through_point {h}x{w} k={k} {bk} pin=({j},{x})")
        s, xs = _run(F, orc, dev, img, k, pin=(j, x), **bk)
        assert xs[j] == x


def test_through_point_on_the_best_polyline_is_the_free_result(F, orc, dev):
    si = synth.make_medium()
    img = si.image
    d = to_device(img, dev)
    s, xs = F.detect_polyline(d, si.k, bend=si.bend)
    torch.cuda.synchronize()
    s, xs = int(host(s)[0]), host(xs)
    for j in (0, 5, si.k):
        announce(f"through_point 1024x1024 on the free optimum j={j}")
        s2, xs2 = F.detect_polyline_ex(d, si.k, bend=si.bend, pin=(j, int(xs[j])))
        torch.cuda.synchronize()
        assert int(host(s2)[0]) == s and host(xs2).tolist() == xs.tolist()


@pytest.mark.parametrize("r", range(0, 8))
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("horizontal", [False, True])
def test_prepared_image_matches_oracle(F, orc, dev, r, dtype, horizontal):
    rng = _rng(1000 + r)
    h, w = 130, 201  # ragged in both tile directions
    img = rng.integers(0, np.iinfo(dtype).max + 1, size=(h, w)).astype(dtype)
    img[:, :3] = np.iinfo(dtype).max
    img[:2, :] = 0
    announce(f"prepare_image r={r} {np.dtype(dtype).name} horizontal={horizontal}")
    out = F.prepare_image(to_device(img, dev), smooth_radius=r, horizontal=horizontal)
    torch.cuda.synchronize()
    src = np.ascontiguousarray(img.T) if horizontal else img
    want = orc.smooth_rows(src, r)
    got = host(out)
    assert got.dtype == want.dtype and got.shape == want.shape
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (7, 64), (64, 65), (4500, 70)])
def test_prepared_image_edge_shapes(F, orc, dev, shape):
    img = _rng(sum(shape)).integers(0, 256, size=shape).astype(np.uint8)
    for horizontal in (False, True):
        for r in (0, 3, 7):
            announce(f"prepare_image shape={shape} r={r} horizontal={horizontal}")
            out = F.prepare_image(to_device(img, dev), smooth_radius=r, horizontal=horizontal)
            torch.cuda.synchronize()
            src = np.ascontiguousarray(img.T) if horizontal else img
            assert np.array_equal(host(out), orc.smooth_rows(src, r))


@pytest.mark.parametrize("cfg,r", [("64x64", 1), ("1024x1024", 2), ("1024x1024", 7)])
def test_smoothed_detection_matches_oracle(F, orc, dev, cfg, r):
    si = synth.make_config(cfg)
    announce(f"smoothed detect {cfg} r={r}")
    _run(F, orc, dev, si.image, si.k, bend=si.bend, smooth_radius=r)


HORIZONTAL_CASES = [
    # (h, w, k, dtype, bend kwargs, r)
    (64, 64, 4, np.uint8, dict(bend=1), 0),
    (50, 128, 8, np.uint16, dict(bend=2), 0),
    (300, 256, 4, np.uint8, dict(gamma=0.4), 2),
    (1000, 1024, 16, np.uint8, dict(bend=4), 1),
]


@pytest.mark.parametrize("h,w,k,dtype,bk,r", HORIZONTAL_CASES)
def test_horizontal_matches_oracle(F, orc, dev, h, w, k, dtype, bk, r):
    rng = _rng(5000 + h + w)
    img = rng.integers(0, np.iinfo(dtype).max + 1, size=(h, w)).astype(dtype)
    announce(f"horizontal {h}x{w} k={k} {bk} r={r}")
    _run(F, orc, dev, img, k, smooth_radius=r, horizontal=True, **bk)
    for j, y in [(0, 0), (k // 2, h // 3), (k, h - 1)]:
        announce(f"horizontal {h}x{w} k={k} pin=({j},{y})")
        _run(F, orc, dev, img, k, smooth_radius=r, horizontal=True, pin=(j, y), **bk)


def test_horizontal_recovers_a_transposed_1024_curve(F, orc, dev):
    """The 1024^2 k=16 image turned on its side: the curve found is the same one."""
    si = synth.make_medium()
    img_t = np.ascontiguousarray(si.image.T)
    announce("horizontal 1024x1024 transposed")
    s, ys = _run(F, orc, dev, img_t, si.k, bend=si.bend, horizontal=True)
    s0, xs0 = orc.detect_polyline(si.image, si.k, bend=si.bend)
    assert s == s0 and ys.tolist() == xs0.tolist()


def test_full_size_options(F, orc, dev):
    """4096^2 uint16, k = 32, B = 8 with smoothing and a pin in the middle boundary."""
    si = synth.make_large()
    s0, xs0 = orc.detect_polyline(si.image, si.k, bend=si.bend)
    announce("4096x4096 pinned through the free optimum, r=0")
    _run(F, orc, dev, si.image, si.k, bend=si.bend, pin=(16, int(xs0[16])))
    announce("4096x4096 smoothed r=2, pinned at column 1000 of boundary 16")
    _run(F, orc, dev, si.image, si.k, bend=si.bend, smooth_radius=2, pin=(16, 1000))


def test_options_repeat_identically(F, dev):
    img = _rng(77).integers(0, 256, size=(512, 512)).astype(np.uint8)
    d = to_device(img, dev)
    outs = []
    for _ in range(3):
        s, xs = F.detect_polyline_ex(d, 8, bend=4, smooth_radius=3, horizontal=True, pin=(3, 100))
        torch.cuda.synchronize()
        outs.append((int(host(s)[0]), host(xs).tolist()))
    assert outs[0] == outs[1] == outs[2]

"""GPU parity of the one-workgroup path for small images.

A detection whose bands are at most 32 rows high and whose image, tables,
value planes and back-pointers fit in 64 KB runs as one workgroup doing the
whole detection in LDS (line sums summed along the dyadic lines, every DP
step, the argmax and the walk): always in a batch, and alone while its work
stays near that of the 64 x 64 image.  Each case checks that this path ran (the
`detect_small` kernel family in the library's timing records), then the
oracle's score and all k + 1 vertices exactly: band heights 1 to 32, k from
1, widths from 1, both pixel types, every window kind (fixed bounds 0 to 16,
larger bounds, no limit, the angle form), tie-heavy, all-zero and saturated
images; the smoothing and horizontal options; the allocation-free entry
point; batches of small images alone and mixed with large ones.
"""

import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside per-test time limits)

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu

SHAPES = [
    # (h, w, k, pixel type)
    (8, 1, 8, np.uint8),        # n = 1, w = 1
    (8, 5, 4, np.uint8),        # n = 2
    (16, 3, 1, np.uint8),       # k = 1, w < n
    (64, 64, 4, np.uint8),      # the 64x64 workload's shape
    (64, 64, 4, np.uint16),
    (32 * 2, 30, 2, np.uint16),  # n = 32
    (16 * 6, 40, 6, np.uint8),
    (4 * 30, 90, 30, np.uint8),  # many short bands
    (8 * 7, 120, 7, np.uint16),
]

BENDS = [dict(bend=0), dict(bend=1), dict(bend=5), dict(bend=16), dict(bend=21),
         dict(bend=1000), dict(gamma=0.2), dict(gamma=1.2), dict(gamma=math.pi / 2)]


def _img(h, w, dtype, seed, kind):
    rng = np.random.default_rng([191201884, 171, seed])
    top = 255 if dtype == np.uint8 else 65535
    img = rng.integers(0, top + 1, size=(h, w)).astype(dtype)
    if kind == "ties":
        img //= top // 2
    elif kind == "zero":
        img[:] = 0
    elif kind == "full":
        img[:] = top
    return img


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _ran_small(fn):
    from paper_1912_01884_amd import fhtp
    fhtp.timing_start()
    try:
        out = fn()
    finally:
        fams = fhtp.timing_stop()
    return out, "detect_small" in fams


@pytest.mark.parametrize("kind", ["random", "ties", "zero", "full"])
@pytest.mark.parametrize("h,w,k,dt", SHAPES, ids=[f"{c[0]}x{c[1]}k{c[2]}{np.dtype(c[3]).name}" for c in SHAPES])
def test_small_images(dev, orc, h, w, k, dt, kind):
    from paper_1912_01884_amd import fhtp
    img = _img(h, w, dt, 3 * h + w + k, kind)
    d = to_device(img, dev)
    for kw in BENDS:
        want_s, want_x = orc.detect_polyline(img, k, **kw)
        announce(f"small {h}x{w} k={k} {kind} {kw}")
        (sc, xs), ran = _ran_small(lambda: fhtp.detect_polyline(d, k, **kw))
        assert ran, kw
        assert int(host(sc)[0]) == want_s, kw
        assert host(xs).tolist() == want_x.tolist(), kw


def test_small_workload_config(dev, orc):
    from paper_1912_01884_amd import fhtp
    s = synth.make_small()
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=s.bend)
    announce("small: the 64x64 workload")
    (sc, xs), ran = _ran_small(lambda: fhtp.detect_polyline(to_device(s.image, dev), s.k, bend=s.bend))
    assert ran
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


@pytest.mark.parametrize("opts", [dict(smooth_radius=2), dict(horizontal=True),
                                  dict(smooth_radius=1, horizontal=True)],
                         ids=["smooth", "horizontal", "both"])
def test_small_with_options(dev, orc, opts):
    from paper_1912_01884_amd import fhtp
    img = _img(64, 64, np.uint8, 77, "random")
    want_s, want_x = orc.detect_ex(img, 4, bend=2, **opts)
    announce(f"small with options {opts}")
    (sc, xs), ran = _ran_small(lambda: fhtp.detect_polyline_ex(to_device(img, dev), 4, bend=2, **opts))
    assert ran
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_small_no_alloc(dev, orc):
    from paper_1912_01884_amd import fhtp
    img = _img(64, 64, np.uint16, 78, "random")
    want_s, want_x = orc.detect_polyline(img, 4, bend=1)
    announce("small through the allocation-free entry point")
    (sc, xs), ran = _ran_small(lambda: fhtp.detect_polyline_noalloc(to_device(img, dev), 4, bend=1))
    assert ran
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_small_batches(dev, orc):
    """200 small images in one call (one launch, a workgroup each), then small
    and large images mixed in one call."""
    from paper_1912_01884_amd import fhtp
    rng = np.random.default_rng([191201884, 172])
    jobs = []
    for q in range(200):
        n = int(rng.choice([1, 2, 4, 8, 16, 32]))
        k = int(rng.integers(1, 9))
        w = int(rng.integers(1, 60))
        dt = np.uint8 if q % 3 else np.uint16
        kind = ("random", "ties", "zero")[q % 3]
        kw = dict(gamma=0.4) if q % 7 == 0 else dict(bend=int(rng.integers(0, 20)))
        jobs.append((_img(n * k, w, dt, 1000 + q, kind), k, kw))
    want = [orc.detect_polyline(img, k, **kw) for img, k, kw in jobs]
    imgs = [to_device(img, dev) for img, _, _ in jobs]
    announce("batch of 200 small images")
    out, ran = _ran_small(lambda: fhtp.detect_batch(
        imgs, [j[1] for j in jobs], bends=[j[2].get("bend") for j in jobs],
        gammas=[j[2].get("gamma") for j in jobs]))
    assert ran
    for q, (s, x) in enumerate(want):
        assert int(host(out[q][0])[0]) == s, q
        assert host(out[q][1]).tolist() == x.tolist(), q
    # mixed with large images
    big = [synth.make_mixed_image(j) for j in range(6)]
    mix = [(img, k, kw) for img, k, kw in jobs[:30]] + [(s.image, s.k, dict(bend=s.bend)) for s in big]
    want = [orc.detect_polyline(img, k, **kw) for img, k, kw in mix]
    imgs = [to_device(img, dev) for img, _, _ in mix]
    announce("batch of 30 small and 6 large images")
    out = fhtp.detect_batch(imgs, [j[1] for j in mix], bends=[j[2].get("bend") for j in mix],
                            gammas=[j[2].get("gamma") for j in mix])
    for q, (s, x) in enumerate(want):
        assert int(host(out[q][0])[0]) == s, q
        assert host(out[q][1]).tolist() == x.tolist(), q


def test_general_path_rule(dev, orc):
    """A tuning rule turns the one-workgroup path off: the general kernels run
    and give the same result."""
    from paper_1912_01884_amd import autotune, fhtp
    img = _img(64, 64, np.uint8, 79, "random")
    want_s, want_x = orc.detect_polyline(img, 4, bend=1)
    d = to_device(img, dev)
    fhtp.tune_set([autotune.rule(small=1)])
    try:
        announce("small image with the one-workgroup path off")
        (sc, xs), ran = _ran_small(lambda: fhtp.detect_polyline(d, 4, bend=1))
    finally:
        fhtp.tune_set([])
    assert not ran
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_heavier_small_image_alone_takes_the_general_path(dev, orc):
    """An image that fits in LDS but has several times the 64 x 64 image's
    work runs on the general kernels when alone, on the one-workgroup path in
    a batch; both give the oracle's result."""
    from paper_1912_01884_amd import fhtp
    img = _img(32 * 3, 40, np.uint16, 80, "random")
    want_s, want_x = orc.detect_polyline(img, 3, bend=4)
    d = to_device(img, dev)
    announce("heavier small image alone")
    (sc, xs), ran = _ran_small(lambda: fhtp.detect_polyline(d, 3, bend=4))
    assert not ran
    assert int(host(sc)[0]) == want_s and host(xs).tolist() == want_x.tolist()
    announce("heavier small image in a batch")
    out, ran = _ran_small(lambda: fhtp.detect_batch([d, d], [3, 3], bends=[4, 4]))
    assert ran
    for sc, xs in out:
        assert int(host(sc)[0]) == want_s and host(xs).tolist() == want_x.tolist()

"""GPU parity of the unbounded bend (every bend admissible).

Without a bend restriction the DP runs as the column recurrence
U_i(x) = max_d H_i(x, d) + U_{i+1}(x + d) with one back-pointer per column,
and the walk follows it.  Both forms of "unbounded" take it: a mode-0 bound
of at least 2n - 2 shifts and a mode-1 angle of at least pi/2.  Every case
must give the oracle's score and all k + 1 vertices exactly (the tie rule
included), over band heights from 2 to 1024 rows (16-bit back-pointers and
the two-pass FHT), 8- and 16-bit pixels (uint16 and int32 tables), k from 2
up, widths down to one column, tie-heavy and all-zero images, batches of
mixed shapes, and through-point queries (which keep the scanning kernel).
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
    (4 * 2, 9, 4, np.uint8),           # n = 2: three displacements
    (8 * 5, 1, 5, np.uint8),           # one column
    (16 * 2, 70, 2, np.uint16),        # k = 2: band 1 read as V_1 directly
    (32 * 3, 333, 3, np.uint8),        # k = 3
    (64 * 9, 130, 9, np.uint16),       # int32 tables, w < 2n + 64
    (128 * 32, 700, 32, np.uint8),     # 255 displacements, uint16 tables, many bands
    (128 * 6, 4096, 6, np.uint16),     # 64 column tiles
    (256 * 4, 300, 4, np.uint8),       # n = 256: two-pass FHT, 16-bit back-pointers
    (512 * 3, 200, 3, np.uint16),      # n = 512
    (1024 * 2, 150, 2, np.uint8),      # n = 1024: 2047 displacements
    (8 * 40, 77, 40, np.uint8),        # many short bands
]


def _img(h, w, dtype, seed, kind):
    rng = np.random.default_rng([191201884, 151, seed])
    top = 255 if dtype == np.uint8 else 60000
    img = rng.integers(0, top + 1, size=(h, w)).astype(dtype)
    if kind == "ties":
        img //= top // 3  # values 0..3: many equal optima
    elif kind == "zero":
        img[:] = 0
    return img


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def F():
    from paper_1912_01884_amd import fhtp
    return fhtp


@pytest.mark.parametrize("kind", ["random", "ties", "zero"])
@pytest.mark.parametrize("h,w,k,dt", SHAPES, ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in SHAPES])
def test_unbounded_bend(dev, F, orc, h, w, k, dt, kind, path):
    img = _img(h, w, dt, 13 * h + w + k, kind)
    n = h // k
    want_s, want_x = orc.detect_polyline(img, k, bend=2 * n - 2)
    d = to_device(img, dev)
    for bend, gamma in ((2 * n - 2, None), (10 ** 6, None), (None, math.pi / 2)):
        announce(f"unbounded {h}x{w} k={k} {kind} bend={bend} gamma={gamma}")
        sc, xs = F.detect_polyline(d, k, bend=bend, gamma=gamma)
        assert int(host(sc)[0]) == want_s, (bend, gamma)
        assert host(xs).tolist() == want_x.tolist(), (bend, gamma)


def test_unbounded_full_size(dev, F, orc):
    s = synth.make_large(0)
    n = s.h // s.k
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=2 * n - 2)
    announce("unbounded 4096x4096 k=32")
    sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, bend=2 * n - 2)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_unbounded_batch(dev, F, orc, path):
    """One batch mixing unbounded images of several shapes with fixed and
    scanned windows: every result equals the oracle's."""
    jobs = []
    for q, (h, w, k, dt) in enumerate(SHAPES):
        n = h // k
        img = _img(h, w, dt, 900 + q, "random" if q % 2 else "ties")
        jobs.append((img, k, 2 * n - 2 if q % 3 else None, math.pi / 2 if q % 3 == 0 else None))
        jobs.append((img, k, min(3, 2 * n - 2), None))  # fixed window beside it
    want = [orc.detect_polyline(img, k, bend=b, gamma=g) for img, k, b, g in jobs]
    imgs = [to_device(img, dev) for img, _, _, _ in jobs]
    announce(f"batch of {len(jobs)} with unbounded bends")
    out = F.detect_batch(imgs, [j[1] for j in jobs], bends=[j[2] for j in jobs],
                         gammas=[j[3] for j in jobs])
    for q, (s, x) in enumerate(want):
        assert int(host(out[q][0])[0]) == s, q
        assert host(out[q][1]).tolist() == x.tolist(), q


@pytest.mark.parametrize("j", [0, 2, 5])
def test_unbounded_through_point(dev, F, orc, j):
    h, w, k = 32 * 5, 200, 5
    img = _img(h, w, np.uint8, 4000 + j, "random")
    x = 17 + 31 * j
    want_s, want_x = orc.detect_through_point(img, k, j, x, bend=62)
    announce(f"unbounded through point j={j} x={x}")
    sc, xs = F.detect_polyline_ex(to_device(img, dev), k, bend=62, pin=(j, x))
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()

"""GPU parity of scanned windows: the angle form and mode-0 bounds above 16.

Steps with per-displacement windows run on the block kernel (V staged in
LDS, prefix and suffix maxima per block of rows, a table of block runs) for
bands of at most 255 displacements without a pin, and on the scanning kernel
otherwise (taller bands, through-point queries, the last step).  Every case
must give the oracle's score and all k + 1 vertices exactly: angles from
nearly 0 to nearly pi/2 (windows of one row up to nearly the whole column),
bounds from 17 up to 2n - 3, band heights 2 to 256, widths around the
16-column tile (1, 15, 16, 17, ragged), tie-heavy images, and batches.
"""

import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside per-test time limits)

from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu

SHAPES = [
    # (h, w, k, pixel type)
    (2 * 6, 15, 6, np.uint8),        # n = 2
    (8 * 5, 16, 5, np.uint8),        # n = 8, one column tile exactly
    (16 * 4, 17, 4, np.uint16),      # a tile and one column
    (32 * 6, 1, 6, np.uint8),        # one column
    (64 * 7, 333, 7, np.uint8),      # narrow tables, ragged width
    (128 * 5, 500, 5, np.uint16),    # 255 displacements, int32 tables
    (128 * 3, 90, 3, np.uint8),      # w < n
    (256 * 3, 120, 3, np.uint8),     # 511 displacements: the scanning kernel
]

GAMMAS = [1e-3, 0.05, 0.2, 0.5, 1.0, 1.4, 1.57]


def _img(h, w, dtype, seed, ties):
    rng = np.random.default_rng([191201884, 161, seed])
    top = 255 if dtype == np.uint8 else 30000
    img = rng.integers(0, top + 1, size=(h, w)).astype(dtype)
    if ties:
        img //= top // 2
    return img


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def F():
    from paper_1912_01884_amd import fhtp
    return fhtp


@pytest.mark.parametrize("ties", [False, True])
@pytest.mark.parametrize("h,w,k,dt", SHAPES, ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in SHAPES])
def test_angle_windows(dev, F, orc, h, w, k, dt, ties, path):
    img = _img(h, w, dt, 7 * h + w + k + ties, ties)
    d = to_device(img, dev)
    for g in GAMMAS:
        want_s, want_x = orc.detect_polyline(img, k, gamma=g)
        announce(f"angle {g} on {h}x{w} k={k} ties={ties}")
        sc, xs = F.detect_polyline(d, k, gamma=g)
        assert int(host(sc)[0]) == want_s, g
        assert host(xs).tolist() == want_x.tolist(), g


@pytest.mark.parametrize("h,w,k,dt", SHAPES, ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in SHAPES])
def test_large_bounds(dev, F, orc, h, w, k, dt, path):
    n = h // k
    img = _img(h, w, dt, 11 * h + w, False)
    d = to_device(img, dev)
    for B in sorted({17, 20, 33, max(17, n - 1), max(17, 2 * n - 3)}):
        want_s, want_x = orc.detect_polyline(img, k, bend=B)
        announce(f"bound {B} on {h}x{w} k={k}")
        sc, xs = F.detect_polyline(d, k, bend=B)
        assert int(host(sc)[0]) == want_s, B
        assert host(xs).tolist() == want_x.tolist(), B


def test_windows_in_batches(dev, F, orc, path):
    """Images of different band counts and heights in one pack: images at
    their last step take the scanning kernel in the same step as others on
    the block kernel."""
    jobs = []
    rng = np.random.default_rng([191201884, 162])
    for q in range(14):
        n = int(rng.choice([4, 16, 64, 128]))
        k = int(rng.integers(2, 9))
        w = int(rng.integers(10, 300))
        dt = np.uint8 if q % 2 else np.uint16
        img = _img(n * k, w, dt, 500 + q, q % 3 == 0)
        jobs.append((img, k, None, 0.3))
    for q in range(6):
        n = int(rng.choice([16, 32, 64]))
        k = int(rng.integers(2, 7))
        img = _img(n * k, int(rng.integers(10, 200)), np.uint8, 600 + q, False)
        jobs.append((img, k, 19, None))
    want = [orc.detect_polyline(img, k, bend=b, gamma=g) for img, k, b, g in jobs]
    imgs = [to_device(img, dev) for img, _, _, _ in jobs]
    announce(f"batch of {len(jobs)} with scanned windows")
    out = F.detect_batch(imgs, [j[1] for j in jobs], bends=[j[2] for j in jobs],
                         gammas=[j[3] for j in jobs])
    for q, (s, x) in enumerate(want):
        assert int(host(out[q][0])[0]) == s, q
        assert host(out[q][1]).tolist() == x.tolist(), q

"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for bit.

Everything is integer, so the bar is exact equality: band tables element by
element, and the best score with its vertices x_0..x_k.  Inputs are the seeded
synthetic configurations plus edge cases (one-row bands, images narrower than
a band, single bands, tall two-pass bands, tie-heavy and saturated images,
every kind of bend window).
"""

import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside per-test time limits)

import synth
from tests.gpu_util import announce, general_path, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def F():
    from paper_1912_01884_amd import fhtp
    return fhtp


def _rng(seed):
    return np.random.default_rng([191201884, 99, seed])


def _img(h, w, dtype, seed, maxval=None):
    top = np.iinfo(dtype).max if maxval is None else maxval
    return _rng(seed).integers(0, top + 1, size=(h, w)).astype(dtype)


TABLE_CASES = [
    # (h, w, k, dtype, values)
    (8, 1, 8, np.uint8, None),        # n = 1
    (8, 5, 4, np.uint8, None),        # n = 2
    (16, 3, 1, np.uint8, None),       # w < n
    (64, 64, 1, np.uint16, None),
    (96, 40, 3, np.uint8, None),      # n = 32
    (128, 100, 1, np.uint16, None),   # n = 128, one band
    (256, 50, 1, np.uint8, None),     # n = 256: two-pass
    (512, 33, 1, np.uint16, None),    # n = 512
    (2048, 70, 2, np.uint8, None),    # n = 1024
    (256, 700, 2, np.uint8, None),    # several tiles per band
    (512, 900, 4, np.uint16, "sat"),  # saturated
    (64, 2000, 2, np.uint8, "sat"),
    (128, 300, 1, np.uint8, "sat"),   # 8-bit, n = 128: the largest packed half-band sums
    (256, 100, 1, np.uint8, "sat"),   # 8-bit two-pass sub-blocks, saturated
    (128 * 3, 517, 3, np.uint8, None),
    # short bands over several waves and tiles (the waves of a tile overlap by
    # a few columns, the first stages move operands between lanes)
    (8, 700, 4, np.uint16, None),     # n = 2
    (16, 600, 4, np.uint8, "sat"),    # n = 4
    (64, 900, 8, np.uint16, None),    # n = 8
    (64, 530, 4, np.uint8, None),     # n = 16
]


@pytest.mark.parametrize("h,w,k,dtype,vals", TABLE_CASES,
                         ids=[f"{c[0]}x{c[1]}k{c[2]}{np.dtype(c[3]).name}{c[4] or ''}"
                              for c in TABLE_CASES])
def test_tables_small(dev, F, orc, h, w, k, dtype, vals):
    img = np.full((h, w), np.iinfo(dtype).max, dtype) if vals == "sat" else _img(h, w, dtype, h + w)
    want = orc.fht_bands(img, k)
    announce(f"fht_bands {h}x{w} k={k} {np.dtype(dtype).name}")
    got = host(F.fht_bands(to_device(img, dev), k))
    assert got.shape == want.shape
    assert np.array_equal(got, want)


@pytest.mark.parametrize("cfg", ["64x64", "1024x1024", "4096x4096"])
def test_tables_configs(dev, F, orc, cfg):
    s = synth.make_config(cfg)
    want = orc.fht_bands(s.image, s.k)
    announce(f"fht_bands {cfg}")
    got = host(F.fht_bands(to_device(s.image, dev), s.k))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("cfg", ["64x64", "1024x1024", "4096x4096"])
def test_detect_configs(dev, F, orc, cfg):
    s = synth.make_config(cfg)
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=s.bend)
    announce(f"detect {cfg} B={s.bend}")
    sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, bend=s.bend)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


@pytest.mark.parametrize("B", [0, 1, 2, 5, 8, 16, 17, 29, 30, 100])
def test_detect_c1_every_window_kind(dev, F, orc, B, path):
    s = synth.make_small()
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=B)
    announce(f"detect 64x64 B={B}")
    sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, bend=B)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


@pytest.mark.parametrize("gamma", [0.0, 0.05, 0.2, math.radians(10), 1.0, math.pi / 2, 2.0])
def test_detect_angle_bound(dev, F, orc, gamma, path):
    for cfg in ("64x64", "1024x1024"):
        s = synth.make_config(cfg)
        want_s, want_x = orc.detect_polyline(s.image, s.k, gamma=gamma)
        announce(f"detect {cfg} gamma={gamma}")
        sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, gamma=gamma)
        assert int(host(sc)[0]) == want_s
        assert host(xs).tolist() == want_x.tolist()


@pytest.mark.parametrize("bend_kw", [dict(gamma=math.radians(10)), dict(gamma=math.radians(45)),
                                     dict(bend=24), dict(bend=254)],
                         ids=["angle10", "angle45", "bound24", "unbounded"])
def test_full_size_generic_windows(dev, F, orc, bend_kw):
    """The 4096x4096 k=32 image with the scanned windows: angle form, a large bound, none."""
    s = synth.make_large()
    want_s, want_x = orc.detect_polyline(s.image, s.k, **bend_kw)
    announce(f"detect 4096x4096 {bend_kw}")
    sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, **bend_kw)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


EDGE = [
    # (h, w, k, dtype, maxval, B)
    (8, 1, 8, np.uint8, 3, 0),        # n = 1, w = 1
    (8, 5, 4, np.uint8, 3, 1),        # n = 2
    (16, 3, 1, np.uint8, 3, 0),       # k = 1, w < n
    (16, 40, 1, np.uint16, None, 2),  # k = 1
    (32, 7, 2, np.uint8, 3, 3),       # w < n
    (64, 64, 4, np.uint8, 0, 1),      # all zero
    (64, 64, 4, np.uint8, 1, 1),      # zeros and ones: ties everywhere
    (128, 130, 4, np.uint8, 3, 2),
    (256, 300, 8, np.uint16, None, 4),
    (512, 200, 2, np.uint8, 3, 5),    # n = 256, two-pass FHT, uint16 back-pointers
    (2048, 300, 4, np.uint8, None, 4),  # n = 512
    (1024, 90, 1, np.uint8, None, 3),   # n = 1024, single band
    (200 * 4, 129, 200, np.uint8, 2, 0),  # n = 4, many bands
]


@pytest.mark.parametrize("h,w,k,dtype,maxval,B", EDGE,
                         ids=[f"{c[0]}x{c[1]}k{c[2]}B{c[5]}" for c in EDGE])
def test_detect_edges(dev, F, orc, h, w, k, dtype, maxval, B, path):
    img = _img(h, w, dtype, 7 * h + w, maxval)
    want_s, want_x = orc.detect_polyline(img, k, bend=B)
    announce(f"detect edge {h}x{w} k={k} B={B}")
    sc, xs = F.detect_polyline(to_device(img, dev), k, bend=B)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


PAIRED = [
    # (h, w, k): a single image with the fixed window takes its steps two per
    # launch; odd and even step counts, ragged widths, several row groups
    (32 * 5, 333, 5),    # n = 32: one single step, then one pair
    (64 * 8, 200, 8),    # n = 64: three pairs
    (128 * 4, 130, 4),   # n = 128: one pair, 255 displacements
    (16 * 9, 70, 9),     # n = 16: odd count
    (8 * 12, 65, 12),    # n = 8: windows wider than the displacement range
    (256 * 4, 333, 4),   # n = 256: 16-bit back-pointers, one pair
    (256 * 6, 100, 6),   # n = 256: two pairs
]


@pytest.mark.parametrize("B", [0, 1, 3, 4, 7, 8, 9, 12, 15, 16])
@pytest.mark.parametrize("h,w,k", PAIRED, ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in PAIRED])
def test_detect_paired_steps(dev, F, orc, h, w, k, B):
    img = _img(h, w, np.uint8, 31 * h + w + B, 3 if B % 2 == 0 else None)
    want_s, want_x = orc.detect_polyline(img, k, bend=B)
    announce(f"detect paired {h}x{w} k={k} B={B}")
    with general_path():  # the two-step kernel, also where the image is small
        sc, xs = F.detect_polyline(to_device(img, dev), k, bend=B)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


EXTREME = [
    # (n, k, w, bend): every link of the planted polyline at a displacement of
    # -(n-1) or n-1, the first or last row of the back-pointer planes, so the
    # walk's candidate rows run past the planes' edges
    (16, 10, 203, 3),
    (16, 10, 203, 8),
    (16, 10, 203, 15),
    (256, 6, 1600, 8),   # 16-bit back-pointers
]


@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("n,k,w,B", EXTREME, ids=[f"n{c[0]}k{c[1]}w{c[2]}b{c[3]}" for c in EXTREME])
def test_walk_along_extreme_displacements(dev, F, orc, n, k, w, B, sign):
    """A bright polyline whose links all shift by sign*(n-1) (one pixel per
    row inside a band, each band starting where the last one ended) on faint
    noise: the best polyline follows it, every link at the edge of the
    displacement range."""
    img = _img(n * k, w, np.uint8, 7 * n + k + B + (sign > 0), 20)
    x = 10 if sign > 0 else w - 11
    for i in range(k):
        for j in range(n):
            img[i * n + j, x + sign * j] = 255
        x += sign * (n - 1)
    want_s, want_x = orc.detect_polyline(img, k, bend=B)
    links = np.diff(want_x)
    assert (links == sign * (n - 1)).all(), links  # the oracle takes the planted polyline
    announce(f"extreme links n={n} k={k} w={w} B={B} sign={sign}")
    with general_path():  # pairs and the general walk, also where the image is small
        sc, xs = F.detect_polyline(to_device(img, dev), k, bend=B)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_maximum_width(dev, F, orc):
    """The widest image the library takes (2^20 columns): 16384 column tiles per
    step launch, tables and planes of several hundred MB."""
    w = 1 << 20
    img = _img(32, w, np.uint8, 4242, 7)
    want_s, want_x = orc.detect_polyline(img, 4, bend=3)
    announce(f"detect maximum width 32x{w} k=4 B=3")
    sc, xs = F.detect_polyline(to_device(img, dev), 4, bend=3)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()
    tables = host(F.fht_bands(to_device(img, dev), 4))
    want_t = orc.fht_bands(img, 4)
    assert np.array_equal(tables[:, :, :4096], want_t[:, :, :4096])
    assert np.array_equal(tables[:, :, -4096:], want_t[:, :, -4096:])


def test_saturated_image(dev, F, orc):
    img = np.full((256, 301), 255, np.uint8)
    announce("detect saturated 256x301")
    sc, xs = F.detect_polyline(to_device(img, dev), 8, bend=2)
    assert int(host(sc)[0]) == 255 * 256
    assert not host(xs).any()
    img16 = np.full((4096, 64), 65535, np.uint16)
    announce("detect saturated u16 4096x64")
    sc, xs = F.detect_polyline(to_device(img16, dev), 32, bend=8)
    assert int(host(sc)[0]) == 65535 * 4096
    assert not host(xs).any()


@pytest.mark.parametrize("seed", range(12))
def test_detect_random_tiny(dev, F, orc, seed, path):
    rng = _rng(500 + seed)
    n = int(rng.choice([1, 2, 4, 8, 16]))
    k = int(rng.integers(1, 6))
    w = int(rng.integers(1, 70))
    B = int(rng.integers(0, 2 * n + 1))
    img = rng.integers(0, 4, size=(n * k, w)).astype(np.uint8)
    want_s, want_x = orc.detect_polyline(img, k, bend=B)
    announce(f"detect tiny seed={seed} {n * k}x{w} k={k} B={B}")
    sc, xs = F.detect_polyline(to_device(img, dev), k, bend=B)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_polyline_dp_on_oracle_tables(dev, F, orc):
    s = synth.make_medium()
    tables = orc.fht_bands(s.image, s.k)
    want_s, want_x = orc.polyline_dp(tables, s.h, s.w, s.k, bend=s.bend)
    announce("polyline_dp 1024x1024 on oracle tables")
    sc, xs = F.polyline_dp(to_device(tables, dev), s.h, s.w, s.k, bend=s.bend)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


def test_repeat_runs_identical(dev, F):
    s = synth.make_medium()
    img = to_device(s.image, dev)
    announce("determinism 1024x1024")
    t1 = host(F.fht_bands(img, s.k))
    t2 = host(F.fht_bands(img, s.k))
    assert np.array_equal(t1, t2)
    r1 = [host(t) for t in F.detect_polyline(img, s.k, bend=s.bend)]
    r2 = [host(t) for t in F.detect_polyline(img, s.k, bend=s.bend)]
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


@pytest.mark.parametrize("j", range(0, 256, 16))
def test_detect_mixed_batch_images(dev, F, orc, j):
    """Images of the mixed-size batch workload (h 128..2048, w 256..2048, k 4..16)."""
    s = synth.make_mixed_image(j)
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=s.bend)
    announce(f"detect mixed image {j}: {s.h}x{s.w} k={s.k}")
    sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, bend=s.bend)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()


NARROW_CASES = [
    # (h, w, k, bend): 8-bit pixels, bands of at most 256 rows, so the
    # detection keeps bands 0..k-2 as uint16 tables (line sums up to 65,280)
    (512, 301, 2, 3),     # n = 256: one narrow band, the last one int32
    (1024, 300, 4, 3),    # n = 256: two-pass FHT into narrow tables, one pair of steps
    (2048, 260, 8, 1),    # n = 256, several pairs
    (1024, 700, 8, 20),   # n = 128, scanned windows
    (1024, 500, 16, 8),   # n = 64, single steps and pairs
]


@pytest.mark.parametrize("h,w,k,bend", NARROW_CASES,
                         ids=[f"{c[0]}x{c[1]}k{c[2]}b{c[3]}" for c in NARROW_CASES])
def test_narrow_tables_at_the_bound(dev, F, orc, h, w, k, bend):
    """Near-saturated 8-bit images: every table value of a narrow band is close
    to (or, on the all-255 columns, exactly) its uint16 ceiling of n * 255."""
    rng = np.random.default_rng([191201884, 77, h, w, k])
    img = rng.integers(200, 256, size=(h, w)).astype(np.uint8)
    img[:, ::7] = 255
    img[rng.random((h, w)) < 0.01] = 0
    announce(f"narrow tables {h}x{w} k={k} bend={bend}")
    sc, xs = F.detect_polyline(to_device(img, dev), k, bend=bend)
    want_s, want_x = orc.detect_polyline(img, k, bend=bend)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()
    full = np.full((h, w), 255, np.uint8)
    sc, xs = F.detect_polyline(to_device(full, dev), k, bend=bend)
    assert int(host(sc)[0]) == 255 * h
    assert not host(xs).any()


LONG = [
    # (h, w, k, dtype): DP chains of hundreds of dependent steps (pair launches
    # and walk trips by the hundred), bands of one to four rows
    (2 * 1024, 37, 1024, np.uint8),   # n = 2: three displacements
    (1024, 20, 1024, np.uint8),       # n = 1: one displacement, vertical links only
    (4 * 600, 61, 600, np.uint16),    # n = 4
]


@pytest.mark.parametrize("h,w,k,dtype", LONG, ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in LONG])
def test_long_chains(dev, F, orc, h, w, k, dtype, path):
    n = h // k
    img = _img(h, w, dtype, 5 * h + w, 3)
    d = to_device(img, dev)
    for kw in (dict(bend=0), dict(bend=1), dict(bend=2 * n - 2), dict(gamma=0.5)):
        want_s, want_x = orc.detect_polyline(img, k, **kw)
        announce(f"long chain {h}x{w} k={k} {kw}")
        sc, xs = F.detect_polyline(d, k, **kw)
        assert int(host(sc)[0]) == want_s, kw
        assert host(xs).tolist() == want_x.tolist(), kw


def test_long_chain_in_a_batch(dev, F, orc):
    """A 1024-band image beside short ones in one batch: the images are aligned
    at their last step, so the short ones sit out hundreds of launches."""
    jobs = [(_img(2 * 1024, 37, np.uint8, 901, 3), 1024, 1),
            (_img(64 * 3, 90, np.uint8, 902, None), 3, 1),
            (_img(8 * 5, 50, np.uint8, 903, 3), 5, 2),
            (_img(16 * 2, 200, np.uint16, 904, None), 2, 0)]
    want = [orc.detect_polyline(img, k, bend=b) for img, k, b in jobs]
    imgs = [to_device(img, dev) for img, _, _ in jobs]
    announce("batch with a 1024-band image")
    out = F.detect_batch(imgs, [j[1] for j in jobs], bends=[j[2] for j in jobs])
    for q, (s, x) in enumerate(want):
        assert int(host(out[q][0])[0]) == s, q
        assert host(out[q][1]).tolist() == x.tolist(), q


def test_largest_image(dev, F, orc):
    """16384 x 16384 uint16 with k = 128 bands of 128 rows (the largest image
    of the sizes tested: 2.2 GB of band tables, 127 DP steps, offsets and
    views at scale): the score and all 129 vertices equal the oracle's."""
    s = synth.make_large(0, h=16384, w=16384, k=128)
    want_s, want_x = orc.detect_polyline(s.image, s.k, bend=s.bend)
    announce("detect 16384x16384 k=128 B=8")
    sc, xs = F.detect_polyline(to_device(s.image, dev), s.k, bend=s.bend)
    assert int(host(sc)[0]) == want_s
    assert host(xs).tolist() == want_x.tolist()

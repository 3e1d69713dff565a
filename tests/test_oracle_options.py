"""Pins of the oracle's optional steps: through-point queries, row smoothing, horizontal curves.

Through a point (Sections 2.2-2.3): brute-force enumeration restricted to the
polylines whose vertex on the given band boundary is the given column; the
maximum over every column of a boundary equals the free optimum (main
problem, steps 2-3); with the bend unbounded, the paper's own construction
(best lower part from the point plus the best part of the upper bands flipped
about the x axis, Section 2.2) gives the same score.

Row smoothing (main problem, step 1), read as the binomial kernel C(2r, i) / 4^r
with replicated edges and rounding half up: identity at r = 0, exact impulse
responses, constant rows, and a library convolution (scipy) on random rows.

Horizontal curves (Fig. 7): the library transpose followed by the vertical
detector, and planted horizontal polylines.
"""

import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from tests.helpers import enumerate_polylines, polyline_pixel_sum, vertices_to_shifts


def _rng(seed):
    return np.random.default_rng([191201884, 89, seed])


def _vertices(x0, ds):
    xs = [x0]
    for d in ds:
        xs.append(xs[-1] + d)
    return xs


def _brute_through(img, k, j, px, bend=None, gamma=None):
    h, w = img.shape
    best, best_key = None, None
    for x0, ds in enumerate_polylines(h, w, k, bend, gamma):
        if _vertices(x0, ds)[j] != px:
            continue
        sc = polyline_pixel_sum(img, k, x0, ds)
        key = (x0,) + tuple(ds)
        if best is None or sc > best or (sc == best and key < best_key):
            best, best_key = sc, key
    return best, _vertices(best_key[0], best_key[1:])


CASES = [(2, 2, 4), (2, 3, 5), (4, 2, 6), (4, 3, 5), (1, 3, 4), (4, 1, 7)]


@pytest.mark.parametrize("n,k,w", CASES)
def test_through_point_brute_force_mode0(orc, n, k, w):
    rng = _rng(n * 100 + k * 10 + w)
    img = rng.integers(0, 4, size=(n * k, w)).astype(np.uint8)
    for B in (0, 1, 2 * n):
        for j in range(k + 1):
            for px in range(w):
                want = _brute_through(img, k, j, px, bend=B)
                got_s, got_x = orc.detect_through_point(img, k, j, px, bend=B)
                assert got_s == want[0], (B, j, px)
                assert got_x.tolist() == want[1], (B, j, px)


@pytest.mark.parametrize("n,k,w", [(4, 2, 6), (4, 3, 4), (8, 2, 7)])
def test_through_point_brute_force_mode1(orc, n, k, w):
    rng = _rng(n * 1000 + k * 10 + w)
    img = rng.integers(0, 4, size=(n * k, w)).astype(np.uint8)
    for g in (0.0, 0.3, 1.2):
        for j in range(k + 1):
            for px in range(0, w, 2):
                want = _brute_through(img, k, j, px, gamma=g)
                got_s, got_x = orc.detect_through_point(img, k, j, px, gamma=g)
                assert got_s == want[0], (g, j, px)
                assert got_x.tolist() == want[1], (g, j, px)


def test_max_over_a_boundary_is_the_free_optimum(orc):
    """Every optimal polyline crosses each boundary somewhere (main problem, steps 2-3)."""
    rng = _rng(7)
    h, w, k = 64, 48, 4
    img = np.clip(rng.normal(20, 10, size=(h, w)), 0, 255).astype(np.uint8)
    img[np.arange(h), (np.arange(h) // 3 + 5)] = 200
    for B in (1, 3):
        s, xs = orc.detect_polyline(img, k, bend=B)
        for j in range(k + 1):
            scores = [orc.detect_through_point(img, k, j, px, bend=B)[0] for px in range(w)]
            assert max(scores) == s
            s2, xs2 = orc.detect_through_point(img, k, j, int(xs[j]), bend=B)
            assert s2 == s and xs2.tolist() == xs.tolist()


def _flip_construction(orc, img, k, j, px, bend):
    """Section 2.2: lower part from the point plus the flipped upper part ending at it."""
    h, w = img.shape
    n = h // k
    total = 0
    if j < k:
        total += orc.detect_from_top(np.ascontiguousarray(img[j * n:]), k - j, px, bend=bend)[0]
    if j > 0:
        up = np.ascontiguousarray(img[:j * n][::-1])
        total += orc.detect_from_top(up, j, px, bend=bend)[0]
    return total


@pytest.mark.parametrize("seed", range(3))
def test_unbounded_bend_equals_paper_halves(orc, seed):
    rng = _rng(300 + seed)
    n, k, w = 8, 4, 40
    img = rng.integers(0, 50, size=(n * k, w)).astype(np.uint8)
    for j in range(k + 1):
        for px in (0, 7, 19, w - 1):
            s_free, xs = orc.detect_through_point(img, k, j, px, bend=2 * n - 2)
            assert s_free == _flip_construction(orc, img, k, j, px, 2 * n - 2), (j, px)
            assert xs[j] == px
            assert polyline_pixel_sum(img, k, int(xs[0]), vertices_to_shifts(xs)) == s_free
            # With a bound the bend at the point is restricted too, so the halves
            # (each optimised alone) can only do better.
            s_b, xs_b = orc.detect_through_point(img, k, j, px, bend=1)
            assert s_b <= _flip_construction(orc, img, k, j, px, 1)
            assert xs_b[j] == px
            assert all(abs(a - b) <= 1 for a, b in zip(vertices_to_shifts(xs_b)[1:],
                                                         vertices_to_shifts(xs_b)[:-1]))


def test_through_point_validation(orc):
    img = np.zeros((16, 10), np.uint8)
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_through_point(img, 4, 5, 0, bend=1)
    assert e.value.code == oracle.ERR_POINT
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_through_point(img, 4, 2, 10, bend=1)
    assert e.value.code == oracle.ERR_POINT
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_through_point(img, 4, -1, 0, bend=1)
    assert e.value.code == oracle.ERR_POINT


# ---- row smoothing -----------------------------------------------------------

def test_smoothing_radius_zero_is_identity(orc):
    img = _rng(1).integers(0, 65536, size=(7, 13)).astype(np.uint16)
    assert np.array_equal(orc.smooth_rows(img, 0), img)


@pytest.mark.parametrize("r", range(1, 8))
def test_smoothing_impulse_response_is_binomial(orc, r):
    w = 40
    img = np.zeros((3, w), np.uint16)
    c = 3
    img[1, 20] = c * 4 ** r  # <= 3 * 16384 < 65536
    out = orc.smooth_rows(img, r)
    want = np.zeros((3, w), np.int64)
    for i in range(2 * r + 1):
        want[1, 20 + i - r] = c * math.comb(2 * r, i)
    assert np.array_equal(out.astype(np.int64), want)


@pytest.mark.parametrize("dtype,maxv", [(np.uint8, 255), (np.uint16, 65535)])
def test_smoothing_keeps_constant_rows(orc, dtype, maxv):
    vals = np.array([0, 1, 7, maxv // 2, maxv], dtype=dtype)
    img = np.repeat(vals[:, None], 23, axis=1)
    for r in range(8):
        assert np.array_equal(orc.smooth_rows(img, r), img)


@pytest.mark.parametrize("r", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_smoothing_matches_library_convolution(orc, r, dtype):
    rng = _rng(50 + r)
    maxv = np.iinfo(dtype).max
    img = rng.integers(0, maxv + 1, size=(9, 31)).astype(dtype)
    img[:, :2] = maxv  # bright edge: replication at the border matters
    weights = np.array([math.comb(2 * r, i) for i in range(2 * r + 1)], np.int64)
    acc = ndimage.correlate1d(img.astype(np.int64), weights, axis=1, mode="nearest")
    want = (acc + 4 ** r // 2) // 4 ** r
    assert np.array_equal(orc.smooth_rows(img, r).astype(np.int64), want)


def test_smoothing_narrow_rows(orc):
    """Rows narrower than the kernel: every tap past an end repeats that end."""
    img = np.array([[10, 30], [255, 0]], np.uint8)
    # r = 1: taps (1, 2, 1)/4 at x = 0: 10, 10, 30 -> (10+20+30+2)//4 = 15; x = 1: 10, 30, 30 -> 25
    assert orc.smooth_rows(img, 1).tolist() == [[15, 25], [191, 64]]
    one = np.array([[77]], np.uint8)
    assert orc.smooth_rows(one, 7).tolist() == [[77]]


def test_smoothing_validation(orc):
    img = np.zeros((2, 2), np.uint8)
    for r in (-1, 8):
        with pytest.raises(oracle.OracleError) as e:
            orc.smooth_rows(img, r)
        assert e.value.code == oracle.ERR_OPTION


# ---- the composite detector: smoothing, orientation, point ---------------------

def test_detect_ex_defaults_are_the_plain_detector(orc):
    rng = _rng(11)
    img = rng.integers(0, 256, size=(64, 50)).astype(np.uint8)
    assert (orc.detect_ex(img, 4, bend=2)[0], orc.detect_ex(img, 4, bend=2)[1].tolist()) == \
        (orc.detect_polyline(img, 4, bend=2)[0], orc.detect_polyline(img, 4, bend=2)[1].tolist())


@pytest.mark.parametrize("seed", range(4))
def test_horizontal_is_the_transposed_problem(orc, seed):
    rng = _rng(400 + seed)
    h, w = int(rng.integers(20, 60)), 64
    k = 8
    img = rng.integers(0, 65536, size=(h, w)).astype(np.uint16)
    for r in (0, 2):
        a = orc.detect_ex(img, k, bend=2, smooth_radius=r, horizontal=True)
        b = orc.detect_ex(np.ascontiguousarray(img.T), k, bend=2, smooth_radius=r)
        assert a[0] == b[0] and a[1].tolist() == b[1].tolist()
        pin = (3, int(rng.integers(0, h)))
        a = orc.detect_ex(img, k, bend=2, smooth_radius=r, horizontal=True, pin=pin)
        b = orc.detect_ex(np.ascontiguousarray(img.T), k, bend=2, smooth_radius=r, pin=pin)
        assert a[0] == b[0] and a[1].tolist() == b[1].tolist()


@pytest.mark.parametrize("seed", range(4))
def test_planted_horizontal_polyline(orc, seed):
    """A model polyline drawn along x (one pixel per column) is recovered row by row."""
    from tests.helpers import pattern_rec
    rng = _rng(500 + seed)
    n, k = 16, 4
    w = n * k
    h = int(rng.integers(3 * n, 5 * n))
    B = 2
    ds = [int(rng.integers(-(n // 2), n // 2))]
    for _ in range(k - 1):
        ds.append(int(np.clip(ds[-1] + rng.integers(-B, B + 1), -(n - 1), n - 1)))
    c = np.concatenate([[0], np.cumsum(ds)])
    y0 = int(rng.integers(-c.min(), h - c.max()))
    img = np.zeros((h, w), np.uint8)
    y = y0
    for i, d in enumerate(ds):
        sg = -1 if d < 0 else 1
        for t, o in enumerate(pattern_rec(n, abs(d))):
            img[y + sg * o, i * n + t] = 9
        y += d
    s, ys = orc.detect_ex(img, k, bend=B, horizontal=True)
    assert s == 9 * w
    assert ys.tolist() == [int(y0 + v) for v in c]


def test_smoothing_spreads_a_thin_curve_but_keeps_its_path(orc):
    """A one-pixel planted curve on a flat background keeps its vertices after smoothing."""
    from tests.helpers import pattern_rec
    n, k, w = 16, 4, 48
    img = np.full((n * k, w), 10, np.uint8)
    x = 20
    for i, d in enumerate([3, 1, -1, -2]):
        sg = -1 if d < 0 else 1
        for t, o in enumerate(pattern_rec(n, abs(d))):
            img[i * n + t, x + sg * o] = 250
        x += d
    s0, xs0 = orc.detect_ex(img, k, bend=2)
    s2, xs2 = orc.detect_ex(img, k, bend=2, smooth_radius=2)
    assert xs2.tolist() == xs0.tolist()
    # center tap 6/16 of 250 plus 10/16 of 10, rounded half up, on every row
    assert s2 == n * k * ((6 * 250 + 10 * 10 + 8) // 16)


def test_detect_ex_validation(orc):
    img = np.zeros((16, 32), np.uint8)
    for kw, code in [(dict(smooth_radius=8), oracle.ERR_OPTION),
                     (dict(smooth_radius=-1), oracle.ERR_OPTION),
                     (dict(pin=(5, 0)), oracle.ERR_POINT),
                     (dict(pin=(1, 32)), oracle.ERR_POINT)]:
        with pytest.raises(oracle.OracleError) as e:
            orc.detect_ex(img, 4, bend=1, **kw)
        assert e.value.code == code, kw
    # horizontal: the bands split the 32 columns, so k = 3 does not divide
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_ex(img, 3, bend=1, horizontal=True)
    assert e.value.code == oracle.ERR_DIMS
    # horizontal pins index rows, so row 15 is fine and 16 is not
    orc.detect_ex(img, 4, bend=1, horizontal=True, pin=(2, 15))
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_ex(img, 4, bend=1, horizontal=True, pin=(2, 16))
    assert e.value.code == oracle.ERR_POINT

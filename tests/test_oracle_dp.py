"""Pins of the oracle's polyline optimum (Sections 2.1-2.3 and the main problem).

The oracle's dynamic programme is checked against brute-force enumeration of
every admissible polyline (scores walked pixel by pixel), closed forms (zero,
constant, planted model polyline, impulse), the unconstrained case against a
separately coded per-column maximum (Section 2.2), k = 1, the angle-form bend
windows, and invariants on the larger configurations.
"""

import math

import numpy as np
import pytest

import synth
from tests.helpers import (brute_force, enumerate_polylines, polyline_pixel_sum, pattern_rec,
                           vertices_to_shifts, admissible_pair)


def _rng(seed):
    return np.random.default_rng([191201884, 88, seed])


TINY = []
for n in (1, 2, 4):
    for k in (1, 2, 3):
        for w in (1, 2, 3, 5, 8):
            TINY.append((n, k, w))


@pytest.mark.parametrize("n,k,w", TINY)
def test_brute_force_tiny_mode0(orc, n, k, w):
    rng = _rng(n * 100 + k * 10 + w)
    h = n * k
    for trial in range(3):
        img = rng.integers(0, 4, size=(h, w)).astype(np.uint8)  # values {0..3}: tie-heavy
        for B in (0, 1, 2, 2 * n):
            want_s, want_x = brute_force(img, k, bend=B)
            got_s, got_x = orc.detect_polyline(img, k, bend=B)
            assert got_s == want_s, (trial, B)
            assert got_x.tolist() == want_x, (trial, B)


def _gamma_is_clear(n, gamma, margin=1e-9):
    """True when no pair of displacements has a bend within margin of gamma."""
    for d in range(-(n - 1), n):
        for dp in range(-(n - 1), n):
            if abs(abs(math.atan(dp / n) - math.atan(d / n)) - gamma) < margin:
                return False
    return True


@pytest.mark.parametrize("n,k,w", [(2, 2, 4), (4, 2, 6), (4, 3, 5), (8, 2, 9)])
def test_brute_force_tiny_mode1(orc, n, k, w):
    rng = _rng(n * 1000 + k * 10 + w)
    h = n * k
    gammas = [0.0, 0.05, 0.2, 0.5, 1.0, math.pi / 2, 3.0]
    for trial in range(2):
        img = rng.integers(0, 4, size=(h, w)).astype(np.uint8)
        for g in gammas:
            if 0 < g < math.pi / 2 and not _gamma_is_clear(n, g):
                continue
            want_s, want_x = brute_force(img, k, gamma=g)
            got_s, got_x = orc.detect_polyline(img, k, gamma=g)
            assert got_s == want_s, (trial, g)
            assert got_x.tolist() == want_x, (trial, g)


def test_brute_force_whole_64x64(orc):
    """Every admissible polyline of the 64x64 k=4 configuration, scores walked pixel by pixel."""
    s = synth.make_small()
    img = s.image.astype(np.int64)
    h, w, k, B = s.h, s.w, s.k, s.bend
    n = h // k
    # Link sums by walking pixels: L[i][x][d] for every link inside the image.
    L = np.full((k, w, 2 * n - 1), -1, dtype=np.int64)
    for i in range(k):
        for d in range(-(n - 1), n):
            pat = np.array(pattern_rec(n, abs(d)))
            sg = -1 if d < 0 else 1
            for x in range(w):
                if not (0 <= x + d < w):
                    continue
                cols = x + sg * pat
                L[i, x, d + n - 1] = int(img[i * n + np.arange(n), cols].sum())
    best, best_key = -1, None
    count = 0
    for x0 in range(w):
        for d0 in range(-(n - 1), n):
            if not (0 <= x0 + d0 < w):
                continue
            # extend depth-first over admissible continuations
            stack = [(1, x0 + d0, (d0,), int(L[0, x0, d0 + n - 1]))]
            while stack:
                i, x, ds, sc = stack.pop()
                if i == k:
                    count += 1
                    key = (x0,) + ds
                    if sc > best or (sc == best and key < best_key):
                        best, best_key = sc, key
                    continue
                dprev = ds[-1]
                for d in range(max(-(n - 1), dprev - B), min(n - 1, dprev + B) + 1):
                    if 0 <= x + d < w:
                        stack.append((i + 1, x + d, ds + (d,), sc + int(L[i, x, d + n - 1])))
    assert count > 10000
    got_s, got_x = orc.detect_polyline(s.image, k, bend=B)
    want_x = [best_key[0]]
    for d in best_key[1:]:
        want_x.append(want_x[-1] + d)
    assert got_s == best
    assert got_x.tolist() == want_x
    # The drawn 200-valued polyline is within reach, so the optimum follows it.
    assert polyline_pixel_sum(s.image, k, got_x[0], vertices_to_shifts(got_x)) == best


@pytest.mark.parametrize("h,w,k,B", [(64, 50, 4, 1), (32, 8, 2, 0), (128, 70, 8, 3)])
def test_zero_and_constant(orc, h, w, k, B):
    z = np.zeros((h, w), np.uint8)
    s, xs = orc.detect_polyline(z, k, bend=B)
    assert s == 0 and np.all(xs == 0)
    c = np.full((h, w), 37, np.uint8)
    s, xs = orc.detect_polyline(c, k, bend=B)
    assert s == 37 * h and np.all(xs == 0)


def _draw_model_polyline(img, k, x0, ds, v):
    h, w = img.shape
    n = h // k
    x = x0
    for i, d in enumerate(ds):
        sg = -1 if d < 0 else 1
        for y, o in enumerate(pattern_rec(n, abs(d))):
            img[i * n + y, x + sg * o] = v
        x += d


@pytest.mark.parametrize("seed", range(6))
def test_planted_model_polyline(orc, seed):
    rng = _rng(1000 + seed)
    k = int(rng.choice([2, 4, 8]))
    n = int(rng.choice([4, 8, 16]))
    h = n * k
    w = int(rng.integers(3 * n, 6 * n))
    B = int(rng.integers(0, 4))
    ds = [int(rng.integers(-(n - 1), n))]
    for _ in range(k - 1):
        ds.append(int(np.clip(ds[-1] + rng.integers(-B, B + 1), -(n - 1), n - 1)))
    c = np.concatenate([[0], np.cumsum(ds)])
    x0 = int(rng.integers(-c.min(), w - c.max()))
    img = np.zeros((h, w), np.uint8)
    _draw_model_polyline(img, k, x0, ds, 9)
    s, xs = orc.detect_polyline(img, k, bend=B)
    assert s == 9 * h
    assert xs.tolist() == [int(x0 + v) for v in c]


@pytest.mark.parametrize("seed", range(4))
def test_impulse_score(orc, seed):
    rng = _rng(2000 + seed)
    k, n, w, B = 4, 8, 20, 1
    h = k * n
    Y, X = int(rng.integers(h)), int(rng.integers(w))
    img = np.zeros((h, w), np.uint8)
    img[Y, X] = 5
    s, xs = orc.detect_polyline(img, k, bend=B)
    assert s == 5
    ds = vertices_to_shifts(xs)
    assert polyline_pixel_sum(img, k, int(xs[0]), ds) == 5


@pytest.mark.parametrize("B", [0, 1])
def test_escaping_streak_is_infeasible(orc, B):
    """A bright link whose only admissible continuations leave the image must not count.

    Band 0 holds a bright 45-degree streak ending on the last column; with a
    tight bend bound every continuation runs off the right edge, so polylines
    through it are infeasible and the optimum is found elsewhere.
    """
    h, w, k = 8, 6, 2
    n = h // k
    img = np.zeros((h, w), np.uint8)
    for y in range(n):
        img[y, 2 + y] = 255
    img[n:, 0] = 1
    want_s, want_x = brute_force(img, k, bend=B)
    got_s, got_x = orc.detect_polyline(img, k, bend=B)
    assert got_s == want_s and got_x.tolist() == want_x
    assert got_s < 4 * 255


def _unconstrained_dp(H, w, k):
    """Section 2.2: each step adds the maximum of the whole successor column (no bend limit)."""
    n = (H.shape[1] + 1) // 2
    D = 2 * n - 1
    d = np.arange(D) - (n - 1)
    x = np.arange(w)
    valid = (x[None, :] + d[:, None] >= 0) & (x[None, :] + d[:, None] < w)  # [D][w]
    V = np.where(valid, H[k - 1, :, :w].astype(np.int64), -1)
    for i in range(k - 2, -1, -1):
        colmax = V.max(axis=0)  # best continuation starting at each column
        nxt = np.full((D, w), -1, dtype=np.int64)
        for r in range(D):
            xp = x + d[r]
            ok = valid[r]
            cm = np.full(w, -1, dtype=np.int64)
            cm[ok] = colmax[xp[ok]]
            nxt[r] = np.where(ok & (cm >= 0), H[i, r, :w] + cm, -1)
        V = nxt
    return int(V.max())


@pytest.mark.parametrize("h,w,k", [(64, 64, 4), (128, 100, 8), (256, 77, 4)])
def test_unconstrained_equals_column_max_dp(orc, h, w, k):
    rng = _rng(h + w)
    img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
    n = h // k
    H = orc.fht_bands(img, k)
    want = _unconstrained_dp(H, w, k)
    for B in (2 * n - 2, 5 * n):
        s, _ = orc.polyline_dp(H, h, w, k, bend=B)
        assert s == want
    s, _ = orc.polyline_dp(H, h, w, k, gamma=math.pi / 2)
    assert s == want


def test_single_band_is_table_max(orc):
    rng = _rng(3)
    h, w = 16, 30
    img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
    H = orc.fht_bands(img, 1)
    n = h
    best = -1
    for r in range(2 * n - 1):
        d = r - (n - 1)
        for x in range(w):
            if 0 <= x + d < w and H[0, r, x] > best:
                best = int(H[0, r, x])
    s, xs = orc.detect_polyline(img, 1, bend=0)
    assert s == best
    assert H[0, xs[1] - xs[0] + n - 1, xs[0]] == best


def test_angle_window_properties(orc):
    for n in (4, 16, 128):
        lo, hi = orc.angle_window(n, 0.0)
        assert np.array_equal(lo, np.arange(2 * n - 1) - (n - 1))
        assert np.array_equal(hi, lo)
        lo, hi = orc.angle_window(n, math.pi / 2)
        assert np.all(lo == -(n - 1)) and np.all(hi == n - 1)
        for g in (0.03, 0.17, 0.6, 1.2):
            lo, hi = orc.angle_window(n, g)
            d = np.arange(2 * n - 1) - (n - 1)
            assert np.all(lo <= d) and np.all(d <= hi)
            assert np.all(np.diff(lo) >= 0) and np.all(np.diff(hi) >= 0)
            # symmetry: d' in W(d)  <=>  d in W(d')
            member = (d[None, :] >= lo[:, None]) & (d[None, :] <= hi[:, None])
            assert np.array_equal(member, member.T)
            if _gamma_is_clear(n, g):
                ang = np.arctan(d / n)
                want = np.abs(ang[None, :] - ang[:, None]) <= g
                assert np.array_equal(member, want)


def test_ten_degree_window_example(orc):
    """The 10 degree bend limit of the bent-document example (Fig. 3d) at n = 64."""
    n = 64
    g = math.radians(10)
    lo, hi = orc.angle_window(n, g)
    for d in (-40, 0, 25):
        r = d + n - 1
        for dp in range(-(n - 1), n):
            inside = lo[r] <= dp <= hi[r]
            assert inside == admissible_pair(n, d, dp, None, g)


def _check_invariants(img, k, B, score, xs):
    h, w = img.shape
    n = h // k
    ds = vertices_to_shifts(xs)
    assert all(0 <= int(x) < w for x in xs)
    assert all(abs(d) <= n - 1 for d in ds)
    assert all(abs(ds[i + 1] - ds[i]) <= B for i in range(k - 1))
    assert polyline_pixel_sum(img, k, int(xs[0]), ds) == score  # the polyline sum of 2.1
    return ds


def test_c2_invariants_and_local_optimality(orc):
    s = synth.make_medium()
    score, xs = orc.detect_polyline(s.image, s.k, bend=s.bend)
    ds = _check_invariants(s.image, s.k, s.bend, score, xs)
    # No single-vertex move (keeping everything else) finds a better admissible polyline.
    h, w, k, B = s.h, s.w, s.k, s.bend
    n = h // k
    xs = [int(v) for v in xs]
    for j in range(k + 1):
        for delta in (-2, -1, 1, 2):
            cand = list(xs)
            cand[j] += delta
            cds = vertices_to_shifts(cand)
            if not all(0 <= x < w for x in cand):
                continue
            if not all(abs(d) <= n - 1 for d in cds):
                continue
            if not all(abs(cds[i + 1] - cds[i]) <= B for i in range(k - 1)):
                continue
            assert polyline_pixel_sum(s.image, k, cand[0], cds) <= score


def test_from_top_matches_best_start(orc):
    rng = _rng(11)
    img = rng.integers(0, 9, size=(32, 12)).astype(np.uint8)
    k, B = 4, 1
    best = max(orc.detect_from_top(img, k, x0, bend=B)[0] for x0 in range(12))
    s, xs = orc.detect_polyline(img, k, bend=B)
    assert s == best
    s0, xs0 = orc.detect_from_top(img, k, int(xs[0]), bend=B)
    assert s0 == s and np.array_equal(xs0, xs)


def test_validation(orc):
    import oracle
    img = np.zeros((16, 8), np.uint8)
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_polyline(img, 2, bend=-1)
    assert e.value.code == oracle.ERR_BEND
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_polyline(img, 2, gamma=float("nan"))
    assert e.value.code == oracle.ERR_BEND
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_polyline(img, 3, bend=1)
    assert e.value.code == oracle.ERR_DIMS
    with pytest.raises(oracle.OracleError) as e:
        orc.detect_from_top(img, 2, 8, bend=1)
    assert e.value.code == oracle.ERR_POINT

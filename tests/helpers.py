"""Independent test-side references used to pin the oracle.

Nothing here is imported by the oracle or by the detector package.  These are
deliberately different formulations from the oracle's code: the dyadic
pattern by its recursive definition (not the oracle's closed form), polyline
scores by walking pixels one row at a time (not table lookups), and the
optimum by enumerating every admissible polyline.
"""

from __future__ import annotations

import itertools
import math
from functools import lru_cache
from typing import Iterable, List, Optional, Tuple

import numpy as np


@lru_cache(maxsize=None)
def pattern_rec(n: int, s: int) -> Tuple[int, ...]:
    """Dyadic pattern by its recursive definition: D^(1)_0 = (0,);
    upper half = D^(n/2)_{s//2}, lower half = ceil(s/2) + D^(n/2)_{s//2}."""
    if n == 1:
        assert s == 0
        return (0,)
    half = pattern_rec(n // 2, s // 2)
    up = (s + 1) // 2
    return half + tuple(up + v for v in half)


def line_columns(n: int, x: int, d: int) -> List[int]:
    s = abs(d)
    sg = -1 if d < 0 else 1
    return [x + sg * o for o in pattern_rec(n, s)]


def polyline_pixel_sum(img: np.ndarray, k: int, x0: int, ds: Iterable[int]) -> int:
    """Sum of one pixel per row along the polyline (x0; d_0..d_{k-1}), walked row by row."""
    h, w = img.shape
    n = h // k
    total = 0
    x = x0
    for i, d in enumerate(ds):
        for y, c in enumerate(line_columns(n, x, d)):
            assert 0 <= c < w
            total += int(img[i * n + y, c])
        x += d
    return total


def admissible_pair(n: int, d: int, dp: int, bend: Optional[int], gamma: Optional[float]) -> bool:
    """Bend test written with angles directly: |atan(d'/n) - atan(d/n)| <= gamma, or |d'-d| <= B."""
    if gamma is None:
        return abs(dp - d) <= bend
    return abs(math.atan(dp / n) - math.atan(d / n)) <= gamma


def enumerate_polylines(h: int, w: int, k: int, bend=None, gamma=None):
    """Every admissible (x0, d_0..d_{k-1}) with all vertices inside [0, w-1]."""
    n = h // k
    rng = range(-(n - 1), n)
    for x0 in range(w):
        for ds in itertools.product(rng, repeat=k):
            ok = True
            x = x0
            for i, d in enumerate(ds):
                x += d
                if not (0 <= x < w):
                    ok = False
                    break
                if i > 0 and not admissible_pair(n, ds[i - 1], d, bend, gamma):
                    ok = False
                    break
            if ok:
                yield x0, ds


def brute_force(img: np.ndarray, k: int, bend=None, gamma=None) -> Tuple[int, List[int]]:
    """Best score and vertices; ties go to the lexicographically smallest (x0, d_0, ...)."""
    h, w = img.shape
    best = None
    best_key = None
    for x0, ds in enumerate_polylines(h, w, k, bend, gamma):
        sc = polyline_pixel_sum(img, k, x0, ds)
        key = (x0,) + tuple(ds)
        if best is None or sc > best or (sc == best and key < best_key):
            best, best_key = sc, key
    x0 = best_key[0]
    xs = [x0]
    for d in best_key[1:]:
        xs.append(xs[-1] + d)
    return best, xs


def vertices_to_shifts(xs) -> List[int]:
    return [int(xs[i + 1] - xs[i]) for i in range(len(xs) - 1)]


def fast_fht_stages(band: np.ndarray, W: int, sign: int):
    """The dyadic shift-and-add recursion on one zero-extended band, with an add counter.

    Stage j merges blocks of 2^(j-1) rows into blocks of 2^j rows:
        T_j(b, x, s) = T_{j-1}(2b, x, s//2) + T_{j-1}(2b+1, x + sign*ceil(s/2) mod W, s//2).
    Returns (T_p[s][x] for s in [0, n), number of scalar additions).
    """
    n, w = band.shape
    ext = np.zeros((n, W), dtype=np.int64)
    ext[:, :w] = band
    # T[b] is an array [2^j][W] for block b.
    T = [ext[r:r + 1, :].copy() for r in range(n)]
    adds = 0
    size = 1
    while size < n:
        nxt = []
        for b in range(len(T) // 2):
            top, bot = T[2 * b], T[2 * b + 1]
            out = np.zeros((2 * size, W), dtype=np.int64)
            for s in range(2 * size):
                half = s // 2
                up = (s + 1) // 2
                out[s] = top[half] + np.roll(bot[half], -sign * up)
                adds += W
            nxt.append(out)
        T = nxt
        size *= 2
    return T[0], adds

"""Seeded synthetic images with drawn top-to-bottom polylines.

Every image is drawn from ``np.random.default_rng(SeedSequence([SEED_ROOT,
config, image]))``, so a (config, image) pair always gives the same pixels.

A drawn polyline has ``k`` links, one per horizontal band of ``n = h/k`` rows
(the k-division of Section 2).  Link ``i`` starts at column ``x_i`` on the
first row of band ``i`` and its horizontal displacement over the band is
``d_i``, so ``x_{i+1} = x_i + d_i``.  Row ``r`` of link ``i`` is painted at
column ``x_i + floor((2*d_i*r + n) / (2n))``: the nearest column to the
straight segment between the two vertices.  This rasterisation is a plain
rounding rule and deliberately not the dyadic line pattern the detector sums
along, so a drawn curve is something the detector has to approximate.

Nothing in this module computes line sums or runs the detector.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SEED_ROOT = 191201884


@dataclass
class Polyline:
    """One drawn polyline: ``x`` holds the k+1 vertex columns, ``d`` the k shifts."""

    x: np.ndarray
    d: np.ndarray
    value: int
    width: int


@dataclass
class SynthImage:
    """A generated image and the parameters it was drawn with."""

    image: np.ndarray          # [h][w], uint8 or uint16, row-major
    h: int
    w: int
    k: int
    bend: int                  # |d_{i+1} - d_i| bound used when drawing (and detecting)
    polylines: List[Polyline] = field(default_factory=list)
    config: str = ""

    @property
    def n(self) -> int:
        return self.h // self.k

    @property
    def dtype_code(self) -> int:
        return 0 if self.image.dtype == np.uint8 else 1


def rng_for(config: int, image: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, config, image]))


def random_walk_shifts(rng: np.random.Generator, k: int, R: int, B: int) -> np.ndarray:
    """Shifts of a bend-limited random walk: d_0 ~ U{-R..R}, then +U{-B..B}, clipped to +-R."""
    d = np.empty(k, dtype=np.int64)
    d[0] = rng.integers(-R, R + 1)
    for i in range(1, k):
        d[i] = min(R, max(-R, d[i - 1] + rng.integers(-B, B + 1)))
    return d


def uniform_bend_limited_shifts(rng: np.random.Generator, k: int, R: int, B: int,
                                max_tries: int = 200000) -> np.ndarray:
    """Shifts drawn uniformly over {-R..R}^k subject to |d_{i+1}-d_i| <= B (by rejection)."""
    for _ in range(max_tries):
        d = rng.integers(-R, R + 1, size=k)
        if k == 1 or np.all(np.abs(np.diff(d)) <= B):
            return d.astype(np.int64)
    return random_walk_shifts(rng, k, R, B)


def place_x0(rng: np.random.Generator, d: np.ndarray, w: int) -> Optional[int]:
    """Draw x_0 uniformly among the starts that keep every vertex inside [0, w-1]."""
    c = np.concatenate([[0], np.cumsum(d)])
    lo = int(-c.min())
    hi = int(w - 1 - c.max())
    if lo > hi:
        return None
    return int(rng.integers(lo, hi + 1))


def draw_shifts_and_start(rng, k, R, B, w, uniform=False) -> Tuple[int, np.ndarray]:
    for _ in range(1000):
        d = uniform_bend_limited_shifts(rng, k, R, B) if uniform else random_walk_shifts(rng, k, R, B)
        x0 = place_x0(rng, d, w)
        if x0 is not None:
            return x0, d
    # The walk never fits (only possible for very narrow images): draw a vertical line.
    d = np.zeros(k, dtype=np.int64)
    return int(rng.integers(0, w)), d


def raster_columns(x0: int, d: np.ndarray, n: int) -> np.ndarray:
    """Column of the drawn curve on every image row (length k*n)."""
    k = len(d)
    cols = np.empty(k * n, dtype=np.int64)
    r = np.arange(n, dtype=np.int64)
    x = x0
    for i in range(k):
        cols[i * n:(i + 1) * n] = x + (2 * d[i] * r + n) // (2 * n)
        x += int(d[i])
    return cols


def draw_polyline(img: np.ndarray, x0: int, d: np.ndarray, n: int, width: int,
                  value: int, additive: bool = False) -> np.ndarray:
    """Paint a polyline into ``img`` in place; returns the flat indices painted."""
    h, w = img.shape
    cols = raster_columns(x0, d, n)
    rows = np.arange(h, dtype=np.int64)
    painted = []
    for off in range(width):
        c = cols + off
        ok = (c >= 0) & (c < w)
        painted.append(rows[ok] * w + c[ok])
    idx = np.unique(np.concatenate(painted))
    flat = img.reshape(-1)
    if additive:
        top = np.iinfo(img.dtype).max
        flat[idx] = np.minimum(flat[idx].astype(np.int64) + value, top).astype(img.dtype)
    else:
        flat[idx] = value
    return idx


def _gauss_bg(rng, shape, mean, sd, dtype=np.uint8):
    v = np.rint(rng.normal(mean, sd, size=shape))
    return np.clip(v, 0, np.iinfo(dtype).max).astype(dtype)


def _poly_record(x0, d, value, width) -> Polyline:
    x = np.concatenate([[x0], x0 + np.cumsum(d)]).astype(np.int64)
    return Polyline(x=x, d=d.astype(np.int64), value=int(value), width=int(width))


def make_small(image: int = 0) -> SynthImage:
    """64x64 uint8, k=4 (16-row bands): N(20,10) noise, one 1-px polyline of value 200, bend 1."""
    rng = rng_for(1, image)
    h = w = 64
    k, B, R = 4, 1, 16
    n = h // k
    img = _gauss_bg(rng, (h, w), 20.0, 10.0)
    x0, d = draw_shifts_and_start(rng, k, R, B, w, uniform=True)
    draw_polyline(img, x0, d, n, 1, 200)
    return SynthImage(img, h, w, k, B, [_poly_record(x0, d, 200, 1)], "64x64")


def _noisy_curves(rng, h, w, k, B, n_curves=3) -> Tuple[np.ndarray, List[Polyline]]:
    n = h // k
    R = max(1, n // 4)
    img = _gauss_bg(rng, (h, w), 30.0, 15.0)
    drawn = []
    polys = []
    for _ in range(n_curves):
        value = int(rng.integers(120, 221))
        width = int(rng.integers(1, 3))
        x0, d = draw_shifts_and_start(rng, k, R, B, w)
        drawn.append(draw_polyline(img, x0, d, n, width, value))
        polys.append(_poly_record(x0, d, value, width))
    idx = np.unique(np.concatenate(drawn))
    n_occ = int(round(0.10 * idx.size))
    if n_occ:
        occ = rng.choice(idx, size=n_occ, replace=False)
        img.reshape(-1)[occ] = _gauss_bg(rng, (n_occ,), 30.0, 15.0)
    return img, polys


def make_medium(image: int = 0) -> SynthImage:
    """1024x1024 uint8, k=16 (64-row bands): N(30,15) noise, 3 polylines, 10% occluded, bend 4."""
    rng = rng_for(2, image)
    h = w = 1024
    k, B = 16, 4
    img, polys = _noisy_curves(rng, h, w, k, B)
    return SynthImage(img, h, w, k, B, polys, "1024x1024")


def make_large(image: int = 0, h: int = 4096, w: int = 4096, k: int = 32) -> SynthImage:
    """4096x4096 uint16, k=32 (128-row bands): Exp(500) noise plus 8 additive polylines, bend 8."""
    rng = rng_for(3, image)
    B = 8
    n = h // k
    R = max(1, n // 4)
    v = np.rint(rng.exponential(500.0, size=(h, w)))
    img = np.clip(v, 0, 65535).astype(np.uint16)
    polys = []
    for _ in range(8):
        amp = int(rng.integers(4000, 12001))
        x0, d = draw_shifts_and_start(rng, k, R, B, w)
        draw_polyline(img, x0, d, n, 1, amp, additive=True)
        polys.append(_poly_record(x0, d, amp, 1))
    return SynthImage(img, h, w, k, B, polys, "4096x4096")


MIXED_HEIGHTS = (128, 256, 512, 1024, 2048)
MIXED_KS = (4, 8, 16)


def make_mixed_image(image: int) -> SynthImage:
    """One image of the mixed-size batch: h in {128..2048}, w ~ U{256..2048}, k in {4,8,16}."""
    rng = rng_for(4, image)
    h = int(rng.choice(MIXED_HEIGHTS))
    w = int(rng.integers(256, 2049))
    k = int(rng.choice(MIXED_KS))
    B = 4
    img, polys = _noisy_curves(rng, h, w, k, B)
    return SynthImage(img, h, w, k, B, polys, "mixed")


def make_mixed_batch(count: int = 256) -> List[SynthImage]:
    return [make_mixed_image(j) for j in range(count)]


CONFIGS = {
    "64x64": dict(h=64, w=64, k=4, bend=1, dtype="u8"),
    "1024x1024": dict(h=1024, w=1024, k=16, bend=4, dtype="u8"),
    "4096x4096": dict(h=4096, w=4096, k=32, bend=8, dtype="u16"),
}


def make_config(name: str, image: int = 0) -> SynthImage:
    if name == "64x64":
        return make_small(image)
    if name == "1024x1024":
        return make_medium(image)
    if name == "4096x4096":
        return make_large(image)
    if name == "mixed":
        return make_mixed_image(image)
    raise ValueError(f"unknown config {name!r}")


def random_small(rng: np.random.Generator, h: int, w: int, maxval: int = 3,
                 dtype=np.uint8) -> np.ndarray:
    """Tie-heavy tiny image with values in {0..maxval} (for brute-force checks)."""
    return rng.integers(0, maxval + 1, size=(h, w)).astype(dtype)

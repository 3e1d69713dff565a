"""Pins of the oracle's band tables H_i(x, d) (Section 2.1).

Checked against facts that do not depend on the oracle's code: single-pixel
impulses land at the one position per shift the line geometry predicts,
every shift's lines partition the band (conservation), one-row bands are the
pixels themselves, constant images give c*n for lines inside the image, and
the FHT's fast stage recursion reproduces the direct sums with exactly
p*n*W additions per band and direction (the O((w+h/k)*(h/k)*log(h/k)) cost).
"""

import numpy as np
import pytest

from tests.helpers import pattern_rec, fast_fht_stages


def _rng(seed):
    return np.random.default_rng([191201884, 77, seed])


@pytest.mark.parametrize("h,w,k", [(8, 5, 2), (16, 9, 2), (16, 16, 1), (32, 7, 4), (64, 40, 4)])
def test_impulse(orc, h, w, k):
    n = h // k
    W = w + n
    rng = _rng(h * 1000 + w)
    spots = [(0, 0), (h - 1, w - 1), (n - 1, 0), (h // 2, w // 2)]
    spots += [(int(rng.integers(h)), int(rng.integers(w))) for _ in range(4)]
    for (Y, X) in spots:
        img = np.zeros((h, w), np.uint8)
        img[Y, X] = 7
        H = orc.fht_bands(img, k)
        band, y = divmod(Y, n)
        for i in range(k):
            if i != band:
                assert not H[i].any()
        for r in range(2 * n - 1):
            d = r - (n - 1)
            sg = -1 if d < 0 else 1
            x = (X - sg * pattern_rec(n, abs(d))[y]) % W
            row = H[band, r]
            assert row[x] == 7, (Y, X, d)
            assert np.count_nonzero(row) == 1, (Y, X, d)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
@pytest.mark.parametrize("h,w,k", [(16, 13, 2), (32, 32, 4), (64, 31, 2), (128, 50, 4), (8, 3, 8)])
def test_conservation(orc, dtype, h, w, k):
    """For each shift the lines of a band cover every band pixel exactly once."""
    rng = _rng(h + w + k)
    top = np.iinfo(dtype).max
    img = rng.integers(0, top + 1, size=(h, w)).astype(dtype)
    H = orc.fht_bands(img, k).astype(np.int64)
    n = h // k
    for i in range(k):
        total = int(img[i * n:(i + 1) * n].astype(np.int64).sum())
        assert np.all(H[i].sum(axis=1) == total)


def test_one_row_bands_are_pixels(orc):
    rng = _rng(5)
    img = rng.integers(0, 256, size=(6, 11)).astype(np.uint8)
    H = orc.fht_bands(img, 6)
    assert H.shape == (6, 1, 12)
    assert np.array_equal(H[:, 0, :11], img.astype(np.int32))
    assert not H[:, 0, 11].any()


@pytest.mark.parametrize("h,w,k,c", [(32, 20, 2, 9), (64, 64, 4, 200), (16, 5, 1, 3)])
def test_constant_image(orc, h, w, k, c):
    n = h // k
    W = w + n
    img = np.full((h, w), c, np.uint8)
    H = orc.fht_bands(img, k)
    for i in range(k):
        for r in range(2 * n - 1):
            d = r - (n - 1)
            for x in range(W):
                inside = 0 <= x < w and 0 <= x + d < w
                if inside:  # the pattern is monotone, so both ends inside means all inside
                    assert H[i, r, x] == c * n


@pytest.mark.parametrize("h,w,k", [(8, 6, 1), (16, 11, 2), (32, 9, 1), (64, 20, 2)])
def test_fast_recursion_matches_direct_sum_and_counts(orc, h, w, k):
    rng = _rng(h * 7 + w)
    img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
    H = orc.fht_bands(img, k).astype(np.int64)
    n = h // k
    p = n.bit_length() - 1
    W = w + n
    for i in range(k):
        band = img[i * n:(i + 1) * n].astype(np.int64)
        right, adds_r = fast_fht_stages(band, W, +1)
        left, adds_l = fast_fht_stages(band, W, -1)
        for s in range(n):
            assert np.array_equal(right[s], H[i, n - 1 + s])
            assert np.array_equal(left[s], H[i, n - 1 - s])
        # p stages, each producing n rows of W sums: the paper's per-band FHT cost.
        assert adds_r == adds_l == p * n * W


def test_validation(orc):
    import oracle
    img = np.zeros((12, 8), np.uint8)
    with pytest.raises(oracle.OracleError) as e:
        orc.fht_bands(img, 4)  # n = 3 is not a power of two
    assert e.value.code == oracle.ERR_DIMS
    with pytest.raises(oracle.OracleError) as e:
        orc.fht_bands(np.zeros((12, 8), np.uint8), 5)  # k does not divide h
    assert e.value.code == oracle.ERR_DIMS
    big = np.zeros((65536, 1), np.uint16)
    with pytest.raises(oracle.OracleError) as e:
        orc.fht_bands(big, 65536)  # h * 65535 >= 2^31
    assert e.value.code == oracle.ERR_OVERFLOW

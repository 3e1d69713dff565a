"""Pins of the oracle's dyadic line pattern (Section 2.1 uses the FHT's dyadic lines).

The oracle computes D_s(y) by a closed form; these tests check it against the
recursive definition, hand-written golden patterns and the endpoint/step
properties every digital line of the FHT must have.
"""

import os

import numpy as np
import pytest

from tests.helpers import pattern_rec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dyadic_patterns.txt")


@pytest.mark.parametrize("p", range(0, 11))
def test_closed_form_equals_recursion(orc, p):
    n = 1 << p
    for s in range(n):
        got = orc.dyadic_pattern(n, s)
        assert tuple(int(v) for v in got) == pattern_rec(n, s), (n, s)


@pytest.mark.parametrize("p", range(0, 11))
def test_endpoints_and_steps(orc, p):
    n = 1 << p
    for s in range(n):
        D = orc.dyadic_pattern(n, s).astype(np.int64)
        assert D[0] == 0
        assert D[-1] == s  # the line is displaced by exactly s over the band
        steps = np.diff(D)
        assert np.all((steps == 0) | (steps == 1))  # 8-connected, mostly vertical
    assert np.all(orc.dyadic_pattern(n, 0) == 0)  # vertical line: column sums
    assert np.all(orc.dyadic_pattern(n, n - 1) == np.arange(n))  # exact 45 degree diagonal


def test_golden_patterns(orc):
    """Patterns for n = 4 and n = 8 written out by hand from the recursive definition."""
    seen = 0
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            n_s, pat = line.split(":")
            n, s = (int(v) for v in n_s.split())
            want = [int(c) for c in pat.split()]
            assert orc.dyadic_pattern(n, s).tolist() == want, (n, s)
            seen += 1
    assert seen == 4 + 8


def test_bad_arguments(orc):
    import oracle
    for n, s in [(3, 0), (0, 0), (4, 4), (4, -1), (2048, 0)]:
        with pytest.raises(oracle.OracleError):
            orc.dyadic_pattern(n, s)

"""Plant plausible mistakes in the oracle (on the CPU) and check the pins catch each one.

Every mutant is the oracle's C source with one small textual change (a dropped
term, a flipped sign, a wrong tie rule, an off-by-one window), compiled into a
temporary library.  The pin tests are then run against that library; at
least one of them must fail, otherwise the pins would not notice the mistake.
"""

import math
import os
import tempfile

import numpy as np
import pytest

import oracle
from oracle import build as obuild
from tests import test_oracle_dp as tdp
from tests import test_oracle_options as topt
from tests import test_oracle_pattern as tpat
from tests import test_oracle_tables as ttab

MUTANTS = {
    "pattern_floor_offset": ("off += (s >> (j + 1)) + ((s >> j) & 1);", "off += (s >> (j + 1));"),
    "pattern_bit_order": ("if ((y >> (p - 1 - j)) & 1)", "if ((y >> j) & 1)"),
    "tables_clamp_not_wrap": ("if (c >= W) c -= W;", "if (c >= W) c = W - 1;"),
    "tables_left_lines_lean_right": ("const int sigma = d < 0 ? -1 : 1;", "const int sigma = 1;"),
    "dp_tie_largest_successor": ("if (!have || v > best) {", "if (!have || v >= best) {"),
    "dp_no_feasibility_check": ("(have && best >= 0 && !pinned_out(i, k, x, d, pin_j, pin_x))",
                                "(have && !pinned_out(i, k, x, d, pin_j, pin_x))"),
    "dp_window_too_narrow": ("return diff <= bound;", "return diff < bound;"),
    "dp_last_band_unmasked": ("(x + d >= 0 && x + d < w && !pinned_out(k - 1, k, x, d, pin_j, pin_x))",
                              "(!pinned_out(k - 1, k, x, d, pin_j, pin_x))"),
    "argmax_tie_last": ("            if (v > best) {\n                best = v;\n                bx = x;",
                        "            if (v >= best) {\n                best = v;\n                bx = x;"),
    "backtrace_last_vertex": ("xs[k] = x + d;", "xs[k] = x;"),
    "pin_last_vertex_is_link_start": ("return x + d != pin_x;", "return x != pin_x;"),
    "pin_one_band_late": ("if (pin_j == i && i < k) return x != pin_x;",
                          "if (pin_j == i + 1 && i < k) return x != pin_x;"),
    "smooth_truncates": ("const int64_t v = (acc + half) >> (2 * radius);",
                         "const int64_t v = acc >> (2 * radius);"),
    "smooth_reflects_edge": ("if (c < 0) c = 0;", "if (c < 0) c = -c;"),
    "smooth_wrong_coefficients": ("coef[i] = coef[i - 1] * (2 * radius - i + 1) / i;",
                                  "coef[i] = coef[i - 1] * (2 * radius - i + 2) / (i + 1);"),
    "horizontal_not_transposed": ("const size_t dst = orientation ? (size_t)x * h + y : src;",
                                  "const size_t dst = src;"),
    "angle_drop_cross_term": ("tan_gamma * ((double)n * (double)n + (double)d * (double)dp)",
                              "tan_gamma * ((double)n * (double)n)"),
}


def _pins():
    """(name, callable(orc)) for the pins run against each mutant."""
    return [
        ("pattern_recursion", lambda o: [tpat.test_closed_form_equals_recursion(o, p)
                                         for p in range(1, 7)]),
        ("pattern_golden", tpat.test_golden_patterns),
        ("impulse", lambda o: [ttab.test_impulse(o, *a) for a in [(16, 9, 2), (32, 7, 4)]]),
        ("conservation", lambda o: ttab.test_conservation(o, np.uint8, 32, 32, 4)),
        ("fast_recursion", lambda o: ttab.test_fast_recursion_matches_direct_sum_and_counts(
            o, 16, 11, 2)),
        ("brute_tiny_mode0", lambda o: [tdp.test_brute_force_tiny_mode0(o, *a)
                                        for a in [(2, 2, 5), (4, 2, 5), (4, 3, 3), (2, 3, 8)]]),
        ("brute_tiny_mode1", lambda o: [tdp.test_brute_force_tiny_mode1(o, *a)
                                        for a in [(4, 2, 6), (8, 2, 9)]]),
        ("brute_64x64", tdp.test_brute_force_whole_64x64),
        ("zero_constant", lambda o: tdp.test_zero_and_constant(o, 64, 50, 4, 1)),
        ("planted", lambda o: [tdp.test_planted_model_polyline(o, s) for s in range(3)]),
        ("unconstrained", lambda o: tdp.test_unconstrained_equals_column_max_dp(o, 64, 64, 4)),
        ("angle_windows", tdp.test_angle_window_properties),
        ("escaping_streak", lambda o: [tdp.test_escaping_streak_is_infeasible(o, b)
                                       for b in (0, 1)]),
        ("through_brute", lambda o: [topt.test_through_point_brute_force_mode0(o, *a)
                                     for a in [(2, 2, 4), (4, 3, 5), (4, 1, 7)]]),
        ("through_halves", lambda o: topt.test_unbounded_bend_equals_paper_halves(o, 0)),
        ("smooth_impulse", lambda o: [topt.test_smoothing_impulse_response_is_binomial(o, r)
                                      for r in (1, 3)]),
        ("smooth_library", lambda o: topt.test_smoothing_matches_library_convolution(
            o, 2, np.uint8)),
        ("smooth_narrow", topt.test_smoothing_narrow_rows),
        ("horizontal", lambda o: topt.test_horizontal_is_the_transposed_problem(o, 0)),
        ("horizontal_planted", lambda o: topt.test_planted_horizontal_polyline(o, 0)),
    ]


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory() as d:
        yield d


def test_unmutated_source_passes_every_pin(workdir):
    out = obuild.build(out=os.path.join(workdir, "base.so"))
    o = oracle.Oracle(out)
    for name, pin in _pins():
        pin(o)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(workdir, name):
    before, after = MUTANTS[name]
    with open(obuild.SRC) as f:
        src = f.read()
    assert src.count(before) == 1, f"mutation anchor for {name} not found exactly once"
    msrc = os.path.join(workdir, f"{name}.c")
    with open(msrc, "w") as f:
        f.write(src.replace(before, after))
    o = oracle.Oracle(obuild.build(src=msrc, out=os.path.join(workdir, f"{name}.so")))
    caught = []
    for pin_name, pin in _pins():
        try:
            pin(o)
        except (AssertionError, oracle.OracleError):
            caught.append(pin_name)
    assert caught, f"no pin notices the mutation {name}"

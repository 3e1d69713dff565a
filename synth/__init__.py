"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package draws images only.  It holds none of the detector's arithmetic
(no dyadic lines, no band sums, no dynamic programme), so the CPU oracle and
the GPU path can both be fed from it without sharing any of the method.
"""

from .images import (  # noqa: F401
    SEED_ROOT,
    Polyline,
    SynthImage,
    draw_polyline,
    random_walk_shifts,
    make_c1,
    make_c2,
    make_c3,
    make_c4_image,
    make_c4_batch,
    make_config,
    CONFIGS,
)

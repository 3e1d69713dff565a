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
    make_small,
    make_medium,
    make_large,
    make_mixed_image,
    make_mixed_batch,
    make_config,
    CONFIGS,
)

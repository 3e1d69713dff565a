"""CPU oracle for the FHT + bend-limited DP polyline detector.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the detector package.  It shares no
code with the HIP path.
"""

from .oracle import (  # noqa: F401
    ERR_NULL, ERR_DIMS, ERR_BEND, ERR_OVERFLOW, ERR_UNSUPPORTED, ERR_DTYPE, ERR_POINT, ERR_OPTION,
    Oracle,
    OracleError,
    lib,
    num_threads,
    dyadic_pattern,
    table_shape,
    fht_bands,
    polyline_dp,
    detect_polyline,
    detect_from_top,
    angle_window,
    detect_through_point,
    smooth_rows,
    detect_ex,
)

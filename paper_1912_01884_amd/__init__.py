"""MI355X-native detector of end-to-end curves of limited curvature.

The k-link polyline with the largest pixel sum and a bounded bend between
links, found with a band-wise Fast Hough Transform and a bottom-up dynamic
programme (Panfilova, Aliev, Kunina, Postnikov, Nikolaev).  The work runs in
hand-written HIP kernels for gfx950 behind the C ABI in include/fhtp.h;
``fhtp`` is the Python binding.
"""

from . import fhtp  # noqa: F401
from .fhtp import (  # noqa: F401
    Bend, FhtpError, make_bend, table_shape, fht_bands, polyline_dp, detect_polyline,
    fht_workspace_bytes, dp_workspace_bytes, detect_workspace_bytes, detect_batch,
    batch_workspace_bytes, Job, Options, make_options, detect_polyline_ex,
    detect_ex_workspace_bytes, prepare_image,
)

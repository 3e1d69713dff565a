"""CPU checks of the C ABI: the library loads, exports every declared entry point,
and rejects invalid requests on the host before touching the GPU.

No compute call here passes validation, so nothing is ever enqueued.
"""

import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1912_01884_amd import fhtp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhtp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fhtp_[a-z0-9_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_symbol():
    L = fhtp.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), f"{name} declared in fhtp.h but not exported"
    assert set(names) == set(fhtp.EXPORTED)
    assert "gfx950" in fhtp.version()


def test_error_strings():
    for code in range(0, -10, -1):
        assert fhtp.strerror(code) != "unknown error"
    assert fhtp.strerror(-99) == "unknown error"


@pytest.mark.parametrize("h,w,k", [(64, 64, 4), (1024, 1024, 16), (4096, 4096, 32), (8, 1, 8),
                                   (2048, 300, 4)])
def test_table_shape_matches_oracle(orc, h, w, k):
    assert fhtp.table_shape(h, w, k) == orc.table_shape(h, w, k)


BAD_SHAPES = [
    (0, 8, 1), (8, 0, 1), (8, 8, 0), (-8, 8, 1),
    (12, 8, 4),            # n = 3
    (12, 8, 5),            # k does not divide h
    (4096, 8, 2),          # n = 2048 > 1024
    (64, (1 << 20) + 1, 4),  # w too wide
]


@pytest.mark.parametrize("h,w,k", BAD_SHAPES)
def test_bad_shapes_rejected(h, w, k):
    with pytest.raises(fhtp.FhtpError) as e:
        fhtp.table_shape(h, w, k)
    assert e.value.code == fhtp.ERR_DIMS
    b = fhtp.make_bend(1)
    for q in (lambda: fhtp.fht_workspace_bytes(0, h, w, k),
              lambda: fhtp.dp_workspace_bytes(h, w, k, b),
              lambda: fhtp.detect_workspace_bytes(0, h, w, k, b)):
        with pytest.raises(fhtp.FhtpError) as e:
            q()
        assert e.value.code == fhtp.ERR_DIMS


def test_overflow_and_dtype_rejected():
    b = fhtp.make_bend(1)
    with pytest.raises(fhtp.FhtpError) as e:
        fhtp.detect_workspace_bytes(1, 65536, 4, 65536, b)  # 65536 * 65535 >= 2^31
    assert e.value.code == fhtp.ERR_OVERFLOW
    assert fhtp.detect_workspace_bytes(1, 32768, 4, 32768, b) > 0  # just below the limit
    with pytest.raises(fhtp.FhtpError) as e:
        fhtp.detect_workspace_bytes(2, 64, 64, 4, b)
    assert e.value.code == fhtp.ERR_DTYPE


@pytest.mark.parametrize("bend", [fhtp.Bend(0, -1, 0.0), fhtp.Bend(2, 1, 0.0),
                                  fhtp.Bend(1, 0, -0.1), fhtp.Bend(1, 0, float("nan")),
                                  fhtp.Bend(1, 0, float("inf"))])
def test_bad_bend_rejected(bend):
    with pytest.raises(fhtp.FhtpError) as e:
        fhtp.dp_workspace_bytes(64, 64, 4, bend)
    assert e.value.code == fhtp.ERR_BEND


def test_validation_matches_oracle(orc):
    """Both implementations reject the same shapes with the same codes."""
    import oracle
    for (h, w, k) in BAD_SHAPES[:7]:
        img = np.zeros((max(h, 1), max(w, 1)), np.uint8)
        rc_o = orc.L.oracle_detect_polyline(img.ctypes.data, 0, h, w, k, 0, 1, 0.0,
                                            np.zeros(1, np.int32).ctypes.data_as(
                                                C.POINTER(C.c_int32)),
                                            np.zeros(64, np.int32).ctypes.data_as(
                                                C.POINTER(C.c_int32)))
        with pytest.raises(fhtp.FhtpError) as e:
            fhtp.detect_workspace_bytes(0, h, w, k, fhtp.make_bend(1))
        assert e.value.code == rc_o == oracle.ERR_DIMS


def test_workspace_sizes_cover_the_buffers():
    h, w, k = 4096, 4096, 32
    n = h // k
    b = fhtp.make_bend(8)
    tables = k * (2 * n - 1) * (w + n) * 4
    backptr = (k - 2) * (2 * n - 1) * w  # uint8 back-pointers for D <= 256
    planes = 2 * (2 * n - 1) * w * 4
    dp = fhtp.dp_workspace_bytes(h, w, k, b)
    assert dp >= backptr + planes
    det = fhtp.detect_workspace_bytes(1, h, w, k, b)
    assert det >= dp + tables
    assert fhtp.fht_workspace_bytes(1, h, w, k) == 0
    # bands of 512 rows need sub-block scratch (128-row line sums: uint16 cells
    # for 8-bit pixels, at most 128 * 255; int32 for 16-bit ones) and uint16
    # back-pointers
    assert fhtp.fht_workspace_bytes(0, 2048, 1000, 4) == (2048 // 128) * 2 * 128 * 1512 * 2
    assert fhtp.fht_workspace_bytes(1, 2048, 1000, 4) == (2048 // 128) * 2 * 128 * 1512 * 4
    assert fhtp.dp_workspace_bytes(2048, 1000, 4, b) >= 2 * 1023 * 1000 * 2


def test_narrow_tables_shrink_the_workspace_exactly_where_they_are_exact():
    """8-bit pixels with bands of at most 256 rows keep bands 0..k-2 as uint16
    (a line sum is at most 256 * 255 < 2^16); the last band stays int32."""
    b = fhtp.make_bend(4)
    for h, w, k in [(1024, 1024, 16), (2048, 777, 8), (512, 300, 2), (256, 100, 1)]:
        n = h // k
        band = (2 * n - 1) * (w + n)
        dp = fhtp.dp_workspace_bytes(h, w, k, b)
        det8 = fhtp.detect_workspace_bytes(0, h, w, k, b)
        det16 = fhtp.detect_workspace_bytes(1, h, w, k, b)
        assert det16 >= dp + k * band * 4
        narrow = k - 1 if k >= 2 else 0
        assert det8 >= dp + narrow * band * 2 + (k - narrow) * band * 4
        if k >= 2:
            assert det8 < det16 - narrow * band * 2 + 4096  # only alignment on top
    # 512-row bands of 8-bit pixels could reach 130,560: int32 tables; only
    # the two-pass FHT's sub-block scratch is narrower (uint16 cells)
    h, w, k = 2048, 500, 4
    scratch16 = (h // 128) * 2 * 128 * (w + 512) * 2
    d8 = fhtp.detect_workspace_bytes(0, h, w, k, b)
    d16 = fhtp.detect_workspace_bytes(1, h, w, k, b)
    assert 0 <= d16 - d8 - scratch16 < 1024  # alignment only


def test_compute_calls_validate_before_launch():
    L = fhtp.lib()
    b = fhtp.make_bend(1)
    dummy = C.c_void_p(256)  # never dereferenced: every call below fails validation
    i32 = C.c_void_p(256)
    assert L.fhtp_fht_bands(None, 0, 64, 64, 4, i32, None, 0, None) == fhtp.ERR_NULL
    assert L.fhtp_fht_bands(dummy, 0, 64, 64, 3, i32, None, 0, None) == fhtp.ERR_DIMS
    assert L.fhtp_fht_bands(dummy, 5, 64, 64, 4, i32, None, 0, None) == fhtp.ERR_DTYPE
    # tall bands need scratch: a missing or short workspace is refused
    assert L.fhtp_fht_bands(dummy, 0, 1024, 64, 4, i32, None, 0, None) == fhtp.ERR_NULL
    assert L.fhtp_fht_bands(dummy, 0, 1024, 64, 4, i32, dummy, 16, None) == fhtp.ERR_WORKSPACE
    assert L.fhtp_polyline_dp(i32, 64, 64, 4, b, None, 0, i32, i32, None) == fhtp.ERR_NULL
    assert L.fhtp_polyline_dp(i32, 64, 64, 4, b, dummy, 1, i32, i32, None) == fhtp.ERR_WORKSPACE
    need = fhtp.dp_workspace_bytes(64, 64, 4, b)
    assert L.fhtp_polyline_dp(i32, 64, 64, 4, b, C.c_void_p(256 + 8), need, i32, i32,
                              None) == fhtp.ERR_WORKSPACE  # misaligned
    assert L.fhtp_polyline_dp(i32, 64, 64, 4, fhtp.Bend(0, -2, 0.0), dummy, need, i32, i32,
                              None) == fhtp.ERR_BEND
    assert L.fhtp_detect_polyline(dummy, 0, 64, 64, 4, b, dummy, 1, i32, None,
                                  None) == fhtp.ERR_NULL
    assert L.fhtp_detect_polyline(dummy, 1, 65536, 4, 65536, b, dummy, 1, i32, i32,
                                  None) == fhtp.ERR_OVERFLOW


def _job(h, w, k, dtype=0, bend=None, img=256, score=256, xs=256):
    return fhtp.Job(img, dtype, h, w, k, bend if bend is not None else fhtp.make_bend(1),
                    score, xs)


def test_batch_workspace_is_sum_of_single_workspaces():
    jobs = [_job(64, 64, 4), _job(1024, 300, 4), _job(256, 100, 8, dtype=1, bend=fhtp.Bend(1, 0, 0.2))]
    total = fhtp.batch_workspace_bytes(jobs)
    singles = [fhtp.detect_workspace_bytes(j.dtype, j.h, j.w, j.k, j.bend) for j in jobs]
    assert total >= sum(singles)
    assert total <= sum(singles) + 256 * len(jobs)
    assert fhtp.batch_workspace_bytes([]) == 0


def test_batch_rejects_any_invalid_job_before_launch():
    L = fhtp.lib()
    good = _job(64, 64, 4)
    for bad, code in [(_job(12, 8, 4), fhtp.ERR_DIMS), (_job(64, 64, 4, dtype=3), fhtp.ERR_DTYPE),
                      (_job(64, 64, 4, bend=fhtp.Bend(0, -1, 0.0)), fhtp.ERR_BEND),
                      (_job(64, 64, 4, img=None), fhtp.ERR_NULL),
                      (_job(65536, 4, 65536, dtype=1), fhtp.ERR_OVERFLOW)]:
        arr = (fhtp.Job * 2)(good, bad)
        out = C.c_size_t()
        assert L.fhtp_batch_workspace_bytes(arr, 2, C.byref(out)) == code
        # nothing is launched: the dummy pointers are never touched
        assert L.fhtp_detect_batch(arr, 2, C.c_void_p(256), 1 << 40, None) == code
    arr = (fhtp.Job * 1)(good)
    assert L.fhtp_detect_batch(arr, 1, C.c_void_p(256), 16, None) == fhtp.ERR_WORKSPACE
    assert L.fhtp_detect_batch(arr, 1, None, 1 << 30, None) == fhtp.ERR_NULL


def test_plan_create_validates_like_batch():
    """fhtp_plan_create rejects what fhtp_detect_batch rejects, before any HIP call."""
    L = fhtp.lib()
    good = _job(64, 64, 4)
    h = C.c_void_p()
    for bad, code in [(_job(12, 8, 4), fhtp.ERR_DIMS), (_job(64, 64, 4, dtype=3), fhtp.ERR_DTYPE),
                      (_job(64, 64, 4, bend=fhtp.Bend(0, -1, 0.0)), fhtp.ERR_BEND),
                      (_job(64, 64, 4, img=None), fhtp.ERR_NULL)]:
        arr = (fhtp.Job * 2)(good, bad)
        assert L.fhtp_plan_create(arr, 2, C.c_void_p(256), 1 << 40, C.byref(h)) == code
        assert h.value is None
    arr = (fhtp.Job * 1)(good)
    assert L.fhtp_plan_create(arr, 1, C.c_void_p(256), 16, C.byref(h)) == fhtp.ERR_WORKSPACE
    assert L.fhtp_plan_create(arr, 1, None, 1 << 30, C.byref(h)) == fhtp.ERR_NULL
    assert L.fhtp_plan_create(arr, 1, C.c_void_p(256), 1 << 30, None) == fhtp.ERR_NULL
    assert h.value is None
    # a null plan: nothing to capture or launch, destroying it is a no-op
    assert L.fhtp_plan_capture(None) == fhtp.ERR_NULL
    assert L.fhtp_plan_launch(None, None) == fhtp.ERR_NULL
    assert L.fhtp_plan_destroy(None) == 0


def test_detect_ex_validation_matches_oracle(orc):
    """Option and point errors agree with the oracle's, and nothing is launched."""
    L = fhtp.lib()
    b = fhtp.make_bend(1)
    dummy = C.c_void_p(256)
    img = np.zeros((16, 32), np.uint8)
    cases = [
        (dict(smooth_radius=8), fhtp.ERR_OPTION),
        (dict(smooth_radius=-1), fhtp.ERR_OPTION),
        (dict(pin=(5, 0)), fhtp.ERR_POINT),
        (dict(pin=(1, 32)), fhtp.ERR_POINT),
        (dict(pin=(1, -1)), fhtp.ERR_POINT),
        (dict(horizontal=True, pin=(2, 16)), fhtp.ERR_POINT),
    ]
    for kw, code in cases:
        with pytest.raises(oracle.OracleError) as e:
            orc.detect_ex(img, 4, bend=1, **kw)
        assert e.value.code == code, kw
        opt = fhtp.make_options(**kw)
        out = C.c_size_t()
        assert L.fhtp_detect_ex_workspace_bytes(0, 16, 32, 4, b, C.byref(opt), C.byref(out)) == code
        assert L.fhtp_detect_polyline_ex(dummy, 0, 16, 32, 4, b, C.byref(opt), dummy, 1 << 40,
                                         dummy, dummy, None) == code
    bad = fhtp.Options(0, 2, -1, 0)
    out = C.c_size_t()
    assert L.fhtp_detect_ex_workspace_bytes(0, 16, 32, 4, b, C.byref(bad), C.byref(out)) == \
        fhtp.ERR_OPTION
    # horizontal: k must split the 32 columns into power-of-two strips
    opt = fhtp.make_options(horizontal=True)
    assert L.fhtp_detect_ex_workspace_bytes(0, 16, 32, 3, b, C.byref(opt), C.byref(out)) == \
        fhtp.ERR_DIMS
    assert L.fhtp_detect_ex_workspace_bytes(0, 16, 32, 4, b, C.byref(opt), C.byref(out)) == 0
    # the overflow bound applies to the rows of the detection image
    assert L.fhtp_detect_ex_workspace_bytes(1, 4, 65536, 65536, b, C.byref(opt),
                                            C.byref(out)) == fhtp.ERR_OVERFLOW
    assert L.fhtp_detect_polyline_ex(None, 0, 16, 32, 4, b, None, dummy, 1 << 40, dummy, dummy,
                                     None) == fhtp.ERR_NULL
    assert L.fhtp_detect_polyline_ex(dummy, 0, 16, 32, 4, b, C.byref(opt), dummy, 1, dummy,
                                     dummy, None) == fhtp.ERR_WORKSPACE


def test_detect_ex_workspace_sizes():
    b = fhtp.make_bend(2)
    plain = fhtp.detect_workspace_bytes(0, 256, 300, 4, b)
    assert fhtp.detect_ex_workspace_bytes(0, 256, 300, 4, b, None) == plain
    assert fhtp.detect_ex_workspace_bytes(0, 256, 300, 4, b, fhtp.make_options(pin=(2, 7))) == plain
    sm = fhtp.detect_ex_workspace_bytes(0, 256, 300, 4, b, fhtp.make_options(smooth_radius=2))
    assert sm == plain + (256 * 300 + 255) // 256 * 256
    hz = fhtp.detect_ex_workspace_bytes(1, 300, 256, 4, b, fhtp.make_options(horizontal=True))
    assert hz == fhtp.detect_workspace_bytes(1, 256, 300, 4, b) + (2 * 256 * 300 + 255) // 256 * 256


def test_timing_hook_is_host_only_when_nothing_ran():
    from paper_1912_01884_amd import fhtp
    fhtp.timing_start()
    assert fhtp.timing_stop() == {}
    L = fhtp.lib()
    assert L.fhtp_timing_stop(None, 4, None) == fhtp.ERR_NULL


def test_noalloc_validates_before_launch():
    """Host-side refusals of the allocation-free entry point (nothing reaches the GPU)."""
    import ctypes as C
    from paper_1912_01884_amd import fhtp
    L = fhtp.lib()
    b = fhtp.make_bend(8)
    p = C.c_void_p(256)  # never dereferenced: every call below is refused on the host
    assert fhtp.noalloc_scratch_bytes() == 64 << 20
    assert L.fhtp_detect_polyline_noalloc(None, 0, 64, 64, 4, b, p, p, None) == fhtp.ERR_NULL
    assert L.fhtp_detect_polyline_noalloc(p, 0, 64, 64, 3, b, p, p, None) == fhtp.ERR_DIMS
    assert L.fhtp_detect_polyline_noalloc(p, 5, 64, 64, 4, b, p, p, None) == fhtp.ERR_DTYPE
    assert L.fhtp_detect_polyline_noalloc(p, 0, 64, 64, 4, fhtp.Bend(0, -1, 0.0), p, p,
                                          None) == fhtp.ERR_BEND
    # larger than the built-in array
    assert L.fhtp_detect_polyline_noalloc(p, 1, 4096, 4096, 32, b, p, p, None) == \
        fhtp.ERR_WORKSPACE

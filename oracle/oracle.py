"""ctypes binding of ``liboracle_fhtp.so`` (test infrastructure only).

Every function takes numpy arrays on the host and returns numpy results.  The
arithmetic lives in ``fhtp_oracle.c``; this file only marshals arguments.
``Oracle(path)`` binds any build of that source (the tests also load
deliberately broken builds to check that the pins catch them); the
module-level functions use the default build.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_fhtp.so")

ERR_NULL = -1
ERR_DIMS = -2
ERR_BEND = -3
ERR_OVERFLOW = -4
ERR_UNSUPPORTED = -7
ERR_DTYPE = -8
ERR_POINT = -9
ERR_OPTION = -10


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(rc, what)


def _dtype_code(img: np.ndarray) -> int:
    if img.dtype == np.uint8:
        return 0
    if img.dtype == np.uint16:
        return 1
    raise TypeError(f"image dtype must be uint8 or uint16, got {img.dtype}")


def _bend_args(bend=None, gamma=None):
    if gamma is not None:
        return 1, 0, float(gamma)
    return 0, int(bend), 0.0


class Oracle:
    """One loaded build of the oracle library."""

    def __init__(self, path: str = LIB_PATH):
        L = C.CDLL(path)
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        L.oracle_num_threads.restype = C.c_int
        L.oracle_dyadic_offset.argtypes = [C.c_int, C.c_int, C.c_int]
        L.oracle_dyadic_offset.restype = C.c_int
        L.oracle_dyadic_pattern.argtypes = [C.c_int, C.c_int, i32p]
        L.oracle_table_shape.argtypes = [C.c_int, C.c_int, C.c_int, i64p, i64p, i64p]
        L.oracle_fht_bands.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, i32p]
        L.oracle_polyline_dp.argtypes = [i32p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_double, i32p, i32p]
        L.oracle_detect_polyline.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                             C.c_int, C.c_int, C.c_double, i32p, i32p]
        L.oracle_detect_from_top.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                             C.c_int, C.c_int, C.c_double, C.c_int, i32p, i32p]
        L.oracle_angle_window.argtypes = [C.c_int, C.c_double, i32p, i32p]
        L.oracle_detect_through_point.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                                  C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                                  i32p, i32p]
        L.oracle_smooth_rows.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_void_p]
        L.oracle_detect_ex.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                       i32p, i32p]
        for f in (L.oracle_dyadic_pattern, L.oracle_table_shape, L.oracle_fht_bands,
                  L.oracle_polyline_dp, L.oracle_detect_polyline, L.oracle_detect_from_top,
                  L.oracle_angle_window, L.oracle_detect_through_point, L.oracle_smooth_rows,
                  L.oracle_detect_ex):
            f.restype = C.c_int
        self.L = L
        self.path = path

    def num_threads(self) -> int:
        return int(self.L.oracle_num_threads())

    def dyadic_pattern(self, n: int, s: int) -> np.ndarray:
        out = np.zeros(max(n, 1), dtype=np.int32)
        _check(self.L.oracle_dyadic_pattern(n, s, _i32p(out)), "dyadic_pattern")
        return out

    def table_shape(self, h: int, w: int, k: int) -> Tuple[int, int, int]:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(self.L.oracle_table_shape(h, w, k, C.byref(a), C.byref(b), C.byref(c)),
               "table_shape")
        return a.value, b.value, c.value

    def fht_bands(self, img: np.ndarray, k: int) -> np.ndarray:
        """Band tables [k][2n-1][w+n] int32 by direct summation along every dyadic line."""
        img = np.ascontiguousarray(img)
        h, w = img.shape
        n = h // k if k > 0 and h % k == 0 else 1
        out = np.zeros((max(k, 1), 2 * n - 1, w + n), dtype=np.int32)
        rc = self.L.oracle_fht_bands(img.ctypes.data, _dtype_code(img), h, w, k, _i32p(out))
        _check(rc, "fht_bands")
        return out

    def polyline_dp(self, tables: np.ndarray, h: int, w: int, k: int, bend: int = None,
                    gamma: float = None) -> Tuple[int, np.ndarray]:
        tables = np.ascontiguousarray(tables, dtype=np.int32)
        mode, b, g = _bend_args(bend, gamma)
        score = np.zeros(1, dtype=np.int32)
        xs = np.zeros(k + 1, dtype=np.int32)
        rc = self.L.oracle_polyline_dp(_i32p(tables), h, w, k, mode, b, g, _i32p(score),
                                       _i32p(xs))
        _check(rc, "polyline_dp")
        return int(score[0]), xs

    def detect_polyline(self, img: np.ndarray, k: int, bend: int = None,
                        gamma: float = None) -> Tuple[int, np.ndarray]:
        img = np.ascontiguousarray(img)
        h, w = img.shape
        mode, b, g = _bend_args(bend, gamma)
        score = np.zeros(1, dtype=np.int32)
        xs = np.zeros(max(k, 0) + 1, dtype=np.int32)
        rc = self.L.oracle_detect_polyline(img.ctypes.data, _dtype_code(img), h, w, k, mode, b,
                                           g, _i32p(score), _i32p(xs))
        _check(rc, "detect_polyline")
        return int(score[0]), xs

    def detect_from_top(self, img: np.ndarray, k: int, x0: int, bend: int = None,
                        gamma: float = None) -> Tuple[int, np.ndarray]:
        img = np.ascontiguousarray(img)
        h, w = img.shape
        mode, b, g = _bend_args(bend, gamma)
        score = np.zeros(1, dtype=np.int32)
        xs = np.zeros(k + 1, dtype=np.int32)
        rc = self.L.oracle_detect_from_top(img.ctypes.data, _dtype_code(img), h, w, k, mode, b,
                                           g, int(x0), _i32p(score), _i32p(xs))
        _check(rc, "detect_from_top")
        return int(score[0]), xs

    def detect_through_point(self, img: np.ndarray, k: int, pin_j: int, pin_x: int,
                             bend: int = None, gamma: float = None) -> Tuple[int, np.ndarray]:
        img = np.ascontiguousarray(img)
        h, w = img.shape
        mode, b, g = _bend_args(bend, gamma)
        score = np.zeros(1, dtype=np.int32)
        xs = np.zeros(k + 1, dtype=np.int32)
        rc = self.L.oracle_detect_through_point(img.ctypes.data, _dtype_code(img), h, w, k, mode,
                                                b, g, int(pin_j), int(pin_x), _i32p(score),
                                                _i32p(xs))
        _check(rc, "detect_through_point")
        return int(score[0]), xs

    def smooth_rows(self, img: np.ndarray, radius: int) -> np.ndarray:
        img = np.ascontiguousarray(img)
        h, w = img.shape
        out = np.zeros_like(img)
        rc = self.L.oracle_smooth_rows(img.ctypes.data, _dtype_code(img), h, w, int(radius),
                                       out.ctypes.data)
        _check(rc, "smooth_rows")
        return out

    def detect_ex(self, img: np.ndarray, k: int, bend: int = None, gamma: float = None,
                  smooth_radius: int = 0, horizontal: bool = False, pin=None
                  ) -> Tuple[int, np.ndarray]:
        """Detector with its options; pin = (boundary j, column) or None."""
        img = np.ascontiguousarray(img)
        h, w = img.shape
        mode, b, g = _bend_args(bend, gamma)
        pj, px = (-1, -1) if pin is None else (int(pin[0]), int(pin[1]))
        score = np.zeros(1, dtype=np.int32)
        xs = np.zeros(max(k, 0) + 1, dtype=np.int32)
        rc = self.L.oracle_detect_ex(img.ctypes.data, _dtype_code(img), h, w, k, mode, b, g,
                                     int(smooth_radius), int(bool(horizontal)), pj, px,
                                     _i32p(score), _i32p(xs))
        _check(rc, "detect_ex")
        return int(score[0]), xs

    def angle_window(self, n: int, gamma: float) -> Tuple[np.ndarray, np.ndarray]:
        lo = np.zeros(2 * n - 1, dtype=np.int32)
        hi = np.zeros(2 * n - 1, dtype=np.int32)
        _check(self.L.oracle_angle_window(n, float(gamma), _i32p(lo), _i32p(hi)),
               "angle_window")
        return lo, hi


_default = None


def lib() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _default = Oracle(LIB_PATH)
    return _default


def num_threads() -> int:
    return lib().num_threads()


def dyadic_pattern(n, s):
    return lib().dyadic_pattern(n, s)


def table_shape(h, w, k):
    return lib().table_shape(h, w, k)


def fht_bands(img, k):
    return lib().fht_bands(img, k)


def polyline_dp(tables, h, w, k, bend=None, gamma=None):
    return lib().polyline_dp(tables, h, w, k, bend=bend, gamma=gamma)


def detect_polyline(img, k, bend=None, gamma=None):
    return lib().detect_polyline(img, k, bend=bend, gamma=gamma)


def detect_from_top(img, k, x0, bend=None, gamma=None):
    return lib().detect_from_top(img, k, x0, bend=bend, gamma=gamma)


def angle_window(n, gamma):
    return lib().angle_window(n, gamma)


def detect_through_point(img, k, pin_j, pin_x, bend=None, gamma=None):
    return lib().detect_through_point(img, k, pin_j, pin_x, bend=bend, gamma=gamma)


def smooth_rows(img, radius):
    return lib().smooth_rows(img, radius)


def detect_ex(img, k, bend=None, gamma=None, smooth_radius=0, horizontal=False, pin=None):
    return lib().detect_ex(img, k, bend=bend, gamma=gamma, smooth_radius=smooth_radius,
                           horizontal=horizontal, pin=pin)

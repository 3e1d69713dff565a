"""Thin ctypes binding of libfhtp.so, with torch tensors as device buffers.

Argument marshalling only: every step of the detector runs in the HIP kernels
behind the C ABI (include/fhtp.h).  torch provides device memory and the
stream; the library itself never allocates.  If libfhtp.so has not been built
this module raises on first use -- there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfhtp.so")

FHTP_U8 = 0
FHTP_U16 = 1

OK = 0
ERR_NULL = -1
ERR_DIMS = -2
ERR_BEND = -3
ERR_OVERFLOW = -4
ERR_WORKSPACE = -5
ERR_HIP = -6
ERR_UNSUPPORTED = -7
ERR_DTYPE = -8
ERR_POINT = -9
ERR_OPTION = -10

EXPORTED = (
    "fhtp_strerror", "fhtp_last_error_detail", "fhtp_version", "fhtp_table_shape",
    "fhtp_fht_workspace_bytes", "fhtp_fht_bands", "fhtp_dp_workspace_bytes", "fhtp_polyline_dp",
    "fhtp_detect_workspace_bytes", "fhtp_detect_polyline", "fhtp_batch_workspace_bytes",
    "fhtp_detect_batch", "fhtp_detect_ex_workspace_bytes", "fhtp_detect_polyline_ex",
    "fhtp_prepare_image", "fhtp_plan_create", "fhtp_plan_capture", "fhtp_plan_launch",
    "fhtp_plan_destroy", "fhtp_timing_start", "fhtp_timing_stop", "fhtp_noalloc_scratch_bytes",
    "fhtp_detect_polyline_noalloc", "fhtp_tune_set", "fhtp_tune_get",
)


class FhtpError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        msg = f"{what} failed: {strerror(code)} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.code = code


class Bend(C.Structure):
    """fhtp_bend: mode 0 = |d_{i+1}-d_i| <= shift_bound, mode 1 = bend angle <= gamma_rad."""

    _fields_ = [("mode", C.c_int32), ("shift_bound", C.c_int32), ("gamma_rad", C.c_double)]


class Job(C.Structure):
    """fhtp_job: one detection of a batch (device pointers inside a host descriptor)."""

    _fields_ = [("img", C.c_void_p), ("dtype", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
                ("k", C.c_int32), ("bend", Bend), ("score", C.c_void_p), ("xs", C.c_void_p)]


class TuneRule(C.Structure):
    """fhtp_tune_rule: launch shapes for the requests a rule covers (see fhtp.h)."""

    _fields_ = [("dtype", C.c_int32), ("log2n", C.c_int32), ("w_min", C.c_int32),
                ("w_max", C.c_int32), ("window", C.c_int32), ("dc", C.c_int32),
                ("steps", C.c_int32), ("stripe", C.c_int32), ("fht_grid", C.c_int32),
                ("small", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class KernelTime(C.Structure):
    """fhtp_kernel_time: one kernel family's launches and summed bracket time."""

    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int32), ("total_ms", C.c_double)]


class Options(C.Structure):
    """fhtp_options: smoothing radius, orientation and the through-point pin."""

    _fields_ = [("smooth_radius", C.c_int32), ("horizontal", C.c_int32),
                ("pin_boundary", C.c_int32), ("pin_pos", C.c_int32)]


def make_options(smooth_radius: int = 0, horizontal: bool = False, pin=None) -> Options:
    """pin = (band boundary j, column or row) or None."""
    pj, pp = (-1, 0) if pin is None else (int(pin[0]), int(pin[1]))
    return Options(int(smooth_radius), int(bool(horizontal)), pj, pp)


def make_bend(bend: Optional[int] = None, gamma: Optional[float] = None) -> Bend:
    if gamma is not None:
        return Bend(1, 0, float(gamma))
    if bend is None:
        raise ValueError("give either a shift bound (bend=) or an angle bound (gamma=)")
    return Bend(0, int(bend), 0.0)


_lib = None


def lib() -> C.CDLL:
    """Load libfhtp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1912_01884_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, sz, i32, i64p = C.c_void_p, C.c_size_t, C.c_int, C.POINTER(C.c_int64)
    szp = C.POINTER(C.c_size_t)
    L.fhtp_strerror.argtypes = [i32]
    L.fhtp_strerror.restype = C.c_char_p
    L.fhtp_last_error_detail.restype = C.c_char_p
    L.fhtp_version.restype = C.c_char_p
    L.fhtp_table_shape.argtypes = [i32, i32, i32, i64p, i64p, i64p]
    L.fhtp_fht_workspace_bytes.argtypes = [i32, i32, i32, i32, szp]
    L.fhtp_fht_bands.argtypes = [vp, i32, i32, i32, i32, vp, vp, sz, vp]
    L.fhtp_dp_workspace_bytes.argtypes = [i32, i32, i32, Bend, szp]
    L.fhtp_polyline_dp.argtypes = [vp, i32, i32, i32, Bend, vp, sz, vp, vp, vp]
    L.fhtp_detect_workspace_bytes.argtypes = [i32, i32, i32, i32, Bend, szp]
    L.fhtp_detect_polyline.argtypes = [vp, i32, i32, i32, i32, Bend, vp, sz, vp, vp, vp]
    L.fhtp_batch_workspace_bytes.argtypes = [C.POINTER(Job), i32, szp]
    L.fhtp_detect_batch.argtypes = [C.POINTER(Job), i32, vp, sz, vp]
    optp = C.POINTER(Options)
    L.fhtp_detect_ex_workspace_bytes.argtypes = [i32, i32, i32, i32, Bend, optp, szp]
    L.fhtp_detect_polyline_ex.argtypes = [vp, i32, i32, i32, i32, Bend, optp, vp, sz, vp, vp, vp]
    L.fhtp_prepare_image.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
    L.fhtp_plan_create.argtypes = [C.POINTER(Job), i32, vp, sz, C.POINTER(vp)]
    L.fhtp_plan_capture.argtypes = [vp]
    L.fhtp_plan_launch.argtypes = [vp, vp]
    L.fhtp_plan_destroy.argtypes = [vp]
    L.fhtp_timing_start.argtypes = []
    L.fhtp_tune_set.argtypes = [C.POINTER(TuneRule), i32]
    L.fhtp_tune_get.argtypes = [C.POINTER(TuneRule), i32, C.POINTER(C.c_int)]
    L.fhtp_noalloc_scratch_bytes.argtypes = []
    L.fhtp_detect_polyline_noalloc.argtypes = [vp, i32, i32, i32, i32, Bend, vp, vp, vp]
    L.fhtp_timing_stop.argtypes = [C.POINTER(KernelTime), i32, C.POINTER(C.c_int)]
    for name in EXPORTED:
        if name not in ("fhtp_strerror", "fhtp_last_error_detail", "fhtp_version"):
            getattr(L, name).restype = C.c_int
    L.fhtp_noalloc_scratch_bytes.restype = C.c_size_t
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().fhtp_strerror(int(code)).decode()


def version() -> str:
    return lib().fhtp_version().decode()


def _check(rc: int, what: str):
    if rc != OK:
        detail = lib().fhtp_last_error_detail().decode() if rc == ERR_HIP else ""
        raise FhtpError(rc, what, detail)


# ---- pure host queries ------------------------------------------------------

def table_shape(h: int, w: int, k: int) -> Tuple[int, int, int]:
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().fhtp_table_shape(h, w, k, C.byref(a), C.byref(b), C.byref(c)), "table_shape")
    return a.value, b.value, c.value


def fht_workspace_bytes(dtype: int, h: int, w: int, k: int) -> int:
    out = C.c_size_t()
    _check(lib().fhtp_fht_workspace_bytes(dtype, h, w, k, C.byref(out)), "fht_workspace_bytes")
    return out.value


def dp_workspace_bytes(h: int, w: int, k: int, bend: Bend) -> int:
    out = C.c_size_t()
    _check(lib().fhtp_dp_workspace_bytes(h, w, k, bend, C.byref(out)), "dp_workspace_bytes")
    return out.value


def detect_workspace_bytes(dtype: int, h: int, w: int, k: int, bend: Bend) -> int:
    out = C.c_size_t()
    _check(lib().fhtp_detect_workspace_bytes(dtype, h, w, k, bend, C.byref(out)),
           "detect_workspace_bytes")
    return out.value


def detect_ex_workspace_bytes(dtype: int, h: int, w: int, k: int, bend: Bend,
                              opt: Optional[Options]) -> int:
    out = C.c_size_t()
    _check(lib().fhtp_detect_ex_workspace_bytes(dtype, h, w, k, bend,
                                                None if opt is None else C.byref(opt),
                                                C.byref(out)),
           "detect_ex_workspace_bytes")
    return out.value


def tune_set(rules) -> None:
    """Install tuning rules (dicts with the fhtp_tune_rule fields, or TuneRule);
    an empty list clears them."""
    objs = [r if isinstance(r, TuneRule) else TuneRule(**r) for r in rules]
    arr = (TuneRule * max(1, len(objs)))(*objs)
    _check(lib().fhtp_tune_set(arr if objs else None, len(objs)), "tune_set")


def tune_get() -> list:
    """The installed tuning rules as dicts, in match order."""
    cnt = C.c_int()
    _check(lib().fhtp_tune_get(None, 0, C.byref(cnt)), "tune_get")
    arr = (TuneRule * max(1, cnt.value))()
    _check(lib().fhtp_tune_get(arr, cnt.value, C.byref(cnt)), "tune_get")
    return [arr[q].as_dict() for q in range(cnt.value)]


def timing_start() -> None:
    """Bracket every following library launch with events (benchmarks only)."""
    _check(lib().fhtp_timing_start(), "timing_start")


def timing_stop() -> dict:
    """Stop timing; {family: (launches, total_ms)} in order of first launch."""
    cap = 64
    arr = (KernelTime * cap)()
    cnt = C.c_int()
    _check(lib().fhtp_timing_stop(arr, cap, C.byref(cnt)), "timing_stop")
    return {arr[q].name.decode(): (int(arr[q].launches), float(arr[q].total_ms))
            for q in range(min(cnt.value, cap))}


# ---- torch marshalling ------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.uint8:
        return FHTP_U8
    if t.dtype == torch.uint16:
        return FHTP_U16
    raise TypeError(f"image must be uint8 or uint16, got {t.dtype}")


def _stream_ptr(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _on_stream(stream, allocates: bool = True):
    """Context in which temporaries are allocated: the launch stream.

    torch's caching allocator hands a freed block only to later allocations
    on the stream it was allocated on, so a workspace or output allocated here
    and dropped after the call cannot be reused while the kernels enqueued on
    `stream` still use it, whichever stream is current.  A call that allocates
    nothing (every buffer given) skips the switch, a few microseconds of host
    time per call.
    """
    import contextlib
    torch = _torch()
    if stream is None or not allocates:
        return contextlib.nullcontext()
    return torch.cuda.stream(stream)


def _require_device(t, name: str):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")


def _ws(nbytes, device, ws):
    """The workspace to pass: the caller's (the library checks its size), or a
    new one of nbytes() bytes (none when that is 0)."""
    torch = _torch()
    if ws is not None:
        return ws, ws.numel() * ws.element_size()
    n = nbytes()
    if n == 0:
        return None, 0
    return torch.empty(n, dtype=torch.uint8, device=device), n


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def fht_bands(img, k: int, tables=None, ws=None, stream=None):
    """Band tables [k][2n-1][w+n] int32 of a device image [h][w] (uint8 or uint16)."""
    torch = _torch()
    _require_device(img, "img")
    h, w = img.shape
    dt = _dtype_code(img)
    kk, D, W = table_shape(h, w, k)
    with _on_stream(stream, tables is None or ws is None):
        if tables is None:
            tables = torch.empty((kk, D, W), dtype=torch.int32, device=img.device)
        ws_t, ws_n = _ws(lambda: fht_workspace_bytes(dt, h, w, k), img.device, ws)
        rc = lib().fhtp_fht_bands(img.data_ptr(), dt, h, w, k, tables.data_ptr(), _ptr(ws_t),
                                  ws_n, _stream_ptr(stream))
    _check(rc, "fht_bands")
    return tables


def polyline_dp(tables, h: int, w: int, k: int, bend: Optional[int] = None,
                gamma: Optional[float] = None, ws=None, score=None, xs=None, stream=None):
    """Best score (1 int32) and vertices x_0..x_k (k+1 int32) as device tensors."""
    torch = _torch()
    _require_device(tables, "tables")
    b = make_bend(bend, gamma)
    with _on_stream(stream, score is None or xs is None or ws is None):
        if score is None:
            score = torch.empty(1, dtype=torch.int32, device=tables.device)
        if xs is None:
            xs = torch.empty(k + 1, dtype=torch.int32, device=tables.device)
        ws_t, ws_n = _ws(lambda: dp_workspace_bytes(h, w, k, b), tables.device, ws)
        rc = lib().fhtp_polyline_dp(tables.data_ptr(), h, w, k, b, _ptr(ws_t), ws_n,
                                    score.data_ptr(), xs.data_ptr(), _stream_ptr(stream))
    _check(rc, "polyline_dp")
    return score, xs


def detect_polyline(img, k: int, bend: Optional[int] = None, gamma: Optional[float] = None,
                    ws=None, score=None, xs=None, stream=None):
    """The whole detector on a device image: (score, xs) as device tensors."""
    torch = _torch()
    _require_device(img, "img")
    h, w = img.shape
    dt = _dtype_code(img)
    b = make_bend(bend, gamma)
    with _on_stream(stream, score is None or xs is None or ws is None):
        if score is None:
            score = torch.empty(1, dtype=torch.int32, device=img.device)
        if xs is None:
            xs = torch.empty(k + 1, dtype=torch.int32, device=img.device)
        ws_t, ws_n = _ws(lambda: detect_workspace_bytes(dt, h, w, k, b), img.device, ws)
        rc = lib().fhtp_detect_polyline(img.data_ptr(), dt, h, w, k, b, _ptr(ws_t), ws_n,
                                        score.data_ptr(), xs.data_ptr(), _stream_ptr(stream))
    _check(rc, "detect_polyline")
    return score, xs


def noalloc_scratch_bytes() -> int:
    """Size of the scratch array fhtp_detect_polyline_noalloc uses on each GPU."""
    return int(lib().fhtp_noalloc_scratch_bytes())


def detect_polyline_noalloc(img, k: int, bend: Optional[int] = None,
                            gamma: Optional[float] = None, score=None, xs=None, stream=None):
    """detect_polyline through the entry point that allocates no device memory."""
    torch = _torch()
    _require_device(img, "img")
    h, w = img.shape
    b = make_bend(bend, gamma)
    with _on_stream(stream):
        if score is None:
            score = torch.empty(1, dtype=torch.int32, device=img.device)
        if xs is None:
            xs = torch.empty(k + 1, dtype=torch.int32, device=img.device)
        rc = lib().fhtp_detect_polyline_noalloc(img.data_ptr(), _dtype_code(img), h, w, k, b,
                                                score.data_ptr(), xs.data_ptr(),
                                                _stream_ptr(stream))
    _check(rc, "detect_polyline_noalloc")
    return score, xs


def prepare_image(img, smooth_radius: int = 0, horizontal: bool = False, out=None, stream=None):
    """Detection image of a device image: transposed if horizontal, rows smoothed."""
    torch = _torch()
    _require_device(img, "img")
    h, w = img.shape
    shape = (w, h) if horizontal else (h, w)
    with _on_stream(stream):
        if out is None:
            out = torch.empty(shape, dtype=img.dtype, device=img.device)
        rc = lib().fhtp_prepare_image(img.data_ptr(), _dtype_code(img), h, w, int(smooth_radius),
                                      int(bool(horizontal)), out.data_ptr(), _stream_ptr(stream))
    _check(rc, "prepare_image")
    return out


def detect_polyline_ex(img, k: int, bend: Optional[int] = None, gamma: Optional[float] = None,
                       smooth_radius: int = 0, horizontal: bool = False, pin=None, ws=None,
                       score=None, xs=None, stream=None):
    """The detector with row smoothing, orientation and a through-point pin.

    pin = (band boundary j, position) or None; positions and the returned xs
    are rows instead of columns when horizontal.
    """
    torch = _torch()
    _require_device(img, "img")
    h, w = img.shape
    dt = _dtype_code(img)
    b = make_bend(bend, gamma)
    opt = make_options(smooth_radius, horizontal, pin)
    with _on_stream(stream):
        if score is None:
            score = torch.empty(1, dtype=torch.int32, device=img.device)
        if xs is None:
            xs = torch.empty(k + 1, dtype=torch.int32, device=img.device)
        ws_t, ws_n = _ws(lambda: detect_ex_workspace_bytes(dt, h, w, k, b, opt), img.device, ws)
        rc = lib().fhtp_detect_polyline_ex(img.data_ptr(), dt, h, w, k, b, C.byref(opt),
                                           _ptr(ws_t), ws_n, score.data_ptr(), xs.data_ptr(),
                                           _stream_ptr(stream))
    _check(rc, "detect_polyline_ex")
    return score, xs


def batch_workspace_bytes(jobs) -> int:
    arr = (Job * len(jobs))(*jobs)
    out = C.c_size_t()
    _check(lib().fhtp_batch_workspace_bytes(arr, len(jobs), C.byref(out)), "batch_workspace_bytes")
    return out.value


def make_jobs(images, ks, bends=None, gammas=None, scores=None, xss=None):
    """Job descriptors for device images; allocates score/xs tensors unless given."""
    torch = _torch()
    jobs, keep = [], []
    for q, img in enumerate(images):
        _require_device(img, "img")
        h, w = img.shape
        k = int(ks[q])
        g = None if gammas is None else gammas[q]
        b = make_bend(None if (bends is None or g is not None) else bends[q], g)
        sc = scores[q] if scores is not None else torch.empty(1, dtype=torch.int32,
                                                              device=img.device)
        x = xss[q] if xss is not None else torch.empty(k + 1, dtype=torch.int32, device=img.device)
        jobs.append(Job(img.data_ptr(), _dtype_code(img), h, w, k, b, sc.data_ptr(), x.data_ptr()))
        keep.append((sc, x))
    return jobs, keep


def detect_batch(images, ks, bends=None, gammas=None, ws=None, scores=None, xss=None,
                 stream=None):
    """Many detections in one call; returns [(score, xs)] device tensors per image."""
    torch = _torch()
    if len(images) == 0:
        return []
    with _on_stream(stream):
        jobs, keep = make_jobs(images, ks, bends, gammas, scores, xss)
        nbytes = batch_workspace_bytes(jobs)
        ws_t, ws_n = _ws(lambda: nbytes, images[0].device, ws)
        arr = (Job * len(jobs))(*jobs)
        rc = lib().fhtp_detect_batch(arr, len(jobs), _ptr(ws_t), ws_n, _stream_ptr(stream))
    _check(rc, "detect_batch")
    return keep


class Plan:
    """A fixed set of detections recorded once as a HIP graph and replayed.

    Wraps fhtp_plan_create / fhtp_plan_capture / fhtp_plan_launch /
    fhtp_plan_destroy.  The images, outputs and workspace are borrowed for the
    plan's lifetime (the plan keeps references to the tensors); refill the
    images in place between launches.  results[q] is the (score, xs) pair of
    image q, valid once the launch's stream has been synchronised.
    """

    def __init__(self, images, ks, bends=None, gammas=None, ws=None, scores=None, xss=None,
                 capture=True):
        if len(images) == 0:
            raise ValueError("a plan needs at least one image")
        jobs, keep = make_jobs(images, ks, bends, gammas, scores, xss)
        nbytes = batch_workspace_bytes(jobs)
        ws_t, ws_n = _ws(lambda: nbytes, images[0].device, ws)
        arr = (Job * len(jobs))(*jobs)
        h = C.c_void_p()
        _check(lib().fhtp_plan_create(arr, len(jobs), _ptr(ws_t), ws_n, C.byref(h)), "plan_create")
        self._h = h
        self._keep = (list(images), ws_t, keep)
        self.results = keep
        if capture:
            self.capture()

    def capture(self) -> None:
        _check(lib().fhtp_plan_capture(self._h), "plan_capture")

    def launch(self, stream=None) -> None:
        if self._h is None:
            raise RuntimeError("plan destroyed")
        _check(lib().fhtp_plan_launch(self._h, _stream_ptr(stream)), "plan_launch")

    def destroy(self) -> None:
        if self._h is not None:
            _check(lib().fhtp_plan_destroy(self._h), "plan_destroy")
            self._h = None

    def __del__(self):
        try:
            if self._h is not None and _lib is not None:
                _lib.fhtp_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass

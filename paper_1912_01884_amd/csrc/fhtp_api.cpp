// Host side of the C ABI declared in include/fhtp.h: validation, workspace
// layout, window planning and kernel dispatch.  Every check runs on the host
// before anything is enqueued, so a rejected call leaves the stream and the
// outputs untouched.
#include "fhtp.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fhtp_internal.h"

namespace {

thread_local std::string g_detail;

constexpr int kMaxN = 1024;
constexpr int kMaxW = 1 << 20;
constexpr int kMaxFixedB = 16;
constexpr size_t kAlign = 256;
// pi/2 rounded to double: at or above it every bend is admissible.
constexpr double kHalfPi = 1.57079632679489661923;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int shape(int h, int w, int k, fhtp::Geometry* g) {
    if (h <= 0 || w <= 0 || k <= 0) return FHTP_ERR_DIMS;
    if (h % k != 0) return FHTP_ERR_DIMS;
    const int n = h / k;
    if (!is_pow2(n) || n > kMaxN) return FHTP_ERR_DIMS;
    if (w > kMaxW) return FHTP_ERR_DIMS;
    int p = 0;
    while ((1 << p) < n) ++p;
    g->h = h;
    g->w = w;
    g->k = k;
    g->n = n;
    g->p = p;
    g->W = w + n;
    g->D = 2 * n - 1;
    g->pitch = (w + 63) / 64 * 64;
    return FHTP_OK;
}

// A polyline takes one pixel per row, so its score is at most h * maxval.
int pixels(fhtp_dtype dtype, int h) {
    if (dtype != FHTP_U8 && dtype != FHTP_U16) return FHTP_ERR_DTYPE;
    const long long maxval = dtype == FHTP_U8 ? 255 : 65535;
    if ((long long)h * maxval >= (1LL << 31)) return FHTP_ERR_OVERFLOW;
    return FHTP_OK;
}

// Displacements per thread of the fixed-window DP step: 8 gives twice the
// waves of 16 at the cost of more halo loads (from cache), which pays until
// the grid fills the chip twice over.
int dp_chunk(const fhtp::Geometry& g) {
    const long long threads16 = (long long)g.w * ((g.D + 15) / 16);
    return threads16 < 256LL * 4 * 64 * 2 ? 8 : 16;
}

// ---- tuning rules (fhtp_tune_set) ----------------------------------------------
//
// Launch-shape choices that never change a result: the first rule matching a
// request overrides the defaults below.  Held process-wide; consulted when a
// request is planned (plans keep what their capture saw).
constexpr int kMaxTuneRules = 1024;
std::mutex g_tune_mu;
std::vector<fhtp_tune_rule> g_tune;

bool rule_valid(const fhtp_tune_rule& r) {
    return r.dtype >= -1 && r.dtype <= 1 && r.log2n >= -1 && r.log2n <= 10 && r.w_min >= 0 &&
           r.w_min <= r.w_max && r.window >= -1 && r.window <= 1 &&
           (r.dc == 0 || r.dc == 8 || r.dc == 16) && (r.steps >= 0 && r.steps <= 3) &&
           r.stripe >= 0 && r.stripe <= 64 && (r.fht_grid == 0 || r.fht_grid == 1) &&
           (r.small == 0 || r.small == 1);
}

// Knobs for a planned request: dtype -1 when the pixel type is not part of
// the request (fhtp_polyline_dp), then only rules for any pixel type match.
void apply_tuning(const fhtp::Geometry& g, int dtype, fhtp::DpPlan* pl) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const int window = pl->kind == fhtp::WindowKind::Fixed ? 0 : 1;
    for (const fhtp_tune_rule& r : g_tune) {
        if (r.dtype != -1 && r.dtype != dtype) continue;
        if (r.log2n != -1 && r.log2n != g.p) continue;
        if (g.w < r.w_min || g.w > r.w_max) continue;
        if (r.window != -1 && r.window != window) continue;
        if (r.dc) pl->dc = r.dc;
        if (r.steps) pl->steps = r.steps;
        pl->stripe = r.stripe ? r.stripe : 16;
        pl->fht_grid = r.fht_grid;
        pl->small = r.small == 0;
        return;
    }
}

// The DP's window kind for a bend restriction (Section 2.3), before tuning.
int plan_window(const fhtp::Geometry& g, fhtp_bend b, fhtp::DpPlan* pl) {
    pl->a16 = g.D > 256;
    pl->dc = dp_chunk(g);
    pl->steps = 2;
    pl->stripe = 16;
    pl->fht_grid = 0;
    pl->small = true;
    pl->bound = 0;
    pl->tan_gamma = 0.0;
    if (b.mode == 0) {
        if (b.shift_bound < 0) return FHTP_ERR_BEND;
        pl->bound = b.shift_bound;
        if ((long long)b.shift_bound >= 2LL * g.n - 2)
            pl->kind = fhtp::WindowKind::Full;
        else if (b.shift_bound <= kMaxFixedB)
            pl->kind = fhtp::WindowKind::Fixed;
        else
            pl->kind = fhtp::WindowKind::Generic;
        return FHTP_OK;
    }
    if (b.mode == 1) {
        if (!std::isfinite(b.gamma_rad) || b.gamma_rad < 0.0) return FHTP_ERR_BEND;
        if (b.gamma_rad >= kHalfPi) {
            pl->kind = fhtp::WindowKind::Full;
        } else {
            pl->kind = fhtp::WindowKind::Angle;
            pl->tan_gamma = std::tan(b.gamma_rad);
        }
        return FHTP_OK;
    }
    return FHTP_ERR_BEND;
}

int plan(const fhtp::Geometry& g, fhtp_bend b, fhtp::DpPlan* pl, int dtype = -1) {
    const int rc = plan_window(g, b, pl);
    if (rc == FHTP_OK) apply_tuning(g, dtype, pl);
    return rc;
}

struct DpLayout {
    size_t v, a, key, succ, win, end;
};

DpLayout dp_layout(const fhtp::Geometry& g, const fhtp::DpPlan& pl, size_t base) {
    DpLayout L;
    L.v = base;  // two value planes used in turn
    L.a = align_up(L.v + 2 * fhtp::dp_plane_bytes(g));
    L.key = align_up(L.a + fhtp::dp_backptr_bytes(g, pl.a16));
    L.succ = align_up(L.key + fhtp::dp_key_count(g) * sizeof(unsigned long long));
    L.win = align_up(L.succ + fhtp::dp_key_count(g) * sizeof(int32_t));
    L.end = align_up(L.win + 2 * (size_t)g.D * sizeof(int32_t));
    return L;
}

// Workspace of a whole detection: the band tables (narrow ones when the
// pixels allow: bands 0 .. k-2 as uint16, then the last band as int32), the
// FHT's scratch for tall bands, then the DP's buffers.
struct DetectLayout {
    size_t tables, wide, scratch;
    int narrow;  // bands stored as uint16
    DpLayout dp;
};

DetectLayout detect_layout(const fhtp::Geometry& g, const fhtp::DpPlan& pl, fhtp_dtype dtype) {
    DetectLayout L;
    const size_t band = (size_t)g.D * (size_t)g.W;
    L.tables = 0;
    L.narrow = fhtp::narrow_tables_apply(g, (int)dtype) ? g.k - 1 : 0;
    L.wide = align_up(L.tables + (size_t)L.narrow * band * sizeof(uint16_t));
    L.scratch = align_up(L.wide + (size_t)(g.k - L.narrow) * band * sizeof(int32_t));
    L.dp = dp_layout(g, pl, align_up(L.scratch + fhtp::fht_scratch_bytes(g, (int)dtype)));
    return L;
}

fhtp::TableSet table_set(char* base, const DetectLayout& L) {
    fhtp::TableSet t;
    t.narrow = L.narrow;
    t.tab16 = L.narrow ? reinterpret_cast<uint16_t*>(base + L.tables) : nullptr;
    t.wide = reinterpret_cast<int32_t*>(base + L.wide);
    return t;
}

fhtp::TableSet wide_tables(const int32_t* tables) {
    fhtp::TableSet t;
    t.wide = const_cast<int32_t*>(tables);
    return t;
}

fhtp::DpBuffers dp_buffers(char* ws, const DpLayout& L) {
    fhtp::DpBuffers b;
    b.vplanes = reinterpret_cast<int32_t*>(ws + L.v);
    b.a = ws + L.a;
    b.key = reinterpret_cast<unsigned long long*>(ws + L.key);
    b.succ = reinterpret_cast<int32_t*>(ws + L.succ);
    b.win = reinterpret_cast<int32_t*>(ws + L.win);
    return b;
}

int check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return FHTP_OK;
    if (!ws) return FHTP_ERR_NULL;
    if (ws_bytes < need) return FHTP_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return FHTP_ERR_WORKSPACE;
    return FHTP_OK;
}

int hip_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return FHTP_OK;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    g_detail = buf;
    return FHTP_ERR_HIP;
}

}  // namespace

extern "C" {

const char* fhtp_strerror(int code) {
    switch (code) {
        case FHTP_OK: return "ok";
        case FHTP_ERR_NULL: return "null pointer";
        case FHTP_ERR_DIMS: return "invalid dimensions (need h,w,k > 0, k | h, n = h/k a power of two <= 1024, w <= 2^20)";
        case FHTP_ERR_BEND: return "invalid bend restriction";
        case FHTP_ERR_OVERFLOW: return "scores could overflow int32 (h * maxval >= 2^31)";
        case FHTP_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
        case FHTP_ERR_HIP: return "HIP runtime error";
        case FHTP_ERR_UNSUPPORTED: return "unsupported request";
        case FHTP_ERR_DTYPE: return "invalid pixel type";
        case FHTP_ERR_POINT: return "point outside the image or band grid";
        case FHTP_ERR_OPTION: return "option out of range";
        default: return "unknown error";
    }
}

const char* fhtp_last_error_detail(void) { return g_detail.c_str(); }

const char* fhtp_version(void) { return "fhtp 0.1.0 gfx950"; }

int fhtp_table_shape(int h, int w, int k, int64_t* bands, int64_t* shifts, int64_t* width) {
    if (!bands || !shifts || !width) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    int rc = shape(h, w, k, &g);
    if (rc != FHTP_OK) return rc;
    *bands = g.k;
    *shifts = g.D;
    *width = g.W;
    return FHTP_OK;
}

int fhtp_fht_workspace_bytes(fhtp_dtype dtype, int h, int w, int k, size_t* bytes) {
    if (!bytes) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = pixels(dtype, h);
    if (rc != FHTP_OK) return rc;
    *bytes = fhtp::fht_scratch_bytes(g, (int)dtype);
    return FHTP_OK;
}

int fhtp_fht_bands(const void* img, fhtp_dtype dtype, int h, int w, int k, int32_t* tables,
                   void* ws, size_t ws_bytes, void* stream) {
    if (!img || !tables) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = pixels(dtype, h);
    if (rc == FHTP_OK) rc = check_ws(ws, ws_bytes, fhtp::fht_scratch_bytes(g, (int)dtype));
    if (rc != FHTP_OK) return rc;
    (void)hipGetLastError();
    return hip_status(fhtp::launch_fht(img, (int)dtype, g, wide_tables(tables), ws,
                                       static_cast<hipStream_t>(stream)),
                      "fht_bands");
}

int fhtp_dp_workspace_bytes(int h, int w, int k, fhtp_bend bend, size_t* bytes) {
    if (!bytes) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = plan(g, bend, &pl);
    if (rc != FHTP_OK) return rc;
    *bytes = dp_layout(g, pl, 0).end;
    return FHTP_OK;
}

int fhtp_polyline_dp(const int32_t* tables, int h, int w, int k, fhtp_bend bend, void* ws,
                     size_t ws_bytes, int32_t* score, int32_t* xs, void* stream) {
    if (!tables || !score || !xs) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = plan(g, bend, &pl);
    if (rc != FHTP_OK) return rc;
    const DpLayout L = dp_layout(g, pl, 0);
    rc = check_ws(ws, ws_bytes, L.end);
    if (rc != FHTP_OK) return rc;
    (void)hipGetLastError();
    return hip_status(fhtp::launch_dp(wide_tables(tables), g, pl,
                                      dp_buffers(static_cast<char*>(ws), L), score, xs,
                                      static_cast<hipStream_t>(stream)),
                      "polyline_dp");
}

int fhtp_tune_set(const fhtp_tune_rule* rules, int count) {
    if (count < 0 || count > kMaxTuneRules) return FHTP_ERR_OPTION;
    if (count > 0 && !rules) return FHTP_ERR_NULL;
    for (int q = 0; q < count; ++q)
        if (!rule_valid(rules[q])) return FHTP_ERR_OPTION;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.assign(rules, rules + count);
    return FHTP_OK;
}

int fhtp_tune_get(fhtp_tune_rule* out, int cap, int* count) {
    if (!count || (cap > 0 && !out)) return FHTP_ERR_NULL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    *count = (int)g_tune.size();
    for (int q = 0; q < cap && q < (int)g_tune.size(); ++q) out[q] = g_tune[q];
    return FHTP_OK;
}

int fhtp_detect_workspace_bytes(fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend,
                                size_t* bytes) {
    if (!bytes) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = pixels(dtype, h);
    if (rc == FHTP_OK) rc = plan(g, bend, &pl, (int)dtype);
    if (rc != FHTP_OK) return rc;
    *bytes = detect_layout(g, pl, dtype).dp.end;
    return FHTP_OK;
}

int fhtp_detect_polyline(const void* img, fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend,
                         void* ws, size_t ws_bytes, int32_t* score, int32_t* xs, void* stream) {
    if (!img || !score || !xs) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = pixels(dtype, h);
    if (rc == FHTP_OK) rc = plan(g, bend, &pl, (int)dtype);
    if (rc != FHTP_OK) return rc;
    const DetectLayout L = detect_layout(g, pl, dtype);
    rc = check_ws(ws, ws_bytes, L.dp.end);
    if (rc != FHTP_OK) return rc;
    char* base = static_cast<char*>(ws);
    const fhtp::TableSet tables = table_set(base, L);
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (fhtp::small_apply(g, (int)dtype, pl, fhtp::Pin{}, true)) {
        const fhtp::SmallJobSpec j{img, (int)dtype, g, pl, score, xs};
        return hip_status(fhtp::launch_small_jobs(&j, 1, s), "detect_polyline/small");
    }
    rc = hip_status(fhtp::launch_fht(img, (int)dtype, g, tables, base + L.scratch, s, pl.fht_grid),
                    "detect_polyline/fht");
    if (rc != FHTP_OK) return rc;
    return hip_status(fhtp::launch_dp(tables, g, pl, dp_buffers(base, L.dp), score, xs, s),
                      "detect_polyline/dp");
}

namespace {

// ---- the allocation-free entry point -----------------------------------------
//
// Device scratch for fhtp_detect_polyline_noalloc: one array per GPU, part of
// the library's code object, held until the process ends.  Host code never
// uses its name as an address: the first call on a device takes the device
// address with hipGetSymbolAddress (that device current) and keeps it.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxScratchDevices = 64;

struct ScratchSlot {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};

ScratchSlot g_scratch[kMaxScratchDevices];

// Device address of the current device's scratch array.
int scratch_of_current_device(void** out) {
    int dev = 0;
    int rc = hip_status(hipGetDevice(&dev), "detect_polyline_noalloc/device");
    if (rc != FHTP_OK) return rc;
    if (dev < 0 || dev >= kMaxScratchDevices) return FHTP_ERR_UNSUPPORTED;
    ScratchSlot& slot = g_scratch[dev];
    std::call_once(slot.once, [&] {
        slot.err = hipGetSymbolAddress(&slot.ptr, HIP_SYMBOL(scratch));
        if (slot.err != hipSuccess) {
            (void)hipGetLastError();
            slot.ptr = nullptr;
        }
    });
    if (slot.err != hipSuccess || !slot.ptr)
        return hip_status(slot.err != hipSuccess ? slot.err : hipErrorInvalidSymbol,
                          "detect_polyline_noalloc/scratch address");
    *out = slot.ptr;
    return FHTP_OK;
}

constexpr int kMaxSmoothRadius = 7;

// Validated extended request: the detection image's geometry and where the
// prepared image (if any) sits in the workspace.
struct ExPlan {
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    fhtp::Pin pin;
    bool prep;          // transpose and/or smoothing writes a detection image
    size_t prep_bytes;  // its size, aligned
    DetectLayout L;     // offsets relative to the end of the prepared image
};

int plan_ex(fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend, const fhtp_options* opt,
            ExPlan* e) {
    fhtp_options o{0, 0, -1, 0};
    if (opt) o = *opt;
    if (o.horizontal != 0 && o.horizontal != 1) return FHTP_ERR_OPTION;
    if (o.smooth_radius < 0 || o.smooth_radius > kMaxSmoothRadius) return FHTP_ERR_OPTION;
    const int hh = o.horizontal ? w : h, ww = o.horizontal ? h : w;
    int rc = shape(hh, ww, k, &e->g);
    if (rc == FHTP_OK) rc = pixels(dtype, hh);
    if (rc == FHTP_OK) rc = plan(e->g, bend, &e->pl, (int)dtype);
    if (rc != FHTP_OK) return rc;
    if (o.pin_boundary < -1 || o.pin_boundary > k) return FHTP_ERR_POINT;
    if (o.pin_boundary >= 0 && (o.pin_pos < 0 || o.pin_pos >= ww)) return FHTP_ERR_POINT;
    e->pin.j = o.pin_boundary;
    e->pin.x = o.pin_boundary >= 0 ? o.pin_pos : 0;
    e->prep = o.horizontal || o.smooth_radius > 0;
    const size_t bpp = dtype == FHTP_U8 ? 1 : 2;
    e->prep_bytes = e->prep ? align_up((size_t)h * (size_t)w * bpp) : 0;
    e->L = detect_layout(e->g, e->pl, dtype);
    return FHTP_OK;
}

}  // namespace

int fhtp_prepare_image(const void* img, fhtp_dtype dtype, int h, int w, int smooth_radius,
                       int horizontal, void* out, void* stream) {
    if (!img || !out) return FHTP_ERR_NULL;
    if (dtype != FHTP_U8 && dtype != FHTP_U16) return FHTP_ERR_DTYPE;
    if (h <= 0 || w <= 0 || h > (1 << 24) || w > (1 << 24)) return FHTP_ERR_DIMS;
    if (horizontal != 0 && horizontal != 1) return FHTP_ERR_OPTION;
    if (smooth_radius < 0 || smooth_radius > kMaxSmoothRadius) return FHTP_ERR_OPTION;
    (void)hipGetLastError();
    return hip_status(fhtp::launch_prep(img, (int)dtype, h, w, smooth_radius, horizontal, out,
                                        static_cast<hipStream_t>(stream)),
                      "prepare_image");
}

size_t fhtp_noalloc_scratch_bytes(void) { return kNoAllocBytes; }

int fhtp_detect_polyline_noalloc(const void* img, fhtp_dtype dtype, int h, int w, int k,
                                 fhtp_bend bend, int32_t* score, int32_t* xs, void* stream) {
    if (!img || !score || !xs) return FHTP_ERR_NULL;
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    int rc = shape(h, w, k, &g);
    if (rc == FHTP_OK) rc = pixels(dtype, h);
    if (rc == FHTP_OK) rc = plan(g, bend, &pl, (int)dtype);
    if (rc != FHTP_OK) return rc;
    const DetectLayout L = detect_layout(g, pl, dtype);
    if (L.dp.end > kNoAllocBytes) return FHTP_ERR_WORKSPACE;
    void* ws = nullptr;
    rc = scratch_of_current_device(&ws);
    if (rc != FHTP_OK) return rc;
    char* base = static_cast<char*>(ws);
    const fhtp::TableSet tables = table_set(base, L);
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (fhtp::small_apply(g, (int)dtype, pl, fhtp::Pin{}, true)) {
        const fhtp::SmallJobSpec j{img, (int)dtype, g, pl, score, xs};
        return hip_status(fhtp::launch_small_jobs(&j, 1, s), "detect_polyline_noalloc/small");
    }
    rc = hip_status(fhtp::launch_fht(img, (int)dtype, g, tables, base + L.scratch, s, pl.fht_grid),
                    "detect_polyline_noalloc/fht");
    if (rc != FHTP_OK) return rc;
    return hip_status(fhtp::launch_dp(tables, g, pl, dp_buffers(base, L.dp), score, xs, s),
                      "detect_polyline_noalloc/dp");
}

int fhtp_detect_ex_workspace_bytes(fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend,
                                   const fhtp_options* opt, size_t* bytes) {
    if (!bytes) return FHTP_ERR_NULL;
    ExPlan e;
    const int rc = plan_ex(dtype, h, w, k, bend, opt, &e);
    if (rc != FHTP_OK) return rc;
    *bytes = e.prep_bytes + e.L.dp.end;
    return FHTP_OK;
}

int fhtp_detect_polyline_ex(const void* img, fhtp_dtype dtype, int h, int w, int k,
                            fhtp_bend bend, const fhtp_options* opt, void* ws, size_t ws_bytes,
                            int32_t* score, int32_t* xs, void* stream) {
    if (!img || !score || !xs) return FHTP_ERR_NULL;
    ExPlan e;
    int rc = plan_ex(dtype, h, w, k, bend, opt, &e);
    if (rc != FHTP_OK) return rc;
    rc = check_ws(ws, ws_bytes, e.prep_bytes + e.L.dp.end);
    if (rc != FHTP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    const void* det = img;
    (void)hipGetLastError();
    if (e.prep) {
        rc = hip_status(fhtp::launch_prep(img, (int)dtype, h, w, opt->smooth_radius,
                                          opt->horizontal, base, s),
                        "detect_polyline_ex/prep");
        if (rc != FHTP_OK) return rc;
        det = base;
        base += e.prep_bytes;
    }
    if (fhtp::small_apply(e.g, (int)dtype, e.pl, e.pin, true)) {
        const fhtp::SmallJobSpec j{det, (int)dtype, e.g, e.pl, score, xs};
        return hip_status(fhtp::launch_small_jobs(&j, 1, s), "detect_polyline_ex/small");
    }
    const fhtp::TableSet tables = table_set(base, e.L);
    rc = hip_status(fhtp::launch_fht(det, (int)dtype, e.g, tables, base + e.L.scratch, s,
                                     e.pl.fht_grid),
                    "detect_polyline_ex/fht");
    if (rc != FHTP_OK) return rc;
    return hip_status(fhtp::launch_dp(tables, e.g, e.pl, dp_buffers(base, e.L.dp), score, xs, s,
                                      e.pin),
                      "detect_polyline_ex/dp");
}

namespace {

// Validated job with its workspace share.
struct BatchEntry {
    fhtp::Geometry g;
    fhtp::DpPlan pl;
    DetectLayout L;
    size_t offset;
};

int plan_batch(const fhtp_job* jobs, int count, std::vector<BatchEntry>* out, size_t* total) {
    if (!jobs && count > 0) return FHTP_ERR_NULL;
    if (count < 0) return FHTP_ERR_DIMS;
    out->clear();
    out->reserve(count);
    size_t off = 0;
    for (int q = 0; q < count; ++q) {
        const fhtp_job& J = jobs[q];
        BatchEntry e;
        if (!J.img || !J.score || !J.xs) return FHTP_ERR_NULL;
        int rc = shape(J.h, J.w, J.k, &e.g);
        if (rc == FHTP_OK) rc = pixels((fhtp_dtype)J.dtype, J.h);
        if (rc == FHTP_OK) rc = plan(e.g, J.bend, &e.pl, J.dtype);
        if (rc != FHTP_OK) {
            char buf[64];
            std::snprintf(buf, sizeof(buf), "job %d", q);
            g_detail = buf;
            return rc;
        }
        e.L = detect_layout(e.g, e.pl, (fhtp_dtype)J.dtype);
        e.offset = off;
        off = align_up(off + e.L.dp.end);
        out->push_back(e);
    }
    *total = off;
    return FHTP_OK;
}

}  // namespace

int fhtp_batch_workspace_bytes(const fhtp_job* jobs, int count, size_t* bytes) {
    if (!bytes) return FHTP_ERR_NULL;
    std::vector<BatchEntry> plan_v;
    size_t total = 0;
    const int rc = plan_batch(jobs, count, &plan_v, &total);
    if (rc != FHTP_OK) return rc;
    *bytes = total;
    return FHTP_OK;
}

namespace {

// A second stream for batches: the images whose tall bands take the two-pass
// FHT and 16-bit back-pointers run their whole pipeline there, the others on
// the caller's stream, so the two chains of dependent DP steps (each bound by
// latency, not by the chip) overlap.  The caller's stream forks to it with an
// event and joins back with another, so graph capture sees a closed
// fork/join.  Eager calls get one second stream per caller stream (created on
// first use outside graph capture and kept until the process ends), so
// batches on different caller streams never share one; a plan owns its own,
// created before its capture opens.  Streams keep the default priority.
struct Aux {
    std::mutex mu;  // calls that share this Aux (ordered on one caller stream)
    bool ok = false;
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

bool aux_init(Aux* a) {
    a->ok = hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&a->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&a->join, hipEventDisableTiming) == hipSuccess;
    (void)hipGetLastError();
    return a->ok;
}

void aux_release(Aux* a) {
    if (a->fork) (void)hipEventDestroy(a->fork);
    if (a->join) (void)hipEventDestroy(a->join);
    if (a->stream) (void)hipStreamDestroy(a->stream);
    a->fork = a->join = nullptr;
    a->stream = nullptr;
    a->ok = false;
}

struct AuxKey {
    int device;
    hipStream_t caller;
    bool operator<(const AuxKey& o) const {
        return device != o.device ? device < o.device : caller < o.caller;
    }
};

std::mutex g_aux_mu;  // guards the map only, never held across launches
std::map<AuxKey, std::unique_ptr<Aux>> g_aux;

// The second stream of eager batches on caller stream s of the current
// device, or null (then the batch runs on s alone): under capture a missing
// one is not created.
Aux* aux_for_caller(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_aux_mu);
    auto it = g_aux.find(AuxKey{dev, s});
    if (it != g_aux.end()) return it->second->ok ? it->second.get() : nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::unique_ptr<Aux> a(new (std::nothrow) Aux);
    if (!a) return nullptr;
    aux_init(a.get());
    Aux* out = a->ok ? a.get() : nullptr;
    g_aux.emplace(AuxKey{dev, s}, std::move(a));
    return out;
}

// FHT then DP of a subset of a batch on one stream.
int run_subset(const std::vector<fhtp::FhtJobSpec>& fj, const std::vector<fhtp::DpJobSpec>& dj,
               const std::vector<int>& pick, hipStream_t s) {
    std::vector<fhtp::FhtJobSpec> f;
    std::vector<fhtp::DpJobSpec> d;
    for (int q : pick) {
        f.push_back(fj[q]);
        d.push_back(dj[q]);
    }
    int rc = hip_status(fhtp::launch_fht_jobs(f.data(), (int)f.size(), s), "detect_batch/fht");
    if (rc != FHTP_OK) return rc;
    return hip_status(fhtp::launch_dp_jobs(d.data(), (int)d.size(), s), "detect_batch/dp");
}

}  // namespace

namespace {

// fhtp_detect_batch with an explicit second stream (`ax`; null: look one up
// for the caller's stream).
int detect_batch_on(const fhtp_job* jobs, int count, void* ws, size_t ws_bytes, void* stream,
                    Aux* ax_given) {
    std::vector<BatchEntry> plan_v;
    size_t total = 0;
    int rc = plan_batch(jobs, count, &plan_v, &total);
    if (rc != FHTP_OK) return rc;
    if (count == 0) return FHTP_OK;
    rc = check_ws(ws, ws_bytes, total);
    if (rc != FHTP_OK) return rc;
    std::vector<fhtp::FhtJobSpec> fj(count);
    std::vector<fhtp::DpJobSpec> dj(count);
    for (int q = 0; q < count; ++q) {
        const BatchEntry& e = plan_v[q];
        char* base = static_cast<char*>(ws) + e.offset;
        const fhtp::TableSet tables = table_set(base, e.L);
        fj[q] = fhtp::FhtJobSpec{jobs[q].img, (int)jobs[q].dtype, e.g, tables, base + e.L.scratch,
                                 e.pl.fht_grid};
        dj[q] = fhtp::DpJobSpec{tables, e.g, e.pl, dp_buffers(base, e.L.dp), jobs[q].score,
                                jobs[q].xs};
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    // small images: one fused workgroup each, in their own launches
    std::vector<fhtp::SmallJobSpec> small;
    std::vector<int> tall, rest;
    for (int q = 0; q < count; ++q) {
        if (fhtp::small_apply(dj[q].g, fj[q].dtype, dj[q].plan, fhtp::Pin{}, false))
            small.push_back(fhtp::SmallJobSpec{fj[q].img, fj[q].dtype, dj[q].g, dj[q].plan,
                                               dj[q].score, dj[q].xs});
        else
            (dj[q].plan.a16 ? tall : rest).push_back(q);
    }
    if (!small.empty()) {
        rc = hip_status(fhtp::launch_small_jobs(small.data(), (int)small.size(), s),
                        "detect_batch/small");
        if (rc != FHTP_OK) return rc;
    }
    if (tall.empty() && rest.empty()) return FHTP_OK;
    Aux* ax = nullptr;
    if (!tall.empty() && !rest.empty()) ax = ax_given ? ax_given : aux_for_caller(s);
    if (ax && !ax->ok) ax = nullptr;
    if (!ax) {  // every remaining image on the caller's stream
        std::vector<int> all(tall);
        all.insert(all.end(), rest.begin(), rest.end());
        std::sort(all.begin(), all.end());
        return run_subset(fj, dj, all, s);
    }
    std::lock_guard<std::mutex> lock(ax->mu);
    rc = hip_status(hipEventRecord(ax->fork, s), "detect_batch/fork");
    if (rc == FHTP_OK) rc = hip_status(hipStreamWaitEvent(ax->stream, ax->fork, 0), "detect_batch/fork");
    if (rc != FHTP_OK) return rc;
    const int rc_tall = run_subset(fj, dj, tall, ax->stream);
    const int rc_rest = rc_tall == FHTP_OK ? run_subset(fj, dj, rest, s) : FHTP_OK;
    // join even after an error, so that a capture is never left forked
    int rc_join = hip_status(hipEventRecord(ax->join, ax->stream), "detect_batch/join");
    if (rc_join == FHTP_OK)
        rc_join = hip_status(hipStreamWaitEvent(s, ax->join, 0), "detect_batch/join");
    return rc_tall != FHTP_OK ? rc_tall : rc_rest != FHTP_OK ? rc_rest : rc_join;
}

}  // namespace

int fhtp_detect_batch(const fhtp_job* jobs, int count, void* ws, size_t ws_bytes, void* stream) {
    return detect_batch_on(jobs, count, ws, ws_bytes, stream, nullptr);
}

}  // extern "C"

// A plan: the jobs of one fhtp_detect_batch call, their workspace, and the
// graph that records the call.
struct fhtp_plan_s {
    std::vector<fhtp_job> jobs;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Aux aux;  // the plan's own second stream (created by the first capture)
};

namespace {

void release_graph(fhtp_plan_s* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// Runs f with the plan's device current, restoring the caller's device.
template <typename F>
int on_device(int device, const char* what, F&& f) {
    int prev = 0;
    int rc = hip_status(hipGetDevice(&prev), what);
    if (rc != FHTP_OK) return rc;
    if (prev != device) {
        rc = hip_status(hipSetDevice(device), what);
        if (rc != FHTP_OK) return rc;
    }
    rc = f();
    if (prev != device) (void)hipSetDevice(prev);
    return rc;
}

}  // namespace

extern "C" {

int fhtp_plan_create(const fhtp_job* jobs, int count, void* ws, size_t ws_bytes, fhtp_plan* out) {
    if (!out) return FHTP_ERR_NULL;
    std::vector<BatchEntry> plan_v;
    size_t total = 0;
    int rc = plan_batch(jobs, count, &plan_v, &total);
    if (rc != FHTP_OK) return rc;
    if (count > 0) {
        rc = check_ws(ws, ws_bytes, total);
        if (rc != FHTP_OK) return rc;
    }
    auto* p = new (std::nothrow) fhtp_plan_s;
    if (!p) return FHTP_ERR_HIP;
    p->jobs.assign(jobs, jobs + count);
    p->ws = ws;
    p->ws_bytes = ws_bytes;
    rc = hip_status(hipGetDevice(&p->device), "plan_create");
    if (rc != FHTP_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return FHTP_OK;
}

int fhtp_plan_capture(fhtp_plan p) {
    if (!p) return FHTP_ERR_NULL;
    return on_device(p->device, "plan_capture", [&]() -> int {
        release_graph(p);
        if (p->jobs.empty()) return FHTP_OK;  // nothing to record: launches enqueue nothing
        hipStream_t cs = nullptr;
        int rc = hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "plan_capture");
        if (rc != FHTP_OK) return rc;
        // the plan's second stream must exist before the capture opens
        if (!p->aux.ok) {
            aux_release(&p->aux);
            aux_init(&p->aux);
        }
        rc = hip_status(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "plan_capture");
        if (rc == FHTP_OK) {
            const int rc_run = detect_batch_on(p->jobs.data(), (int)p->jobs.size(), p->ws,
                                               p->ws_bytes, cs, p->aux.ok ? &p->aux : nullptr);
            hipGraph_t g = nullptr;
            const int rc_end = hip_status(hipStreamEndCapture(cs, &g), "plan_capture/end");
            rc = rc_run != FHTP_OK ? rc_run : rc_end;
            if (rc == FHTP_OK) {
                p->graph = g;
                rc = hip_status(hipGraphInstantiateWithFlags(&p->exec, g, 0), "plan_capture/instantiate");
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
            if (rc != FHTP_OK) release_graph(p);
        }
        (void)hipStreamDestroy(cs);
        return rc;
    });
}

int fhtp_plan_launch(fhtp_plan p, void* stream) {
    if (!p) return FHTP_ERR_NULL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!p->exec)
        return detect_batch_on(p->jobs.data(), (int)p->jobs.size(), p->ws, p->ws_bytes, s,
                               p->aux.ok ? &p->aux : nullptr);
    return hip_status(hipGraphLaunch(p->exec, s), "plan_launch");
}

int fhtp_plan_destroy(fhtp_plan p) {
    if (!p) return FHTP_OK;
    const int rc = on_device(p->device, "plan_destroy", [&]() -> int {
        release_graph(p);
        aux_release(&p->aux);
        return FHTP_OK;
    });
    delete p;
    return rc;
}

}  // extern "C"

/*
 * fhtp.h -- C ABI of libfhtp.so: end-to-end curves of limited curvature on MI355X.
 *
 * The library finds the k-link "mostly vertical uniform polyline" (paper:
 * "A Method of Detecting End-To-End Curves of Limited Curvature", Section 2,
 * definitions 1-5 and the main problem statement) whose summed pixel values
 * are largest, subject to a bound on the bend between adjacent links.  It
 * follows the paper's method: a Fast Hough Transform of every horizontal band
 * (Section 2.1), then a bottom-up dynamic programme over band boundaries with
 * a range maximum over admissible successors (Sections 2.2-2.3, eqs. (3)-(7)),
 * then the global choice and backtrace (eq. (5) and the main-problem steps 2-3).
 *
 * Geometry and notation (the paper leaves the discrete details open; these are
 * the readings the library implements):
 *   - the image is h rows by w columns, row-major, no padding (stride w);
 *   - k bands of n = h/k rows each; n must be a power of two, n <= 1024;
 *   - each band is extended to the right by n zero columns (Section 2.1), so
 *     band tables are W = w + n columns wide and cyclic over W;
 *   - a link over band i starts at column x on the band's first row and is
 *     displaced by d in [-(n-1), n-1] columns on its last row, following the
 *     dyadic digital line of the FHT (upper half with shift floor(s/2), lower
 *     half offset by ceil(s/2), mirrored for d < 0);
 *   - the paper's Hough coordinate of eq. (1) is shift = n - d; this ABI
 *     indexes table rows by r = d + n - 1 instead;
 *   - a polyline is (x_0; d_0 .. d_{k-1}) with x_{i+1} = x_i + d_i, every
 *     vertex x_0 .. x_k inside [0, w-1]; x_k is the column on the last row;
 *   - its score is the sum of one pixel per image row along it (Section 2.1);
 *   - bend mode 0: |d_{i+1} - d_i| <= shift_bound;
 *     bend mode 1: |atan(d_{i+1}/n) - atan(d_i/n)| <= gamma_rad, the angle
 *     form of eqs. (6)-(7), decided exactly as
 *     n*|d' - d| <= tan(gamma) * (n*n + d*d') in IEEE double (gamma >= pi/2
 *     admits every pair);
 *   - among polylines with the best score the lexicographically smallest
 *     (x_0, d_0, d_1, ..., d_{k-1}) is returned.
 *   All arithmetic is integer and exact; results are bit-identical to the
 *   CPU definition.
 *
 * Conventions for every entry point:
 *   - return FHTP_OK (0) or a negative FHTP_ERR_* code;
 *   - all arguments are validated on the host before anything is enqueued;
 *     on error nothing is enqueued and no output is touched;
 *   - compute calls are asynchronous on `stream` (a hipStream_t passed as
 *     void*, NULL = the default stream); outputs are valid once the stream
 *     has been synchronised;
 *   - every data pointer of a compute call is DEVICE memory owned by the
 *     caller; the library never allocates, frees or synchronises it;
 *   - `ws` is caller-owned device scratch of at least the size reported by
 *     the matching *_workspace_bytes query, aligned to 256 bytes; its
 *     contents on entry do not matter; two calls that share a workspace must
 *     be ordered on one stream;
 *   - size queries are pure host functions and never touch the GPU.
 */
#ifndef FHTP_H
#define FHTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pixel types of the input image. */
typedef enum {
    FHTP_U8 = 0,
    FHTP_U16 = 1,
    /* Not pixel types: these two give the enumeration the whole int32 range,
     * so that any int a caller passes is a defined value in C++ as well as C,
     * which the library then rejects with FHTP_ERR_DTYPE. */
    FHTP_DTYPE_RANGE_MIN_ = -2147483647 - 1,
    FHTP_DTYPE_RANGE_MAX_ = 2147483647
} fhtp_dtype;

/* Bend restriction between adjacent links (Section 2.3).
 * mode 0: |d_{i+1} - d_i| <= shift_bound (shift_bound >= 0; gamma_rad ignored).
 * mode 1: bending angle <= gamma_rad (finite, >= 0; shift_bound ignored). */
typedef struct {
    int32_t mode;
    int32_t shift_bound;
    double gamma_rad;
} fhtp_bend;

#define FHTP_OK 0
#define FHTP_ERR_NULL (-1)        /* a required pointer is NULL */
#define FHTP_ERR_DIMS (-2)        /* h,w,k <= 0; k does not divide h; n not a power of two;
                                     n > 1024; w > 2^20 */
#define FHTP_ERR_BEND (-3)        /* bad mode, negative bound, gamma not finite or < 0 */
#define FHTP_ERR_OVERFLOW (-4)    /* h * maxval(dtype) >= 2^31: a score might not fit int32 */
#define FHTP_ERR_WORKSPACE (-5)   /* workspace too small or not 256-byte aligned */
#define FHTP_ERR_HIP (-6)         /* HIP launch or runtime failure; see fhtp_last_error_detail */
#define FHTP_ERR_UNSUPPORTED (-7) /* valid request this build does not implement */
#define FHTP_ERR_DTYPE (-8)       /* dtype is not FHTP_U8 or FHTP_U16 */
#define FHTP_ERR_POINT (-9)       /* through-point query outside the image or band grid */
#define FHTP_ERR_OPTION (-10)     /* an option of fhtp_options is out of range */

/* Human-readable name of an error code (static storage). */
const char* fhtp_strerror(int code);

/* Detail of the last FHTP_ERR_HIP on the calling thread (thread-local storage). */
const char* fhtp_last_error_detail(void);

/* Library version string (static storage). */
const char* fhtp_version(void);

/* Shape of the band tables: bands = k, shifts = 2n-1, width = w+n.
 * Validates h, w, k as above (the pixel type is not involved). */
int fhtp_table_shape(int h, int w, int k, int64_t* bands, int64_t* shifts, int64_t* width);

/* ---------------------------------------------------------------------------
 * Band FHT (Section 2.1, "Subproblem 1"): the Hough image for mostly vertical
 * lines of every zero-extended band.
 *
 *   tables[i][d + n - 1][x] = sum over band rows y of
 *       pixel(i*n + y, (x + sign(d) * D_{|d|}(y)) mod W),  pixel = 0 beyond column w-1,
 *   for i in [0,k), d in [-(n-1), n-1], x in [0, W).
 *
 * img:    device, [h][w] of uint8 or uint16 (per `dtype`), read only.
 * tables: device, [k][2n-1][W] int32, written in full.
 * ws:     device scratch, fhtp_fht_workspace_bytes(...) bytes (0 for n <= 128).
 * Cost: O(W * h * log n) additions (Section 2.1, asymptotic complexity).
 * ------------------------------------------------------------------------- */
int fhtp_fht_workspace_bytes(fhtp_dtype dtype, int h, int w, int k, size_t* bytes);
int fhtp_fht_bands(const void* img, fhtp_dtype dtype, int h, int w, int k, int32_t* tables,
                   void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Bend-limited polyline DP over given band tables (Sections 2.2-2.3, eqs.
 * (3)-(7); main problem steps 2-3; backtrace by eq. (5)).
 *
 * tables: device, [k][2n-1][W] int32 in the layout written by fhtp_fht_bands
 *         (only columns x < w are read); every entry must be >= 0 and the sum
 *         along any polyline must be < 2^31 (true for tables of an image that
 *         passes validation).
 * score:  device, 1 int32: the best polyline score.
 * xs:     device, k+1 int32: x_0 .. x_k (x_i on row i*n for i < k, x_k on row h-1).
 * ws:     device scratch, fhtp_dp_workspace_bytes(...) bytes.
 * ------------------------------------------------------------------------- */
int fhtp_dp_workspace_bytes(int h, int w, int k, fhtp_bend bend, size_t* bytes);
int fhtp_polyline_dp(const int32_t* tables, int h, int w, int k, fhtp_bend bend, void* ws,
                     size_t ws_bytes, int32_t* score, int32_t* xs, void* stream);

/* ---------------------------------------------------------------------------
 * The whole detector: band FHT, then the DP, then the backtrace (the paper's
 * main problem without its Gaussian pre-filter; the input is taken as the
 * already filtered or gradient image).
 *
 * img, dtype, h, w, k as fhtp_fht_bands; bend, score, xs as fhtp_polyline_dp.
 * ws: device scratch, fhtp_detect_workspace_bytes(...) bytes (holds the tables).
 * ------------------------------------------------------------------------- */
int fhtp_detect_workspace_bytes(fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend,
                                size_t* bytes);
int fhtp_detect_polyline(const void* img, fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend,
                         void* ws, size_t ws_bytes, int32_t* score, int32_t* xs, void* stream);

/* ---------------------------------------------------------------------------
 * fhtp_detect_polyline without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It computes exactly what
 * fhtp_detect_polyline computes (same arguments, same results, same errors)
 * but keeps its band tables, value planes, back-pointers and keys in a
 * device array built into the library: fhtp_noalloc_scratch_bytes() bytes
 * (64 MiB) per GPU, held from the library's first use of that GPU until the
 * process ends.  The call allocates and frees nothing.
 *
 * Limit: requests whose fhtp_detect_workspace_bytes exceeds the scratch size
 * (for example a 4096 x 4096 image) return FHTP_ERR_WORKSPACE and enqueue
 * nothing.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap in time on one GPU (different streams,
 * or threads without ordering) race and give undefined results; order them
 * on one stream.  img, score and xs are caller-owned device memory as above.
 * ------------------------------------------------------------------------- */
size_t fhtp_noalloc_scratch_bytes(void);
int fhtp_detect_polyline_noalloc(const void* img, fhtp_dtype dtype, int h, int w, int k,
                                 fhtp_bend bend, int32_t* score, int32_t* xs, void* stream);

/* ---------------------------------------------------------------------------
 * The detector with its optional steps (all off when opt is NULL or zeroed
 * with pin_boundary = -1), applied in this order:
 *
 *   horizontal = 1: mostly horizontal curves (Fig. 7).  The detector runs on
 *       the transposed image: the k bands are vertical strips of w/k columns
 *       (w/k a power of two <= 1024, h <= 2^20, w * maxval < 2^31), links run
 *       left to right, and xs[i] is the ROW of the curve on column i*n
 *       (xs[k] on column w-1).
 *   smooth_radius = r in [0, 7]: each row of the detection image (each
 *       column of the input when horizontal, i.e. always across the curve) is
 *       smoothed before the transform (main problem, step 1).  The Gaussian is
 *       read as the binomial kernel C(2r, i) / 4^r, i = 0..2r (variance r/2),
 *       rows extended by repeating their end pixels, rounded half up:
 *         out(y, x) = (sum_i C(2r, i) * in(y, clamp(x + i - r)) + 4^r/2) >> 2r.
 *       The result keeps the pixel type; r = 0 skips the step.
 *   pin_boundary = j in [0, k], pin_pos = p: only polylines through the
 *       point on band boundary j at position p (a column, or a row when
 *       horizontal) compete: x_j = p (Sections 2.2-2.3, "Subproblems 2-3";
 *       j = 0 is a top point as in main-problem step 2, j = k the last row).
 *       The bend bound holds at every vertex, the point included, so this is
 *       the exact best polyline through the point.  With an unbounded bend it
 *       equals the paper's construction (best lower part from the point plus
 *       the best upper part of the flipped bands above it).  pin_boundary = -1
 *       leaves every polyline free.
 *
 * img: device [h][w] as fhtp_detect_polyline (h, w of the image as stored).
 * ws:  device scratch, fhtp_detect_ex_workspace_bytes(...) bytes (it holds the
 *      transposed / smoothed image when either step is on, then the tables).
 * Errors: FHTP_ERR_OPTION for horizontal not in {0,1} or r outside [0,7];
 *         FHTP_ERR_POINT for j outside [-1, k] or p outside the image;
 *         FHTP_ERR_DIMS / _OVERFLOW checked on the detection image.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t smooth_radius; /* 0 .. 7 */
    int32_t horizontal;    /* 0: mostly vertical curves, 1: mostly horizontal */
    int32_t pin_boundary;  /* -1: no point; else the band boundary j in [0, k] */
    int32_t pin_pos;       /* column (vertical) or row (horizontal) of the point */
} fhtp_options;

/* The detection image alone (the first two optional steps above), for callers
 * that keep it or run the stages themselves:
 *   out = smooth_rows(horizontal ? transpose(img) : img, smooth_radius)
 * img: device [h][w] of dtype; out: device [w][h] when horizontal, else
 * [h][w], same dtype, must not overlap img.  h, w in [1, 2^24].
 * Errors: FHTP_ERR_NULL, FHTP_ERR_DTYPE, FHTP_ERR_DIMS, FHTP_ERR_OPTION. */
int fhtp_prepare_image(const void* img, fhtp_dtype dtype, int h, int w, int smooth_radius,
                       int horizontal, void* out, void* stream);

int fhtp_detect_ex_workspace_bytes(fhtp_dtype dtype, int h, int w, int k, fhtp_bend bend,
                                   const fhtp_options* opt, size_t* bytes);
int fhtp_detect_polyline_ex(const void* img, fhtp_dtype dtype, int h, int w, int k,
                            fhtp_bend bend, const fhtp_options* opt, void* ws, size_t ws_bytes,
                            int32_t* score, int32_t* xs, void* stream);

/* ---------------------------------------------------------------------------
 * Many detections in one call: images of different h, w, k, pixel type and
 * bend restriction.  The result of every job is bit-identical to
 * fhtp_detect_polyline on that job alone; images of the same band height
 * share FHT launches and images of the same window class share every DP step
 * launch, so a batch costs a few launches per band step instead of a few per
 * image and step.
 *
 * jobs:  HOST array of `count` descriptors (read during the call only); the
 *        pointers inside are device pointers as in fhtp_detect_polyline.
 * ws:    device scratch, fhtp_batch_workspace_bytes(...) bytes.
 * Streams: part of the batch (the images with bands of more than 128 rows)
 *        may run on a second, library-owned stream, forked from `stream` and
 *        joined back into it with events; all results are still complete once
 *        `stream` has been synchronised, and the fork/join is valid under
 *        graph capture.  Each caller stream (per device) gets its own second
 *        stream, created on first use outside capture and kept until the
 *        process ends; a plan owns one of its own.  Batches on different
 *        caller streams therefore never share a second stream.
 * Errors: the first invalid job's code; nothing is enqueued in that case.
 * ------------------------------------------------------------------------- */
typedef struct {
    const void* img;  /* device, [h][w] of `dtype` */
    int32_t dtype;    /* fhtp_dtype */
    int32_t h, w, k;
    fhtp_bend bend;
    int32_t* score;   /* device, 1 int32 */
    int32_t* xs;      /* device, k+1 int32 */
} fhtp_job;

int fhtp_batch_workspace_bytes(const fhtp_job* jobs, int count, size_t* bytes);
int fhtp_detect_batch(const fhtp_job* jobs, int count, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Plans: a fixed set of detections (one job or a batch, as fhtp_detect_batch
 * takes them) recorded once as a HIP graph and replayed.  The FHT and the DP
 * of Sections 2.1-2.3 and the backtrace of eq. (5) are a chain of a few dozen
 * dependent launches; a replay submits them as one graph launch.  Results are
 * bit-identical to fhtp_detect_batch on the same jobs.
 *
 * fhtp_plan_create: validates the jobs as fhtp_detect_batch does (same error
 *   codes; nothing is created on error) and copies the descriptors.  The
 *   device buffers they name and `ws` (fhtp_batch_workspace_bytes bytes) are
 *   borrowed: they must stay allocated while the plan exists.  Their contents
 *   may change between launches; every launch reads the images afresh.  The
 *   plan belongs to the current device.
 * fhtp_plan_capture: records the plan's launches into a graph on a stream
 *   the library creates and destroys for the purpose, and instantiates it.
 *   Host call; enqueues nothing.  Calling it again re-records the graph.
 *   FHTP_ERR_HIP if capture or instantiation fails (the plan then stays
 *   usable uncaptured).
 * fhtp_plan_launch: replays the graph on `stream` (a stream of the plan's
 *   device) or, if the plan has not been captured, enqueues the launches
 *   directly; asynchronous.  Launches of one plan share `ws`, so two of them
 *   must not run at the same time (on different streams).
 * fhtp_plan_destroy: frees the plan and its graph (host call).  The caller
 *   first makes sure that no launch of the plan is still running.  A null
 *   plan is accepted.
 * ------------------------------------------------------------------------- */
typedef struct fhtp_plan_s* fhtp_plan;

int fhtp_plan_create(const fhtp_job* jobs, int count, void* ws, size_t ws_bytes, fhtp_plan* plan);
int fhtp_plan_capture(fhtp_plan plan);
int fhtp_plan_launch(fhtp_plan plan, void* stream);
int fhtp_plan_destroy(fhtp_plan plan);

/* ---------------------------------------------------------------------------
 * Tuning rules: launch shapes chosen per kind of request (not part of the
 * method; no rule changes any result, only how the work is cut into
 * launches and workgroups).
 *
 * A rule covers requests by pixel type (-1: any), band height 2^log2n (-1:
 * any), image width in [w_min, w_max] and window kind (0: the fixed window of
 * a mode-0 bound of at most 16 shifts; 1: scanned windows, i.e. larger
 * bounds, the angle form and the unbounded bend; -1: any).  For the requests
 * it covers it sets:
 *   dc:       displacements per thread of one-step fixed-window launches, 8 or
 *             16 (0: the library's choice by grid size);
 *   steps:    the most DP steps one launch takes, 1, 2 or 3 (0: the
 *             library's choice, 2); two and three need dc 8 (or 0), three a
 *             bound of at most 8 shifts and no through-point pin (else two);
 *   stripe:   column tiles per stripe of the multi-step kernels' workgroup
 *             order, 1..64 (0: 16);
 *   fht_grid: 0: the FHT's resident grid loops over the work items; 1: one
 *             workgroup per work item;
 *   small:    0: a detection whose bands are at most 32 rows high and whose
 *             image, tables, value planes and back-pointers fit in 64 KB (and
 *             that has no through-point pin) runs as one workgroup doing the
 *             whole detection in LDS, in a batch always and alone while its
 *             work stays near that of a 64 x 64 image with k = 4; 1: never
 *             (the general kernels).
 * fhtp_tune_set replaces the process-wide rule list (count 0 clears it); at
 *   most 1024 rules, each validated (FHTP_ERR_OPTION, nothing changed, if one
 *   is out of range).  Requests are matched against the rules, first match
 *   wins, when they are planned: every detect call, batch call and plan
 *   capture (a captured plan keeps the shapes it was recorded with).  Requests
 *   without a pixel type (fhtp_polyline_dp) match only rules with dtype -1.
 * fhtp_tune_get copies up to `cap` rules to `out` (host memory) and the rule
 *   count to *count.
 * Host calls, safe to call from any thread.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t dtype;
    int32_t log2n;
    int32_t w_min, w_max;
    int32_t window;
    int32_t dc;
    int32_t steps;
    int32_t stripe;
    int32_t fht_grid;
    int32_t small;
} fhtp_tune_rule;

int fhtp_tune_set(const fhtp_tune_rule* rules, int count);
int fhtp_tune_get(fhtp_tune_rule* out, int cap, int* count);

/* ---------------------------------------------------------------------------
 * Kernel timing, for benchmarks and tuning (not part of the method).
 *
 * fhtp_timing_start: clears earlier records and turns timing on for the
 *   whole process: from then on every run of consecutive launches of one
 *   kernel family that the library makes outside graph capture (a single
 *   launch, or for example the run of two-step DP launches of a detection) is
 *   bracketed by two HIP events recorded on its stream.  A bracket covers its
 *   launches and the gaps between them, plus a little time of its own.
 * fhtp_timing_stop: turns timing off, waits for every recorded event, and
 *   returns one entry per kernel family in order of first launch: the family
 *   name ("fht_reg_kernel", "fht_combine_kernel", "dp_pair_fixed",
 *   "dp_step_fixed", "dp_step_generic", "argmax_table", "walk",
 *   "angle_windows", "prep_kernel", ...), its launch count and the summed
 *   elapsed time of its brackets in milliseconds.  Up to `cap` entries
 *   are written to `out` (host memory); *count receives the number of
 *   families.  FHTP_ERR_HIP if an event could not be read (the entries are
 *   then incomplete).  Host calls; not thread-safe against concurrent
 *   launches on other threads.
 * ------------------------------------------------------------------------- */
typedef struct {
    char name[32];
    int32_t launches;
    double total_ms;
} fhtp_kernel_time;

int fhtp_timing_start(void);
int fhtp_timing_stop(fhtp_kernel_time* out, int cap, int* count);

#ifdef __cplusplus
}
#endif

#endif /* FHTP_H */

/*
 * fhtp_oracle.c -- plain CPU oracle for the FHT + bend-limited DP polyline detector.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP path, and the HIP path never calls it.
 *
 * What it computes (paper: "A Method of Detecting End-To-End Curves of Limited
 * Curvature", Sections 2.1-2.3 and the main-problem solution):
 *
 *   - dyadic digital line pattern D_s(y) for n = 2^p rows (closed form of the
 *     recursive dyadic construction behind the FHT the paper uses in 2.1);
 *   - band tables H_i(x, d): the sum of band i, zero-extended to the right by
 *     n = h/k columns (Section 2.1), along the dyadic line that starts at column
 *     x on the band's first row and is displaced by d columns on its last row.
 *     Computed by DIRECT SUMMATION along every line, one line at a time
 *     (no shift-and-add tree);
 *   - the exact optimum of the k-link polyline problem: the maximum over all
 *     admissible polylines of sum_i H_i(x_i, d_i) (Section 2.1, the polyline
 *     sum), with the bend restriction of Section 2.3, found by the bottom-up
 *     dynamic programme of Sections 2.2-2.3 (eqs. (3)-(4)) with the range
 *     maximum done by a plain scan of every admissible successor, then the
 *     backtrace of eq. (5) and the global choice of the main-problem steps 2-3;
 *   - the same optimum restricted to polylines through a given point on a band
 *     boundary (Sections 2.2-2.3, with the bend bounded at every vertex,
 *     the point included);
 *   - row smoothing with an integer binomial kernel (main problem, step 1) and
 *     the transposed problem for mostly horizontal curves (Fig. 7).
 *
 * Discrete reading (the paper leaves these open; each is stated where used):
 *   - displacements d in [-(n-1), n-1]; table row index d + n - 1;
 *   - link i covers the n rows of band i; x_{i+1} = x_i + d_i; x_k is the
 *     column on the last image row; every vertex lies in [0, w-1];
 *   - tables are cyclic over W = w + n columns (the zero extension);
 *   - bend mode 0: |d_{i+1} - d_i| <= B;  mode 1 (angle form of eqs. (6)-(7)):
 *     |atan(d'/n) - atan(d/n)| <= gamma, tested exactly as
 *     n*|d' - d| <= tan(gamma) * (n*n + d*d') in IEEE double (n*n + d*d' > 0);
 *     gamma >= pi/2 admits every pair;
 *   - infeasible cells hold -1; ties go to the lexicographically smallest
 *     (x_0, d_0, d_1, ..., d_{k-1}).
 *
 * Pins (tests/test_oracle_*.py, all CPU): closed form vs the recursive
 * definition of the pattern, endpoint and step properties, single-pixel
 * impulses, per-shift conservation, n = 1 identity, constant images,
 * brute-force enumeration of every admissible polyline on tiny images and on
 * the whole 64x64 configuration, planted model polylines, the unconstrained
 * special case against a separately coded per-column maximum (Section 2.2),
 * and the fast stage recursion against these direct sums with its exact add
 * count (Section 2.1 complexity).  Through-point results: brute force over
 * the polylines through the point, the maximum over all points of a boundary
 * equal to the free optimum, and, with the bend unbounded, the paper's own
 * construction (lower part plus the flipped upper part).  Smoothing: the
 * identity at radius 0, binomial impulse responses, constant rows, and a
 * library convolution with edge replication.  Horizontal: planted horizontal
 * polylines and the library transpose.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_NULL (-1)
#define OR_ERR_DIMS (-2)
#define OR_ERR_BEND (-3)
#define OR_ERR_OVERFLOW (-4)
#define OR_ERR_UNSUPPORTED (-7)
#define OR_ERR_DTYPE (-8)
#define OR_ERR_POINT (-9)
#define OR_ERR_OPTION (-10)

#define OR_MAX_N 1024
#define OR_MAX_W (1 << 20)
/* pi/2 rounded to double: at or above it every bend is admissible. */
#define OR_HALF_PI 1.57079632679489661923

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static int log2i(int v) {
    int p = 0;
    while ((1 << p) < v) ++p;
    return p;
}

/* Shape checks shared by every entry point of the oracle. */
static int check_shape(int dtype, int h, int w, int k) {
    if (dtype != 0 && dtype != 1) return OR_ERR_DTYPE;
    if (h <= 0 || w <= 0 || k <= 0) return OR_ERR_DIMS;
    if (h % k != 0) return OR_ERR_DIMS;
    int n = h / k;
    if (!is_pow2(n) || n > OR_MAX_N) return OR_ERR_DIMS;
    if (w > OR_MAX_W) return OR_ERR_DIMS;
    /* A polyline takes exactly one pixel per row, so its sum is at most h*maxval. */
    int64_t maxval = dtype == 0 ? 255 : 65535;
    if ((int64_t)h * maxval >= ((int64_t)1 << 31)) return OR_ERR_OVERFLOW;
    return OR_OK;
}

static int check_bend(int mode, int bound, double gamma) {
    if (mode == 0) return bound < 0 ? OR_ERR_BEND : OR_OK;
    if (mode == 1) return (!isfinite(gamma) || gamma < 0.0) ? OR_ERR_BEND : OR_OK;
    return OR_ERR_BEND;
}

/*
 * Dyadic pattern, closed form.  For n = 2^p rows and shift s in [0, n-1] the
 * pattern is defined recursively: D^(1)_0 = [0]; the upper half of D^(n)_s is
 * D^(n/2)_{floor(s/2)} and the lower half is ceil(s/2) + D^(n/2)_{floor(s/2)}.
 * Unrolling: bit (p-1-j) of y adds ceil((s >> j) / 2) = (s >> (j+1)) + ((s >> j) & 1).
 * Returns the column offset of row y (0 <= y < n).
 */
int oracle_dyadic_offset(int n, int s, int y) {
    int p = log2i(n);
    int off = 0;
    for (int j = 0; j < p; ++j) {
        if ((y >> (p - 1 - j)) & 1) off += (s >> (j + 1)) + ((s >> j) & 1);
    }
    return off;
}

int oracle_dyadic_pattern(int n, int s, int32_t* out) {
    if (!out) return OR_ERR_NULL;
    if (!is_pow2(n) || n > OR_MAX_N || s < 0 || s >= n) return OR_ERR_DIMS;
    for (int y = 0; y < n; ++y) out[y] = oracle_dyadic_offset(n, s, y);
    return OR_OK;
}

int oracle_table_shape(int h, int w, int k, int64_t* bands, int64_t* shifts, int64_t* width) {
    if (!bands || !shifts || !width) return OR_ERR_NULL;
    int rc = check_shape(0, h, w, k);
    if (rc != OR_OK && rc != OR_ERR_OVERFLOW) return rc;
    int n = h / k;
    *bands = k;
    *shifts = 2 * (int64_t)n - 1;
    *width = (int64_t)w + n;
    return OR_OK;
}

static inline int64_t pixel(const void* img, int dtype, int w, int row, int col) {
    if (dtype == 0) return ((const uint8_t*)img)[(int64_t)row * w + col];
    return ((const uint16_t*)img)[(int64_t)row * w + col];
}

/*
 * Band tables by direct summation (Section 2.1).  Band i (rows i*n .. i*n+n-1)
 * is extended to the right by n zero columns, giving W = w + n columns; the
 * line with displacement d starting at column x takes, on band row y, the
 * pixel in column (x + sign(d) * D_{|d|}(y)) mod W.
 * tables: [k][2n-1][W] int32, row index d + n - 1, x fastest.
 */
int oracle_fht_bands(const void* img, int dtype, int h, int w, int k, int32_t* tables) {
    if (!img || !tables) return OR_ERR_NULL;
    int rc = check_shape(dtype, h, w, k);
    if (rc != OR_OK) return rc;
    const int n = h / k;
    const int W = w + n;
    const int D = 2 * n - 1;

    int32_t* pat = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * n);
    if (!pat) return OR_ERR_UNSUPPORTED;
    for (int s = 0; s < n; ++s)
        for (int y = 0; y < n; ++y) pat[(size_t)s * n + y] = oracle_dyadic_offset(n, s, y);

    int failed = 0;
#pragma omp parallel
    {
        int64_t* acc = (int64_t*)malloc(sizeof(int64_t) * (size_t)W);
        if (!acc) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for collapse(2) schedule(dynamic)
        for (int i = 0; i < k; ++i) {
            for (int r = 0; r < D; ++r) {
                if (!acc) continue;
                const int d = r - (n - 1);
                const int s = d < 0 ? -d : d;
                const int sigma = d < 0 ? -1 : 1;
                for (int x = 0; x < W; ++x) acc[x] = 0;
                for (int y = 0; y < n; ++y) {
                    const int off = sigma * pat[(size_t)s * n + y];
                    const int row = i * n + y;
                    for (int x = 0; x < W; ++x) {
                        int c = x + off;
                        if (c < 0) c += W;
                        if (c >= W) c -= W;
                        if (c < w) acc[x] += pixel(img, dtype, w, row, c);
                    }
                }
                int32_t* dst = tables + ((size_t)i * D + r) * (size_t)W;
                for (int x = 0; x < W; ++x) dst[x] = (int32_t)acc[x];
            }
        }
        free(acc);
    }
    free(pat);
    return failed ? OR_ERR_UNSUPPORTED : OR_OK;
}

/*
 * Admissible successor test for the bend restriction (Section 2.3).
 * mode 0: |d' - d| <= bound.
 * mode 1: the bending angle between links of displacements d and d' over a band
 * of height n is |atan(d'/n) - atan(d/n)|; it is at most gamma exactly when
 * n*|d'-d| <= tan(gamma)*(n*n + d*d'), because both angles lie in (-pi/4, pi/4),
 * so their difference is below pi/2 and n*n + d*d' > 0.
 */
static int admissible(int mode, int bound, double tan_gamma, int all, int n, int d, int dp) {
    if (mode == 0) {
        int diff = dp - d;
        if (diff < 0) diff = -diff;
        return diff <= bound;
    }
    if (all) return 1;
    double lhs = (double)n * (double)abs(dp - d);
    double rhs = tan_gamma * ((double)n * (double)n + (double)d * (double)dp);
    return lhs <= rhs;
}

/* Host-side window bounds for mode 1, by testing every d' (reported for tests). */
int oracle_angle_window(int n, double gamma, int32_t* lo, int32_t* hi) {
    if (!lo || !hi) return OR_ERR_NULL;
    if (!is_pow2(n) || n > OR_MAX_N) return OR_ERR_DIMS;
    if (!isfinite(gamma) || gamma < 0.0) return OR_ERR_BEND;
    const int all = gamma >= OR_HALF_PI;
    const double t = all ? 0.0 : tan(gamma);
    for (int d = -(n - 1); d <= n - 1; ++d) {
        int first = n, last = -n;
        for (int dp = -(n - 1); dp <= n - 1; ++dp) {
            if (admissible(1, 0, t, all, n, d, dp)) {
                if (first == n) first = dp;
                last = dp;
            }
        }
        lo[d + n - 1] = first;
        hi[d + n - 1] = last;
    }
    return OR_OK;
}

/*
 * Exact optimum of the k-link polyline problem over the band tables.
 *
 * V_{k-1}(x, d) = H_{k-1}(x, d) when 0 <= x + d < w, else -1.
 * For i = k-2 down to 0 (the bottom-up order of Sections 2.2-2.3):
 *   V_i(x, d) = H_i(x, d) + max over admissible d' of V_{i+1}(x + d, d'),
 *   or -1 when x + d leaves [0, w) or no admissible successor is feasible;
 *   pi_i(x, d) = the smallest d' reaching that maximum (a plain ascending scan
 *   that keeps the first strictly larger value).
 * The answer is the first strictly larger V_0(x, d) scanning x then d ascending
 * (main problem, steps 2-3), and the vertices follow eq. (5):
 * x_{i+1} = x_i + d_i, d_{i+1} = pi_i(x_i, d_i).
 *
 * The optional pin (pin_j in [0, k], pin_x) keeps only polylines whose vertex
 * x_{pin_j} equals pin_x: the extreme polyline through the point (pin_x, pin_j*n)
 * of Sections 2.2-2.3 ("Subproblem 2/3"), with every bend restricted, including
 * the one at the point.  pin_j = 0 is a top point of the main problem, step 2.
 * Vertex x_j is the start of link j (j < k) or the end of link k-1 (j = k), so
 * the pin masks V_j(x, d) to x = pin_x, or V_{k-1}(x, d) to x + d = pin_x.
 */
static int pinned_out(int i, int k, int x, int d, int pin_j, int pin_x) {
    if (pin_j < 0) return 0;
    if (pin_j == i && i < k) return x != pin_x;
    if (pin_j == k && i == k - 1) return x + d != pin_x;
    return 0;
}

static int dp_core(const int32_t* tables, int h, int w, int k, int mode, int bound, double gamma,
                   int pin_j, int pin_x, int32_t* score, int32_t* xs) {
    const int n = h / k;
    const int W = w + n;
    const int D = 2 * n - 1;
    const int all = (mode == 1) && gamma >= OR_HALF_PI;
    const double t = (mode == 1 && !all) ? tan(gamma) : 0.0;

    size_t plane = (size_t)D * (size_t)w;
    int64_t* V = (int64_t*)malloc(sizeof(int64_t) * plane);
    int64_t* Vn = (int64_t*)malloc(sizeof(int64_t) * plane);
    int32_t* pi = (int32_t*)malloc(sizeof(int32_t) * plane * (size_t)(k > 1 ? k - 1 : 1));
    unsigned char* adm = (unsigned char*)malloc((size_t)D * D);
    int* lo = (int*)malloc(sizeof(int) * (size_t)D);
    int* hi = (int*)malloc(sizeof(int) * (size_t)D);
    if (!V || !Vn || !pi || !adm || !lo || !hi) {
        free(V); free(Vn); free(pi); free(adm); free(lo); free(hi);
        return OR_ERR_UNSUPPORTED;
    }
    /* adm[r][r'] = is d' = r' - (n-1) an admissible successor of d = r - (n-1);
       lo/hi bracket the admissible r' so the scan below skips the rest. */
    for (int r = 0; r < D; ++r) {
        lo[r] = D;
        hi[r] = -1;
        for (int rp = 0; rp < D; ++rp) {
            int a = admissible(mode, bound, t, all, n, r - (n - 1), rp - (n - 1));
            adm[(size_t)r * D + rp] = (unsigned char)a;
            if (a) {
                if (lo[r] == D) lo[r] = rp;
                hi[r] = rp;
            }
        }
    }

#define TAB(i, x, r) ((int64_t)tables[(((size_t)(i) * D + (r)) * (size_t)W) + (x)])
#define IDX(x, r) ((size_t)(x) * D + (r))

    for (int x = 0; x < w; ++x)
        for (int r = 0; r < D; ++r) {
            int d = r - (n - 1);
            V[IDX(x, r)] = (x + d >= 0 && x + d < w && !pinned_out(k - 1, k, x, d, pin_j, pin_x))
                               ? TAB(k - 1, x, r)
                               : -1;
        }

    for (int i = k - 2; i >= 0; --i) {
        int32_t* pii = pi + (size_t)i * plane;
#pragma omp parallel for schedule(static)
        for (int x = 0; x < w; ++x) {
            for (int r = 0; r < D; ++r) {
                int d = r - (n - 1);
                int xp = x + d;
                if (xp < 0 || xp >= w) {
                    Vn[IDX(x, r)] = -1;
                    pii[IDX(x, r)] = d;
                    continue;
                }
                int64_t best = 0;
                int arg = 0;
                int have = 0;
                for (int rp = lo[r]; rp <= hi[r]; ++rp) {
                    if (!adm[(size_t)r * D + rp]) continue;
                    int64_t v = V[IDX(xp, rp)];
                    if (!have || v > best) {
                        best = v;
                        arg = rp - (n - 1);
                        have = 1;
                    }
                }
                Vn[IDX(x, r)] = (have && best >= 0 && !pinned_out(i, k, x, d, pin_j, pin_x))
                                    ? TAB(i, x, r) + best
                                    : -1;
                pii[IDX(x, r)] = have ? arg : d;
            }
        }
        int64_t* tmp = V;
        V = Vn;
        Vn = tmp;
    }

    int64_t best = -2;
    int bx = 0, bd = 0;
    for (int x = 0; x < w; ++x) {
        for (int r = 0; r < D; ++r) {
            int64_t v = V[IDX(x, r)];
            if (v > best) {
                best = v;
                bx = x;
                bd = r - (n - 1);
            }
        }
    }
    *score = (int32_t)best;
    int x = bx, d = bd;
    xs[0] = x;
    for (int i = 0; i + 1 < k; ++i) {
        int nd = pi[(size_t)i * plane + IDX(x, d + n - 1)];
        x = x + d;
        xs[i + 1] = x;
        d = nd;
    }
    xs[k] = x + d;
#undef TAB
#undef IDX
    free(V); free(Vn); free(pi); free(adm); free(lo); free(hi);
    return OR_OK;
}

int oracle_polyline_dp(const int32_t* tables, int h, int w, int k, int mode, int bound,
                       double gamma, int32_t* score, int32_t* xs) {
    if (!tables || !score || !xs) return OR_ERR_NULL;
    int rc = check_shape(0, h, w, k);
    if (rc != OR_OK && rc != OR_ERR_OVERFLOW) return rc;
    rc = check_bend(mode, bound, gamma);
    if (rc != OR_OK) return rc;
    return dp_core(tables, h, w, k, mode, bound, gamma, -1, -1, score, xs);
}

static int detect_common(const void* img, int dtype, int h, int w, int k, int mode, int bound,
                         double gamma, int pin_j, int pin_x, int32_t* score, int32_t* xs) {
    if (!img || !score || !xs) return OR_ERR_NULL;
    int rc = check_shape(dtype, h, w, k);
    if (rc != OR_OK) return rc;
    rc = check_bend(mode, bound, gamma);
    if (rc != OR_OK) return rc;
    const int n = h / k;
    size_t cells = (size_t)k * (size_t)(2 * n - 1) * (size_t)(w + n);
    int32_t* tables = (int32_t*)malloc(sizeof(int32_t) * cells);
    if (!tables) return OR_ERR_UNSUPPORTED;
    rc = oracle_fht_bands(img, dtype, h, w, k, tables);
    if (rc == OR_OK) rc = dp_core(tables, h, w, k, mode, bound, gamma, pin_j, pin_x, score, xs);
    free(tables);
    return rc;
}

int oracle_detect_polyline(const void* img, int dtype, int h, int w, int k, int mode, int bound,
                           double gamma, int32_t* score, int32_t* xs) {
    return detect_common(img, dtype, h, w, k, mode, bound, gamma, -1, -1, score, xs);
}

/* Best polyline whose first vertex is the top point (x0, 0) (main problem, step 2). */
int oracle_detect_from_top(const void* img, int dtype, int h, int w, int k, int mode, int bound,
                           double gamma, int x0, int32_t* score, int32_t* xs) {
    if (x0 < 0 || x0 >= w) return OR_ERR_POINT;
    return detect_common(img, dtype, h, w, k, mode, bound, gamma, 0, x0, score, xs);
}

/* Best polyline through the point (pin_x, row pin_j*n), pin_j in [0, k]
 * (Sections 2.2-2.3, a point on a band boundary; pin_j = k is the last row). */
int oracle_detect_through_point(const void* img, int dtype, int h, int w, int k, int mode,
                                int bound, double gamma, int pin_j, int pin_x, int32_t* score,
                                int32_t* xs) {
    if (!img || !score || !xs) return OR_ERR_NULL;
    int rc = check_shape(dtype, h, w, k);
    if (rc != OR_OK) return rc;
    if (pin_j < 0 || pin_j > k || pin_x < 0 || pin_x >= w) return OR_ERR_POINT;
    return detect_common(img, dtype, h, w, k, mode, bound, gamma, pin_j, pin_x, score, xs);
}

/*
 * Row-wise smoothing before the transform (main problem, step 1: each image
 * row is convolved with a one-dimensional Gaussian).  Integer reading: the
 * binomial kernel C(2r, i), i = 0..2r (variance r/2), with the row extended by
 * repeating its end pixels, normalised by 4^r with rounding half up:
 *   out(y, x) = (sum_i C(2r, i) * pixel(y, clamp(x + i - r)) + 4^r / 2) >> 2r,
 * r = 0 leaves the image unchanged.  Output has the input's pixel type.
 */
int oracle_smooth_rows(const void* img, int dtype, int h, int w, int radius, void* out) {
    if (!img || !out) return OR_ERR_NULL;
    if (dtype != 0 && dtype != 1) return OR_ERR_DTYPE;
    if (h <= 0 || w <= 0) return OR_ERR_DIMS;
    if (radius < 0 || radius > 7) return OR_ERR_OPTION;
    int64_t coef[15];
    const int L = 2 * radius + 1;
    coef[0] = 1;
    for (int i = 1; i < L; ++i) coef[i] = coef[i - 1] * (2 * radius - i + 1) / i;
    const int64_t half = radius > 0 ? ((int64_t)1 << (2 * radius - 1)) : 0;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            int64_t acc = 0;
            for (int i = 0; i < L; ++i) {
                int c = x + i - radius;
                if (c < 0) c = 0;
                if (c >= w) c = w - 1;
                acc += coef[i] * pixel(img, dtype, w, y, c);
            }
            const int64_t v = (acc + half) >> (2 * radius);
            if (dtype == 0)
                ((uint8_t*)out)[(int64_t)y * w + x] = (uint8_t)v;
            else
                ((uint16_t*)out)[(int64_t)y * w + x] = (uint16_t)v;
        }
    }
    return OR_OK;
}

/*
 * The detector with its optional steps, in this order:
 *   1. orientation 1, mostly horizontal curves (Fig. 7): the image is
 *      transposed, so the k bands become vertical strips of w/k columns and
 *      the result gives the row of the curve on each strip boundary;
 *   2. row smoothing with radius smooth_radius (main problem, step 1), along
 *      the rows of the (possibly transposed) image, i.e. across the curve;
 *   3. the polyline search, through the point (pin_x, pin_j * n) when
 *      pin_j >= 0, else over every polyline.
 * h, w are the dimensions of the image as given; xs receives k + 1 entries.
 */
int oracle_detect_ex(const void* img, int dtype, int h, int w, int k, int mode, int bound,
                     double gamma, int smooth_radius, int orientation, int pin_j, int pin_x,
                     int32_t* score, int32_t* xs) {
    if (!img || !score || !xs) return OR_ERR_NULL;
    if (dtype != 0 && dtype != 1) return OR_ERR_DTYPE;
    if (h <= 0 || w <= 0) return OR_ERR_DIMS;
    if (orientation != 0 && orientation != 1) return OR_ERR_OPTION;
    if (smooth_radius < 0 || smooth_radius > 7) return OR_ERR_OPTION;
    const int hh = orientation ? w : h, ww = orientation ? h : w;
    int rc = check_shape(dtype, hh, ww, k);
    if (rc != OR_OK) return rc;
    if (pin_j >= 0 && (pin_j > k || pin_x < 0 || pin_x >= ww)) return OR_ERR_POINT;
    const size_t bpp = dtype == 0 ? 1 : 2;
    const size_t bytes = bpp * (size_t)h * (size_t)w;
    unsigned char* t = (unsigned char*)malloc(bytes);
    unsigned char* sm = (unsigned char*)malloc(bytes);
    if (!t || !sm) {
        free(t);
        free(sm);
        return OR_ERR_UNSUPPORTED;
    }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const size_t src = (size_t)y * w + x;
            const size_t dst = orientation ? (size_t)x * h + y : src;
            if (dtype == 0)
                t[dst] = ((const uint8_t*)img)[src];
            else
                ((uint16_t*)t)[dst] = ((const uint16_t*)img)[src];
        }
    rc = oracle_smooth_rows(t, dtype, hh, ww, smooth_radius, sm);
    if (rc == OR_OK)
        rc = detect_common(sm, dtype, hh, ww, k, mode, bound, gamma, pin_j, pin_j >= 0 ? pin_x : -1,
                           score, xs);
    free(t);
    free(sm);
    return rc;
}

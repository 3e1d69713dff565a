/* Driver for the sanitizer build of the CPU oracle: every entry point on
 * small seeded images (both pixel types, both bend modes, pins, smoothing,
 * the horizontal form) and on invalid arguments.  Returns 0 when every call
 * returned the expected code; the sanitizers report any memory or
 * undefined-behaviour error on the way. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dyadic_offset(int n, int s, int y);
int oracle_dyadic_pattern(int n, int s, int32_t* out);
int oracle_table_shape(int h, int w, int k, int64_t* bands, int64_t* shifts, int64_t* width);
int oracle_fht_bands(const void* img, int dtype, int h, int w, int k, int32_t* tables);
int oracle_angle_window(int n, double gamma, int32_t* lo, int32_t* hi);
int oracle_polyline_dp(const int32_t* tables, int h, int w, int k, int mode, int bound,
                       double gamma, int32_t* score, int32_t* xs);
int oracle_detect_polyline(const void* img, int dtype, int h, int w, int k, int mode, int bound,
                           double gamma, int32_t* score, int32_t* xs);
int oracle_detect_through_point(const void* img, int dtype, int h, int w, int k, int mode,
                                int bound, double gamma, int pin_j, int pin_x, int32_t* score,
                                int32_t* xs);
int oracle_smooth_rows(const void* img, int dtype, int h, int w, int radius, void* out);
int oracle_detect_ex(const void* img, int dtype, int h, int w, int k, int mode, int bound,
                     double gamma, int radius, int horizontal, int pin_j, int pin_x,
                     int32_t* score, int32_t* xs);

static unsigned int state = 191201884u;
static unsigned int next(void) {
    state = state * 1664525u + 1013904223u;
    return state >> 8;
}

int main(void) {
    int fails = 0;
    int32_t pat[64], lo[127], hi[127], score, xs[33];
    for (int n = 1; n <= 64; n *= 2)
        for (int s = 0; s < n; ++s) fails += oracle_dyadic_pattern(n, s, pat) != 0;
    fails += oracle_angle_window(64, 0.3, lo, hi) != 0;
    const int shapes[][3] = {{8, 5, 4}, {32, 17, 2}, {64, 40, 4}, {48, 9, 3}, {16, 1, 16}, {128, 30, 4}};
    for (unsigned q = 0; q < sizeof shapes / sizeof shapes[0]; ++q) {
        const int h = shapes[q][0], w = shapes[q][1], k = shapes[q][2], n = h / k;
        for (int dtype = 0; dtype < 2; ++dtype) {
            const size_t px = (size_t)h * w;
            void* img = malloc(px * (dtype ? 2 : 1));
            void* sm = malloc(px * (dtype ? 2 : 1));
            for (size_t i = 0; i < px; ++i) {
                if (dtype) ((uint16_t*)img)[i] = (uint16_t)(next() & 0xffff);
                else ((uint8_t*)img)[i] = (uint8_t)(next() & 0xff);
            }
            int32_t* tab = malloc(sizeof(int32_t) * (size_t)k * (2 * n - 1) * (w + n));
            fails += oracle_fht_bands(img, dtype, h, w, k, tab) != 0;
            fails += oracle_polyline_dp(tab, h, w, k, 0, 2, 0.0, &score, xs) != 0;
            fails += oracle_detect_polyline(img, dtype, h, w, k, 0, 1, 0.0, &score, xs) != 0;
            fails += oracle_detect_polyline(img, dtype, h, w, k, 1, 0, 0.4, &score, xs) != 0;
            fails += oracle_detect_polyline(img, dtype, h, w, k, 0, 2 * n, 0.0, &score, xs) != 0;
            fails += oracle_detect_through_point(img, dtype, h, w, k, 0, 1, 0.0, k / 2, w / 2,
                                                 &score, xs) != 0;
            fails += oracle_smooth_rows(img, dtype, h, w, 3, sm) != 0;
            fails += oracle_detect_ex(img, dtype, h, w, k, 0, 1, 0.0, 2, 0, -1, 0, &score, xs) != 0;
            if (h % k == 0 && w % k == 0 && ((w / k) & (w / k - 1)) == 0)
                fails += oracle_detect_ex(img, dtype, h, w, k, 0, 1, 0.0, 1, 1, -1, 0, &score, xs) != 0;
            /* invalid arguments are rejected */
            fails += oracle_detect_polyline(img, dtype, h, w, k + 1, 0, 1, 0.0, &score, xs) == 0;
            fails += oracle_detect_polyline(img, dtype, h, w, k, 0, -1, 0.0, &score, xs) == 0;
            fails += oracle_detect_polyline(img, dtype, h, w, k, 1, 0, NAN, &score, xs) == 0;
            fails += oracle_detect_through_point(img, dtype, h, w, k, 0, 1, 0.0, k + 1, 0, &score,
                                                 xs) == 0;
            free(tab);
            free(sm);
            free(img);
        }
    }
    if (fails) fprintf(stderr, "%d failure(s)\n", fails);
    else printf("oracle driver: all checks passed\n");
    return fails ? 1 : 0;
}

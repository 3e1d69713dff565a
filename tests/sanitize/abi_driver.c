/* Host-side driver for the sanitizer build of the library: every call here
 * fails host validation (or touches no device), so it runs without a GPU.
 * Returns 0 when every code is the expected one; the sanitizers report any
 * memory or undefined-behaviour error on the way. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "fhtp.h"

static int fails = 0;
#define EXPECT(call, want)                                                         \
    do {                                                                           \
        int rc_ = (call);                                                          \
        if (rc_ != (want)) {                                                       \
            fprintf(stderr, "%s:%d: %s returned %d, want %d\n", __FILE__, __LINE__, \
                    #call, rc_, (want));                                           \
            ++fails;                                                               \
        }                                                                          \
    } while (0)

int main(void) {
    uint8_t img[64];
    int32_t score[1], xs[64];
    _Alignas(256) static uint8_t ws[4096];
    size_t bytes = 0;
    fhtp_bend b4 = {0, 4, 0.0}, bneg = {0, -1, 0.0}, bang = {1, 0, 0.3}, bnan = {1, 0, 0.0 / 0.0};
    int64_t bands, shifts, width;

    for (int code = 0; code >= -12; --code)
        if (!fhtp_strerror(code) || !fhtp_strerror(code)[0]) ++fails;
    if (!fhtp_version() || !fhtp_last_error_detail()) ++fails;

    EXPECT(fhtp_table_shape(64, 64, 4, &bands, &shifts, &width), FHTP_OK);
    if (bands != 4 || shifts != 31 || width != 80) ++fails;
    EXPECT(fhtp_table_shape(64, 64, 3, &bands, &shifts, &width), FHTP_ERR_DIMS);
    EXPECT(fhtp_table_shape(96, 64, 4, &bands, &shifts, &width), FHTP_ERR_DIMS);
    EXPECT(fhtp_table_shape(0, 64, 4, &bands, &shifts, &width), FHTP_ERR_DIMS);
    EXPECT(fhtp_table_shape(64, 64, 4, NULL, &shifts, &width), FHTP_ERR_NULL);

    EXPECT(fhtp_detect_workspace_bytes(FHTP_U8, 64, 64, 4, b4, &bytes), FHTP_OK);
    EXPECT(fhtp_detect_workspace_bytes(FHTP_U8, 64, 64, 4, bneg, &bytes), FHTP_ERR_BEND);
    EXPECT(fhtp_detect_workspace_bytes(FHTP_U8, 64, 64, 4, bnan, &bytes), FHTP_ERR_BEND);
    EXPECT(fhtp_detect_workspace_bytes((fhtp_dtype)7, 64, 64, 4, b4, &bytes), FHTP_ERR_DTYPE);
    EXPECT(fhtp_detect_workspace_bytes(FHTP_U16, 1 << 16, 64, 1 << 9, b4, &bytes), FHTP_ERR_OVERFLOW);
    EXPECT(fhtp_dp_workspace_bytes(64, 64, 4, bang, &bytes), FHTP_OK);
    EXPECT(fhtp_fht_workspace_bytes(FHTP_U8, 2048, 100, 4, &bytes), FHTP_OK);
    EXPECT(fhtp_detect_workspace_bytes(FHTP_U8, 64, 64, 4, b4, NULL), FHTP_ERR_NULL);

    /* compute calls rejected before anything is enqueued */
    EXPECT(fhtp_detect_polyline(NULL, FHTP_U8, 64, 64, 4, b4, ws, sizeof ws, score, xs, NULL),
           FHTP_ERR_NULL);
    EXPECT(fhtp_detect_polyline(img, FHTP_U8, 64, 64, 3, b4, ws, sizeof ws, score, xs, NULL),
           FHTP_ERR_DIMS);
    EXPECT(fhtp_detect_polyline(img, FHTP_U8, 64, 64, 4, b4, ws, 16, score, xs, NULL),
           FHTP_ERR_WORKSPACE);
    EXPECT(fhtp_detect_polyline(img, FHTP_U8, 64, 64, 4, b4, ws + 1, sizeof ws - 1, score, xs, NULL),
           FHTP_ERR_WORKSPACE);
    EXPECT(fhtp_polyline_dp(NULL, 64, 64, 4, b4, ws, sizeof ws, score, xs, NULL), FHTP_ERR_NULL);
    EXPECT(fhtp_fht_bands(img, FHTP_U8, 64, 64, 5, (int32_t*)ws, ws, sizeof ws, NULL), FHTP_ERR_DIMS);
    EXPECT(fhtp_detect_polyline_noalloc(img, FHTP_U8, 64, 64, 3, b4, score, xs, NULL), FHTP_ERR_DIMS);
    EXPECT(fhtp_detect_polyline_noalloc(img, FHTP_U16, 4096, 4096, 32, b4, score, xs, NULL),
           FHTP_ERR_WORKSPACE);
    if (fhtp_noalloc_scratch_bytes() == 0) ++fails;

    fhtp_options o = {8, 0, -1, 0};
    EXPECT(fhtp_detect_ex_workspace_bytes(FHTP_U8, 64, 64, 4, b4, &o, &bytes), FHTP_ERR_OPTION);
    o.smooth_radius = 2;
    o.horizontal = 2;
    EXPECT(fhtp_detect_ex_workspace_bytes(FHTP_U8, 64, 64, 4, b4, &o, &bytes), FHTP_ERR_OPTION);
    o.horizontal = 1;
    o.pin_boundary = 5;
    EXPECT(fhtp_detect_ex_workspace_bytes(FHTP_U8, 64, 64, 4, b4, &o, &bytes), FHTP_ERR_POINT);
    o.pin_boundary = 2;
    o.pin_pos = 64;
    EXPECT(fhtp_detect_ex_workspace_bytes(FHTP_U8, 64, 64, 4, b4, &o, &bytes), FHTP_ERR_POINT);
    o.pin_pos = 10;
    EXPECT(fhtp_detect_ex_workspace_bytes(FHTP_U8, 64, 64, 4, b4, &o, &bytes), FHTP_OK);
    EXPECT(fhtp_prepare_image(img, FHTP_U8, 8, 8, 9, 0, ws, NULL), FHTP_ERR_OPTION);

    fhtp_job jobs[3];
    memset(jobs, 0, sizeof jobs);
    for (int q = 0; q < 3; ++q) {
        jobs[q].img = img;
        jobs[q].dtype = FHTP_U8;
        jobs[q].h = 64;
        jobs[q].w = 64;
        jobs[q].k = 4;
        jobs[q].bend = b4;
        jobs[q].score = score;
        jobs[q].xs = xs;
    }
    EXPECT(fhtp_batch_workspace_bytes(jobs, 3, &bytes), FHTP_OK);
    jobs[2].k = 5;
    EXPECT(fhtp_batch_workspace_bytes(jobs, 3, &bytes), FHTP_ERR_DIMS);
    EXPECT(fhtp_detect_batch(jobs, 3, ws, sizeof ws, NULL), FHTP_ERR_DIMS);
    jobs[2].k = 4;
    jobs[1].score = NULL;
    EXPECT(fhtp_detect_batch(jobs, 3, ws, sizeof ws, NULL), FHTP_ERR_NULL);
    EXPECT(fhtp_detect_batch(NULL, 2, ws, sizeof ws, NULL), FHTP_ERR_NULL);
    EXPECT(fhtp_detect_batch(jobs, 0, NULL, 0, NULL), FHTP_OK);
    fhtp_plan plan = NULL;
    EXPECT(fhtp_plan_create(jobs, 3, ws, sizeof ws, &plan), FHTP_ERR_NULL);
    EXPECT(fhtp_plan_launch(NULL, NULL), FHTP_ERR_NULL);
    EXPECT(fhtp_plan_destroy(NULL), FHTP_OK);

    /* tuning rules: validation, replacement, reading back */
    fhtp_tune_rule r[1100];
    memset(r, 0, sizeof r);
    for (int q = 0; q < 1100; ++q) {
        r[q].dtype = -1;
        r[q].log2n = -1;
        r[q].w_min = 0;
        r[q].w_max = 1 << 20;
        r[q].window = -1;
        r[q].steps = q % 4;
        r[q].stripe = q % 65;
        r[q].small = q & 1;
    }
    EXPECT(fhtp_tune_set(r, 1024), FHTP_OK);
    EXPECT(fhtp_tune_set(r, 1025), FHTP_ERR_OPTION);
    int cnt = 0;
    EXPECT(fhtp_tune_get(r + 1024, 10, &cnt), FHTP_OK);
    if (cnt != 1024 || r[1024 + 9].stripe != 9) ++fails;
    r[0].steps = 4;
    EXPECT(fhtp_tune_set(r, 1), FHTP_ERR_OPTION);
    r[0].steps = 0;
    r[0].small = 2;
    EXPECT(fhtp_tune_set(r, 1), FHTP_ERR_OPTION);
    EXPECT(fhtp_tune_set(NULL, 0), FHTP_OK);
    EXPECT(fhtp_tune_get(NULL, 0, &cnt), FHTP_OK);
    if (cnt != 0) ++fails;

    fhtp_kernel_time kt[4];
    EXPECT(fhtp_timing_start(), FHTP_OK);
    EXPECT(fhtp_timing_stop(kt, 4, &cnt), FHTP_OK);
    if (cnt != 0) ++fails;

    if (fails) fprintf(stderr, "%d failure(s)\n", fails);
    else printf("abi driver: all checks passed\n");
    return fails ? 1 : 0;
}

/* Host-side argument validation of every C-ABI entry point, built with AddressSanitizer
 * and UndefinedBehaviorSanitizer (host code only) and run without a GPU. Every call below
 * is rejected by the library's checks before anything is enqueued: the pointers are fake
 * (never dereferenced) addresses. Prints one FAIL line per unexpected status and exits
 * non-zero if there was any; the sanitizers abort on the first error they find. */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "hybrid_denoise.h"

static int n_calls = 0, n_bad = 0;

#define EXPECT(expr, want)                                                                      \
    do {                                                                                        \
        hd_status st_ = (expr);                                                                 \
        ++n_calls;                                                                              \
        if (st_ != (want)) {                                                                    \
            printf("FAIL line %d: %s -> %d (want %d): %s\n", __LINE__, #expr, (int)st_, (int)(want), \
                   hd_last_error());                                                            \
            ++n_bad;                                                                            \
        } else if ((want) != HD_OK && hd_last_error()[0] == '\0') {                             \
            printf("FAIL line %d: %s gave no error message\n", __LINE__, #expr);                \
            ++n_bad;                                                                            \
        }                                                                                       \
    } while (0)

#define IN ((const void *)(uintptr_t)0x100000)
#define OUT ((float *)(uintptr_t)0x4000000)
#define OUT8 ((void *)(uintptr_t)0x4000000)
#define AMF ((void *)(uintptr_t)0x8000000)

static void amf_cases(void) {
    EXPECT(amf_filter(NULL, OUT8, 8, 8, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_NULL);
    EXPECT(amf_filter(IN, NULL, 8, 8, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_NULL);
    EXPECT(amf_filter(IN, OUT8, 0, 8, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, -1, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, INT32_MAX, 8, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, INT32_MIN, INT32_MIN, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, (1 << 20) + 1, 8, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 4, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, -8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, INT64_MAX, 8, HD_U16, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, INT64_MAX, HD_U16, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, INT64_MIN, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, (1LL << 32) + 1, 8, HD_U8, 3, 0, NULL), HD_ERR_DIMS);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, 8, 0, 3, 0, NULL), HD_ERR_DTYPE);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, 8, 3, 3, 0, NULL), HD_ERR_DTYPE);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, 8, -1, 3, 0, NULL), HD_ERR_DTYPE);
    const int32_t bad_smax[] = {1, 2, 4, 0, -3, 33, HD_SMAX_LIMIT + 2, INT32_MIN, INT32_MAX};
    for (size_t i = 0; i < sizeof bad_smax / sizeof bad_smax[0]; ++i)
        EXPECT(amf_filter(IN, OUT8, 8, 8, 8, 8, HD_U8, bad_smax[i], 0, NULL), HD_ERR_SMAX);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, 8, HD_U8, 3, HD_CONTRAST_STRETCH, NULL), HD_ERR_ARG);
    EXPECT(amf_filter(IN, OUT8, 8, 8, 8, 8, HD_U8, 3, 0x80000000u, NULL), HD_ERR_ARG);
    /* overlaps: output inside the input's span, and input inside the output's */
    EXPECT(amf_filter(IN, (char *)IN + 63, 8, 8, 8, 8, HD_U8, 3, 0, NULL), HD_ERR_ALIAS);
    EXPECT(amf_filter((const char *)OUT8 + 100, OUT8, 8, 8, 16, 16, HD_U16, 3, 0, NULL), HD_ERR_ALIAS);
    EXPECT(amf_filter(IN, IN, 1, 1, 1, 1, HD_U8, 3, 0, NULL), HD_ERR_ALIAS);

    EXPECT(amf_filter_parts(IN, OUT8, 8, 8, 8, 8, HD_U8, 3, 0, 0, NULL), HD_ERR_ARG);
    EXPECT(amf_filter_parts(IN, OUT8, 8, 8, 8, 8, HD_U8, 3, 9, 0, NULL), HD_ERR_ARG);
    EXPECT(amf_filter_parts(IN, OUT8, 1000, 8, 8, 8, HD_U8, 3, HD_PARTS_LIMIT + 1, 0, NULL), HD_ERR_ARG);
    EXPECT(amf_filter_parts(IN, OUT8, 8, 8, 8, 8, HD_U8, 3, INT32_MIN, 0, NULL), HD_ERR_ARG);
    EXPECT(amf_filter_parts(IN, OUT8, 8, 8, 8, 8, HD_U8, 6, 2, 0, NULL), HD_ERR_SMAX);
    EXPECT(amf_filter_parts(IN, IN, 8, 8, 8, 8, HD_U8, 3, 2, 0, NULL), HD_ERR_ALIAS);
}

static void wiener_cases(void) {
    const int32_t bad_win[][2] = {{4, 5}, {0, 3}, {17, 3}, {3, -1}, {INT32_MAX, 3}, {3, INT32_MIN},
                                  {HD_WIN_LIMIT + 2, 3}, {2, 2}};
    for (size_t i = 0; i < sizeof bad_win / sizeof bad_win[0]; ++i)
        EXPECT(wiener_filter(IN, OUT, 8, 8, 8, 8, HD_U8, 255, bad_win[i][0], bad_win[i][1], -1.0, NULL, NULL),
               HD_ERR_WINDOW);
    EXPECT(wiener_filter(IN, OUT, 8, 8, 8, 8, HD_U8, 0, 3, 3, -1.0, NULL, NULL), HD_ERR_MAXVAL);
    EXPECT(wiener_filter(IN, OUT, 8, 8, 8, 8, HD_U8, 256, 3, 3, -1.0, NULL, NULL), HD_ERR_MAXVAL);
    EXPECT(wiener_filter(IN, OUT, 8, 8, 8, 8, HD_U16, 65536, 3, 3, -1.0, NULL, NULL), HD_ERR_MAXVAL);
    EXPECT(wiener_filter(IN, OUT, 8, 8, 8, 8, HD_U16, INT32_MIN, 3, 3, -1.0, NULL, NULL), HD_ERR_MAXVAL);
    EXPECT(wiener_filter(IN, (float *)((char *)IN + 60), 8, 8, 8, 8, HD_U8, 255, 3, 3, -1.0, NULL, NULL),
           HD_ERR_ALIAS);
    EXPECT(wiener_filter(IN, OUT, 8, 8, 8, INT64_MAX, HD_U8, 255, 3, 3, -1.0, NULL, NULL), HD_ERR_DIMS);

    EXPECT(wiener_fft(IN, IN, OUT, 7, 8, 8, 8, 8, HD_U8, 255, NULL), HD_ERR_DIMS);
    EXPECT(wiener_fft(IN, IN, OUT, 8, 4097, 4097, 4097, 4097, HD_U8, 255, NULL), HD_ERR_DIMS);
    EXPECT(wiener_fft(IN, IN, OUT, 8192, 8, 8, 8, 8, HD_U8, 255, NULL), HD_ERR_DIMS);
    EXPECT(wiener_fft(IN, NULL, OUT, 8, 8, 8, 8, 8, HD_U8, 255, NULL), HD_ERR_NULL);
    EXPECT(wiener_fft(IN, IN, (float *)IN, 8, 8, 8, 8, 8, HD_U8, 255, NULL), HD_ERR_ALIAS);

    EXPECT(degrade_image(IN, OUT8, 8, 8, 8, 8, HD_U8, 255, -1.0, 0.1, 1, 0, NULL), HD_ERR_ARG);
    EXPECT(degrade_image(IN, OUT8, 8, 8, 8, 8, HD_U8, 255, NAN, 0.1, 1, 0, NULL), HD_ERR_ARG);
    EXPECT(degrade_image(IN, OUT8, 8, 8, 8, 8, HD_U8, 255, INFINITY, 0.1, 1, 0, NULL), HD_ERR_ARG);
    EXPECT(degrade_image(IN, OUT8, 8, 8, 8, 8, HD_U8, 255, 1.0, 1.5, 1, 0, NULL), HD_ERR_ARG);
    EXPECT(degrade_image(IN, OUT8, 8, 8, 8, 8, HD_U8, 255, 1.0, NAN, 1, 0, NULL), HD_ERR_ARG);
    EXPECT(degrade_image(IN, (void *)IN, 8, 8, 8, 16, HD_U8, 255, 1.0, 0.1, 1, 0, NULL), HD_ERR_ALIAS);
    EXPECT(degrade_image(IN, (char *)IN + 3, 8, 8, 8, 8, HD_U8, 255, 1.0, 0.1, 1, 0, NULL), HD_ERR_ALIAS);
    EXPECT(degrade_image(IN, OUT8, 8, 8, 8, 8, HD_U8, 300, 1.0, 0.1, 1, 0, NULL), HD_ERR_MAXVAL);

    EXPECT(contrast_stretch(NULL, 8, 8, 8, NULL), HD_ERR_NULL);
    EXPECT(contrast_stretch(OUT, 8, 0, 8, NULL), HD_ERR_DIMS);
    EXPECT(contrast_stretch(OUT, 8, 8, 7, NULL), HD_ERR_DIMS);
}

static void hybrid_cases(void) {
    typedef hd_status (*hybrid_fn)(const void *, float *, int32_t, int32_t, int64_t, int64_t, int32_t,
                                   int32_t, int32_t, int32_t, int32_t, double, uint32_t, void *, int64_t,
                                   double *, void *);
    const hybrid_fn fns[2] = {hybrid_denoise, hybrid_denoise_noalloc};
    for (int f = 0; f < 2; ++f) {
        hybrid_fn fn = fns[f];
        EXPECT(fn(NULL, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_NULL);
        EXPECT(fn(IN, NULL, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_NULL);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, 7, 255, 3, 3, 3, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_DTYPE);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 2, 3, 3, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_SMAX);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 4, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_WINDOW);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 256, 3, 3, 3, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_MAXVAL);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 4u, NULL, 0, NULL, NULL), HD_ERR_ARG);
        EXPECT(fn(IN, (float *)IN, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL, 0, NULL, NULL), HD_ERR_ALIAS);
        /* the caller's AMF buffer: its own geometry, no overlap with the input or the output */
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, AMF, 4, NULL, NULL), HD_ERR_DIMS);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, AMF, INT64_MAX, NULL, NULL), HD_ERR_DIMS);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, (void *)IN, 8, NULL, NULL), HD_ERR_ALIAS);
        EXPECT(fn(IN, OUT, 8, 8, 8, 8, HD_U8, 255, 3, 3, 3, -1.0, 0, (char *)OUT + 4, 8, NULL, NULL),
               HD_ERR_ALIAS);
    }
    /* the no-allocation entry point rejects images whose scratch exceeds its static array */
    float *far_out = (float *)(uintptr_t)(1ULL << 44);  /* beyond the largest input span */
    EXPECT(hybrid_denoise_noalloc(IN, far_out, 8192, 8192, 8192, 8192, HD_U16, 4095, 3, 3, 3, -1.0, 0, NULL, 0,
                                  NULL, NULL),
           HD_ERR_DIMS);
    EXPECT(hybrid_denoise_noalloc(IN, far_out, 1 << 20, 1 << 20, 1 << 20, 1 << 20, HD_U16, 4095, 3, 3, 3, -1.0,
                                  0, NULL, 0, NULL, NULL),
           HD_ERR_DIMS);
}

static void batched_cases(void) {
    hd_slice sl[3];
    for (int i = 0; i < 3; ++i) {
        sl[i].in = (const char *)IN + i * 0x10000;
        sl[i].out = (float *)((char *)OUT + i * 0x40000);
        sl[i].h = 16;
        sl[i].w = 16;
        sl[i].in_pitch = 16;
        sl[i].out_pitch = 16;
    }
    float ms[HD_STAGES];
    EXPECT(hybrid_denoise_batched(NULL, 3, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_NULL);
    EXPECT(hybrid_denoise_batched(sl, 0, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_ARG);
    EXPECT(hybrid_denoise_batched(sl, -5, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_ARG);
    EXPECT(hybrid_denoise_batched(sl, 3, 9, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_DTYPE);
    EXPECT(hybrid_denoise_batched(sl, 3, HD_U8, 255, 5, 3, 8, -1.0, 0, NULL), HD_ERR_WINDOW);
    EXPECT(hybrid_denoise_batched_timed(sl, 3, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL, NULL), HD_ERR_NULL);
    EXPECT(hd_autotune_batched(sl, 3, HD_U8, 255, 3, 3, 3, 0, NULL, NULL, NULL, NULL), HD_ERR_ARG);
    EXPECT(hd_autotune_batched(NULL, 3, HD_U8, 255, 3, 3, 3, 2, NULL, NULL, NULL, NULL), HD_ERR_NULL);
    sl[2].h = 0;
    EXPECT(hybrid_denoise_batched(sl, 3, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_DIMS);
    if (!strstr(hd_last_error(), "slice 2")) {
        printf("FAIL: batched error does not name the slice: %s\n", hd_last_error());
        ++n_bad;
    }
    sl[2].h = 16;
    sl[1].in_pitch = INT64_MAX;
    EXPECT(hybrid_denoise_batched_timed(sl, 3, HD_U8, 255, 3, 3, 3, -1.0, 0, ms, NULL), HD_ERR_DIMS);
    sl[1].in_pitch = 16;
    sl[0].out = (float *)sl[0].in;
    EXPECT(hybrid_denoise_batched(sl, 3, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_ALIAS);
    sl[0].out = NULL;
    EXPECT(hybrid_denoise_batched(sl, 3, HD_U8, 255, 3, 3, 3, -1.0, 0, NULL), HD_ERR_NULL);
    sl[0].out = (float *)OUT;

    EXPECT(hd_autotune_hybrid(IN, 16, 16, 16, HD_U8, 255, 3, 3, 3, 0, NULL, NULL, NULL, NULL), HD_ERR_ARG);
    EXPECT(hd_autotune_hybrid(IN, 16, 16, 16, HD_U8, 255, 3, 3, 3, INT32_MIN, NULL, NULL, NULL, NULL), HD_ERR_ARG);
    EXPECT(hd_autotune_hybrid(IN, 16, 16, 8, HD_U8, 255, 3, 3, 3, 2, NULL, NULL, NULL, NULL), HD_ERR_DIMS);
    hd_release_plans();
}

static void option_cases(void) {
    EXPECT(hd_set_option(0, 0), HD_ERR_ARG);
    EXPECT(hd_set_option(99, 0), HD_ERR_ARG);
    EXPECT(hd_set_option(INT32_MIN, 0), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_SELECT, 4), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_SELECT, -2), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_FUSE_MOMENTS, 2), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_GRAPHS, -1), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_RESIDENT, INT32_MAX), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_WAIT_LIMIT_US, -2), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_FAIL_ALLOC, -1), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_TILE_ROWS, 48), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_TILE_ROWS, 0), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_SURROGATE_FUSED, 2), HD_ERR_ARG);
    EXPECT(hd_set_option(HD_OPT_SELECT, 2), HD_OK);
    EXPECT(hd_set_option(HD_OPT_SELECT, -1), HD_OK);
    EXPECT(hd_set_option(HD_OPT_WAIT_LIMIT_US, INT32_MAX), HD_OK);
    EXPECT(hd_set_option(HD_OPT_WAIT_LIMIT_US, -1), HD_OK);
    const int32_t caps[] = {hd_resident_capacity(0, 9, 5, 5, -1), hd_resident_capacity(HD_U8, 4, 5, 5, -1),
                            hd_resident_capacity(HD_U8, 9, 6, 5, -1), hd_resident_capacity(HD_U8, 9, 5, 5, 7),
                            hd_resident_capacity(HD_U16, INT32_MIN, 5, 5, -1),
                            hd_resident_capacity(HD_U16, 9, 5, INT32_MAX, -1)};
    for (size_t i = 0; i < sizeof caps / sizeof caps[0]; ++i) {
        ++n_calls;
        if (caps[i] != 0) {
            printf("FAIL: hd_resident_capacity case %zu gave %d for bad keys\n", i, caps[i]);
            ++n_bad;
        }
    }
}

static void surrogate_cases(void) {
    ++n_calls;
    if (surrogate_num_params() != 37601) {
        printf("FAIL: surrogate_num_params %d\n", surrogate_num_params());
        ++n_bad;
    }
    EXPECT(surrogate_create(NULL, NULL), HD_ERR_NULL);
    EXPECT(surrogate_get_state(NULL, NULL, NULL, NULL, NULL), HD_ERR_NULL);
    EXPECT(surrogate_set_state(NULL, NULL, NULL, NULL, 0), HD_ERR_NULL);
    EXPECT(surrogate_get_activation(NULL, 1, NULL, 0), HD_ERR_NULL);
    EXPECT(surrogate_forward(NULL, IN, 1, 8, 8, 8, 64, HD_U8, 255, OUT, 8, 64, NULL), HD_ERR_NULL);
    EXPECT(surrogate_train_step(NULL, IN, 1, 8, 8, 8, 64, HD_U8, 255, OUT, 1e-3f, NULL, NULL, 1, NULL),
           HD_ERR_NULL);
    hd_slice sl;
    sl.in = IN;
    sl.out = OUT;
    sl.h = 8;
    sl.w = 8;
    sl.in_pitch = 8;
    sl.out_pitch = 8;
    EXPECT(surrogate_denoise(NULL, &sl, 1, HD_U8, 255, 9, 5, 5, 0.5f, 0.0f, 1.0f, 0.0f, 3, 1.0f, NULL, NULL, NULL),
           HD_ERR_NULL);
    surrogate_destroy(NULL);
}

int main(void) {
    ++n_calls;
    if (hd_version() < 100) {
        printf("FAIL: hd_version %d\n", hd_version());
        ++n_bad;
    }
    amf_cases();
    wiener_cases();
    hybrid_cases();
    batched_cases();
    option_cases();
    surrogate_cases();
    printf("abi checks: %d calls, %d unexpected\n", n_calls, n_bad);
    return n_bad ? 1 : 0;
}

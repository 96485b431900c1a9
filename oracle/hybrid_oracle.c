/*
 * Plain CPU oracle of the hybrid de-noiser: adaptive median filter (AMF) followed by
 * the local mean / variance adaptive Wiener filter.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct definition that
 * the GPU library is checked against. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it. It shares no code, header or table with the
 * HIP library and must never be called on the product path.
 *
 * Sources (paper: "A Parallel Hybrid Technique for Multi-Noise Removal from Grayscale
 * Medical Images", arXiv 2005.05371):
 *   - Smax must be an odd integer greater than 1, else an error (Alg. 1, procedure
 *     parallelAdapMedian, step a).
 *   - Window sizes k = 3, 5, ..., Smax are tried in order (Alg. 1, level loop).
 *   - Per level: zmin, zmax, zmed of the k x k window (Alg. 1, level loop, statistics).
 *   - Stage A: zmin < zmed < zmax on a pixel not yet resolved; Stage B: zmin < g < zmax;
 *     a pixel passing A keeps g when it passes B, else takes zmed, and is then frozen
 *     (Alg. 1, level-loop masks and output selection).
 *   - Hybrid = Wiener applied to the AMF output (Sec. IV, Fig. 4; Alg. 1, procedure
 *     parallelHybrid).
 * Readings where the paper is silent (each listed with its reason in the design notes):
 *   - border: symmetric padding, repeated periodically for windows larger than the image;
 *   - a pixel that never passes stage A takes zmed of the Smax window (default) or keeps
 *     g (keep mode, the literal reading of the listing's initial copy f = g);
 *   - Wiener: local mean mu and population variance s2 over a wh x ww window of the AMF
 *     output a; noise power nu2 = caller value when >= 0, else the mean of s2 over the
 *     image; out = mu + (a - mu) * max(s2 - nu2, 0) / max(s2, nu2), out = mu when both
 *     are 0; the result is divided by max_value (normalised intensity).
 *
 * Integers: images are int32 arrays, row-major, no padding (pitch = width).
 * Floating point: double throughout; window sums are exact int64 / __int128.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_SMAX (-1)
#define ORC_ERR_DIMS (-2)
#define ORC_ERR_WINDOW (-3)
#define ORC_ERR_NOMEM (-4)

/* Symmetric (half-sample) mirror of index i into [0, n): ... c b a | a b c | c b a ...
 * The extension has period 2n, so it also covers windows wider than the image. */
static long mirror_index(long i, long n) {
    long p = 2 * n;
    long m = i % p;
    if (m < 0) m += p;
    return (m < n) ? m : (p - 1 - m);
}

long oracle_mirror(long i, long n) { return mirror_index(i, n); }

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Adaptive median filter of one image.
 *   g      : noisy input, h*w int32
 *   out    : AMF output, h*w int32
 *   level  : per pixel, the window size k at which stage A passed, or 0 if none did
 *            (may be NULL)
 *   keep   : 0 -> unresolved pixels take zmed of the Smax window; 1 -> they keep g
 * Returns ORC_OK or a negative error code. */
int oracle_amf(const int32_t *g, int32_t *out, int32_t *level, int h, int w, int smax,
               int keep, int nthreads) {
    if (smax <= 1 || (smax % 2) == 0) return ORC_ERR_SMAX;
    if (h < 1 || w < 1) return ORC_ERR_DIMS;
    const int nmax = smax * smax;
    int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        int32_t *win = (int32_t *)malloc(sizeof(int32_t) * (size_t)nmax);
        if (!win) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < h; ++y) {
            if (!win) continue;
            for (int x = 0; x < w; ++x) {
                const int32_t gxy = g[(size_t)y * w + x];
                int32_t result = gxy;
                int32_t resolved_at = 0;
                int32_t zmed = gxy;
                for (int k = 3; k <= smax; k += 2) {
                    const int r = k / 2, n = k * k;
                    int c = 0;
                    for (int dy = -r; dy <= r; ++dy) {
                        const long yy = mirror_index((long)y + dy, h);
                        for (int dx = -r; dx <= r; ++dx) {
                            const long xx = mirror_index((long)x + dx, w);
                            win[c++] = g[(size_t)yy * w + xx];
                        }
                    }
                    qsort(win, (size_t)n, sizeof(int32_t), cmp_i32);
                    const int32_t zmin = win[0];
                    const int32_t zmax = win[n - 1];
                    zmed = win[(n - 1) / 2];
                    if (zmin < zmed && zmed < zmax) {            /* stage A */
                        if (zmin < gxy && gxy < zmax) result = gxy; /* stage B */
                        else result = zmed;
                        resolved_at = k;
                        break;
                    }
                }
                if (!resolved_at) result = keep ? gxy : zmed; /* zmed of the Smax window */
                out[(size_t)y * w + x] = result;
                if (level) level[(size_t)y * w + x] = resolved_at;
            }
        }
        free(win);
    }
    return err ? ORC_ERR_NOMEM : ORC_OK;
}

/* Local window sums of a (exact): s1 = sum a, s2 = sum a^2 over the wh x ww window with
 * symmetric padding; num = N*s2 - s1^2 (N^2 times the population variance). */
static void window_sums(const int32_t *a, int h, int w, int wh, int ww, int y, int x,
                        int64_t *s1, int64_t *s2) {
    const int rh = wh / 2, rw = ww / 2;
    int64_t t1 = 0, t2 = 0;
    for (int dy = -rh; dy <= rh; ++dy) {
        const long yy = mirror_index((long)y + dy, h);
        for (int dx = -rw; dx <= rw; ++dx) {
            const long xx = mirror_index((long)x + dx, w);
            const int64_t v = a[(size_t)yy * w + xx];
            t1 += v;
            t2 += v * v;
        }
    }
    *s1 = t1;
    *s2 = t2;
}

/* Noise power estimate: mean over the image of the local population variance,
 * computed as (sum over pixels of exact numerators) / (N^2 * h * w). */
double oracle_noise_estimate(const int32_t *a, int h, int w, int wh, int ww, int nthreads) {
    const int64_t N = (int64_t)wh * ww;
    __int128 *row_total = (__int128 *)calloc((size_t)h, sizeof(__int128));
    if (!row_total) return -1.0;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int y = 0; y < h; ++y) {
        __int128 t = 0;
        for (int x = 0; x < w; ++x) {
            int64_t s1, s2;
            window_sums(a, h, w, wh, ww, y, x, &s1, &s2);
            t += (__int128)(N * s2 - s1 * s1);
        }
        row_total[y] = t;
    }
    __int128 total = 0;
    for (int y = 0; y < h; ++y) total += row_total[y];
    free(row_total);
    return (double)total / ((double)N * (double)N * (double)h * (double)w);
}

/* Adaptive Wiener filter of the (integer) AMF output a.
 *   noise_var >= 0: use it as nu2; < 0: estimate it (oracle_noise_estimate).
 *   out = [mu + (a - mu) * max(s2 - nu2, 0) / max(s2, nu2)] / max_value, double.
 *   nu2_out receives the nu2 used (may be NULL). */
int oracle_wiener(const int32_t *a, double *out, int h, int w, int wh, int ww,
                  double noise_var, double max_value, double *nu2_out, int nthreads) {
    if (h < 1 || w < 1) return ORC_ERR_DIMS;
    if (wh < 1 || ww < 1 || (wh % 2) == 0 || (ww % 2) == 0) return ORC_ERR_WINDOW;
    const double nu2 = (noise_var >= 0.0) ? noise_var : oracle_noise_estimate(a, h, w, wh, ww, nthreads);
    if (nu2 < 0.0) return ORC_ERR_NOMEM;
    if (nu2_out) *nu2_out = nu2;
    const int64_t N = (int64_t)wh * ww;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            int64_t s1, s2;
            window_sums(a, h, w, wh, ww, y, x, &s1, &s2);
            const double mu = (double)s1 / (double)N;
            const double s2var = (double)(N * s2 - s1 * s1) / ((double)N * (double)N);
            const double axy = (double)a[(size_t)y * w + x];
            const double den = s2var > nu2 ? s2var : nu2;
            double v;
            if (den == 0.0) {
                v = mu;
            } else {
                const double num = (s2var - nu2) > 0.0 ? (s2var - nu2) : 0.0;
                v = mu + (axy - mu) * num / den;
            }
            out[(size_t)y * w + x] = v / max_value;
        }
    }
    return ORC_OK;
}

/* Hybrid = Wiener(AMF(g)). amf_out (h*w int32) receives the AMF stage (may be NULL). */
int oracle_hybrid(const int32_t *g, double *out, int32_t *amf_out, int32_t *level, int h,
                  int w, int smax, int keep, int wh, int ww, double noise_var,
                  double max_value, double *nu2_out, int nthreads) {
    if (h < 1 || w < 1) return ORC_ERR_DIMS;
    int32_t *a = amf_out;
    int own = 0;
    if (!a) {
        a = (int32_t *)malloc(sizeof(int32_t) * (size_t)h * (size_t)w);
        if (!a) return ORC_ERR_NOMEM;
        own = 1;
    }
    int rc = oracle_amf(g, a, level, h, w, smax, keep, nthreads);
    if (rc == ORC_OK)
        rc = oracle_wiener(a, out, h, w, wh, ww, noise_var, max_value, nu2_out, nthreads);
    if (own) free(a);
    return rc;
}

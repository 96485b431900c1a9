/* The CPU oracle's C functions run under AddressSanitizer and UndefinedBehaviorSanitizer.
 * Usage: oracle_checks <dir>. <dir>/cases.txt holds one case per line:
 *     name h w smax keep wh ww max_value threads
 * with the int32 input image in <dir>/<name>.in (h*w values, row-major). For each case the
 * driver writes <name>.amf (int32), <name>.level (int32), <name>.out (float64) and
 * <name>.nu2 (one float64) from oracle_amf + oracle_hybrid (noise power estimated), and
 * checks a few symmetric-padding indices. The test compares the files with the regular
 * build's results bit for bit. Exits non-zero on any failure. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_amf(const int32_t *g, int32_t *out, int32_t *level, int h, int w, int smax, int keep, int nthreads);
int oracle_hybrid(const int32_t *g, double *out, int32_t *amf_out, int32_t *level, int h, int w, int smax,
                  int keep, int wh, int ww, double noise_var, double max_value, double *nu2_out, int nthreads);
long oracle_mirror(long i, long n);

static int read_file(const char *path, void *buf, size_t bytes) {
    FILE *f = fopen(path, "rb");
    if (!f) return -1;
    const size_t got = fread(buf, 1, bytes, f);
    fclose(f);
    return got == bytes ? 0 : -1;
}

static int write_file(const char *path, const void *buf, size_t bytes) {
    FILE *f = fopen(path, "wb");
    if (!f) return -1;
    const size_t put = fwrite(buf, 1, bytes, f);
    return (fclose(f) == 0 && put == bytes) ? 0 : -1;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s <dir>\n", argv[0]);
        return 2;
    }
    /* symmetric padding: period 2n, index i and -1-i and 2n-1-i meet */
    for (long n = 1; n <= 7; ++n)
        for (long i = -40; i <= 40; ++i) {
            const long m = oracle_mirror(i, n);
            if (m < 0 || m >= n || m != oracle_mirror(-1 - i, n) || m != oracle_mirror(i + 2 * n, n)) {
                printf("FAIL mirror(%ld, %ld) = %ld\n", i, n, m);
                return 1;
            }
        }
    char path[4096];
    snprintf(path, sizeof path, "%s/cases.txt", argv[1]);
    FILE *cf = fopen(path, "r");
    if (!cf) {
        printf("FAIL cannot open %s\n", path);
        return 1;
    }
    char name[256];
    int h, w, smax, keep, wh, ww, threads, ncase = 0;
    double maxv;
    while (fscanf(cf, "%255s %d %d %d %d %d %d %lf %d", name, &h, &w, &smax, &keep, &wh, &ww, &maxv, &threads) ==
           9) {
        const size_t n = (size_t)h * (size_t)w;
        int32_t *g = malloc(n * sizeof *g), *a = malloc(n * sizeof *a), *a2 = malloc(n * sizeof *a2);
        int32_t *level = malloc(n * sizeof *level);
        double *out = malloc(n * sizeof *out), nu2 = 0.0;
        if (!g || !a || !a2 || !level || !out) {
            printf("FAIL allocation for %s\n", name);
            return 1;
        }
        snprintf(path, sizeof path, "%s/%s.in", argv[1], name);
        if (read_file(path, g, n * sizeof *g)) {
            printf("FAIL reading %s\n", path);
            return 1;
        }
        int rc = oracle_amf(g, a, level, h, w, smax, keep, threads);
        if (rc == 0) rc = oracle_hybrid(g, out, a2, NULL, h, w, smax, keep, wh, ww, -1.0, maxv, &nu2, threads);
        if (rc != 0) {
            printf("FAIL %s: oracle status %d\n", name, rc);
            return 1;
        }
        if (memcmp(a, a2, n * sizeof *a) != 0) {
            printf("FAIL %s: oracle_amf and oracle_hybrid's AMF stage differ\n", name);
            return 1;
        }
        const char *ext[4] = {"amf", "level", "out", "nu2"};
        const void *buf[4] = {a, level, out, &nu2};
        const size_t bytes[4] = {n * sizeof *a, n * sizeof *level, n * sizeof *out, sizeof nu2};
        for (int i = 0; i < 4; ++i) {
            snprintf(path, sizeof path, "%s/%s.%s", argv[1], name, ext[i]);
            if (write_file(path, buf[i], bytes[i])) {
                printf("FAIL writing %s\n", path);
                return 1;
            }
        }
        free(g);
        free(a);
        free(a2);
        free(level);
        free(out);
        ++ncase;
    }
    fclose(cf);
    /* argument errors come back as status codes */
    int32_t one = 7, o1 = 0;
    double d1 = 0.0;
    if (oracle_amf(&one, &o1, NULL, 1, 1, 4, 0, 1) == 0 || oracle_amf(&one, &o1, NULL, 0, 1, 3, 0, 1) == 0 ||
        oracle_hybrid(&one, &d1, NULL, NULL, 1, 1, 3, 0, 2, 3, -1.0, 255.0, NULL, 1) == 0) {
        printf("FAIL bad arguments accepted\n");
        return 1;
    }
    printf("oracle checks: %d cases\n", ncase);
    return ncase > 0 ? 0 : 1;
}

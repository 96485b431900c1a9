// C ABI of libhybrid_denoise: argument checks, scratch management and launch sequencing.
// The declarations and their contract are in include/hybrid_denoise.h.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../include/hybrid_denoise.h"
#include "hd_internal.h"

namespace {

thread_local char g_last_error[512] = "";

hd_status fail(hd_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

hd_status ok() {
    g_last_error[0] = '\0';
    return HD_OK;
}

hd_status hip_fail(hipError_t e, const char *what) {
    return fail(HD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int dtype_bytes(hd_dtype dt) { return dt == HD_U8 ? 1 : (dt == HD_U16 ? 2 : 0); }

// The grid covers ceil(h / 32) tile rows; keep well inside gridDim.y and int indexing.
constexpr int32_t kMaxSide = 1 << 20;

hd_status check_image(const void *p, int32_t h, int32_t w, int64_t pitch, const char *name) {
    if (!p) return fail(HD_ERR_NULL, "%s is NULL", name);
    if (h < 1 || w < 1 || h > kMaxSide || w > kMaxSide)
        return fail(HD_ERR_DIMS, "bad dimensions %d x %d (each must be in 1..%d)", h, w, kMaxSide);
    if (pitch < w) return fail(HD_ERR_DIMS, "%s pitch %lld < width %d", name, (long long)pitch, w);
    return HD_OK;
}

hd_status check_smax(int32_t smax) {
    if (smax <= 1 || (smax % 2) == 0)
        return fail(HD_ERR_SMAX, "SMAX must be an odd integer > 1 (got %d)", smax);
    if (smax > HD_SMAX_LIMIT)
        return fail(HD_ERR_SMAX, "Smax %d above the library limit %d", smax, HD_SMAX_LIMIT);
    return HD_OK;
}

hd_status check_window(int32_t wh, int32_t ww) {
    if (wh < 1 || ww < 1 || (wh % 2) == 0 || (ww % 2) == 0 || wh > HD_WIN_LIMIT || ww > HD_WIN_LIMIT)
        return fail(HD_ERR_WINDOW, "Wiener window %d x %d must be odd, 1..%d", wh, ww, HD_WIN_LIMIT);
    return HD_OK;
}

hd_status check_maxval(int32_t m, hd_dtype dt) {
    const int32_t top = dt == HD_U8 ? 255 : 65535;
    if (m < 1 || m > top) return fail(HD_ERR_MAXVAL, "max_value %d outside 1..%d", m, top);
    return HD_OK;
}

// Byte ranges [p, p + bytes) overlap?
bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

size_t span_bytes(int32_t h, int32_t w, int64_t pitch, int elem) {
    return ((size_t)(h - 1) * (size_t)pitch + (size_t)w) * (size_t)elem;
}

}  // namespace

extern "C" {

int32_t hd_version(void) { return 100; }

const char *hd_last_error(void) { return g_last_error; }

hd_status amf_filter(const void *in, void *out, int32_t h, int32_t w, int64_t in_pitch,
                     int64_t out_pitch, hd_dtype dt, int32_t smax, uint32_t flags,
                     void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_smax(smax)) != HD_OK) return st;
    if (flags & ~HD_AMF_UNRESOLVED_KEEP) return fail(HD_ERR_ARG, "unknown flags 0x%x", flags);
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, eb)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    hipError_t e = hd::launch_amf(in, out, h, w, in_pitch, out_pitch, eb, smax,
                                  (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "amf launch");
    return ok();
}

// Wiener stage on an integer image `a` (already validated), with scratch for the
// noise accumulator when nu2 is estimated.
static hd_status wiener_core(const void *a, float *out, int32_t h, int32_t w, int64_t a_pitch,
                             int64_t out_pitch, int eb, int32_t max_value, int32_t wh, int32_t ww,
                             double noise_var, double *nu2_out, hipStream_t s) {
    hipError_t e;
    if (noise_var >= 0.0) {
        e = hd::launch_wiener_apply(a, out, h, w, a_pitch, out_pitch, eb, max_value, wh, ww,
                                    nullptr, noise_var, nu2_out, s);
        if (e != hipSuccess) return hip_fail(e, "wiener apply launch");
        return HD_OK;
    }
    hd::NoiseAcc *acc = nullptr;
    e = hipMallocAsync((void **)&acc, sizeof(hd::NoiseAcc), s);
    if (e != hipSuccess || !acc) {
        (void)hipGetLastError();
        return fail(HD_ERR_NOMEM, "scratch allocation failed: %s", hipGetErrorString(e));
    }
    hd_status st = HD_OK;
    if ((e = hd::launch_zero_acc(acc, 1, s)) != hipSuccess) st = hip_fail(e, "zero launch");
    if (st == HD_OK &&
        (e = hd::launch_wiener_partials(a, h, w, a_pitch, eb, wh, ww, acc, s)) != hipSuccess)
        st = hip_fail(e, "wiener partials launch");
    if (st == HD_OK &&
        (e = hd::launch_wiener_apply(a, out, h, w, a_pitch, out_pitch, eb, max_value, wh, ww, acc,
                                     -1.0, nu2_out, s)) != hipSuccess)
        st = hip_fail(e, "wiener apply launch");
    hipError_t ef = hipFreeAsync(acc, s);
    if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "scratch free");
    return st;
}

hd_status wiener_filter(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                        int64_t out_pitch, hd_dtype dt, int32_t max_value, int32_t win_h,
                        int32_t win_w, double noise_var, double *nu2_out, void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_window(win_h, win_w)) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, 4)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    st = wiener_core(in, out, h, w, in_pitch, out_pitch, eb, max_value, win_h, win_w, noise_var,
                     nu2_out, (hipStream_t)stream);
    return st == HD_OK ? ok() : st;
}

hd_status hybrid_denoise(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                         int64_t out_pitch, hd_dtype dt, int32_t max_value, int32_t smax,
                         int32_t win_h, int32_t win_w, double noise_var, uint32_t flags,
                         void *amf_out, int64_t amf_pitch, double *nu2_out, void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_smax(smax)) != HD_OK) return st;
    if ((st = check_window(win_h, win_w)) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (flags & ~HD_AMF_UNRESOLVED_KEEP) return fail(HD_ERR_ARG, "unknown flags 0x%x", flags);
    const size_t in_span = span_bytes(h, w, in_pitch, eb);
    if (overlaps(in, in_span, out, span_bytes(h, w, out_pitch, 4)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    if (amf_out) {
        if ((st = check_image(amf_out, h, w, amf_pitch, "amf_out")) != HD_OK) return st;
        const size_t a_span = span_bytes(h, w, amf_pitch, eb);
        if (overlaps(in, in_span, amf_out, a_span) ||
            overlaps(out, span_bytes(h, w, out_pitch, 4), amf_out, a_span))
            return fail(HD_ERR_ALIAS, "amf_out overlaps the input or the output");
    }
    hipStream_t s = (hipStream_t)stream;
    void *a = amf_out;
    int64_t ap = amf_pitch;
    bool own = false;
    hipError_t e;
    if (!a) {
        ap = w;
        e = hipMallocAsync(&a, (size_t)h * (size_t)w * (size_t)eb, s);
        if (e != hipSuccess || !a) {
            (void)hipGetLastError();
            return fail(HD_ERR_NOMEM, "scratch allocation failed: %s", hipGetErrorString(e));
        }
        own = true;
    }
    e = hd::launch_amf(in, a, h, w, in_pitch, ap, eb, smax, (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0, s);
    if (e != hipSuccess) st = hip_fail(e, "amf launch");
    else st = wiener_core(a, out, h, w, ap, out_pitch, eb, max_value, win_h, win_w, noise_var, nu2_out, s);
    if (own) {
        hipError_t ef = hipFreeAsync(a, s);
        if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "scratch free");
    }
    return st == HD_OK ? ok() : st;
}

}  // extern "C"

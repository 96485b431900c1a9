// C ABI of the learned surrogate: parameter / optimizer state, workspace, forward,
// training step, and de-noising with the per-tile check and fallback to the plain path.
// Declarations and contract: include/hybrid_denoise.h.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/hybrid_denoise.h"
#include "hd_internal.h"
#include "surrogate_internal.h"

using namespace hd::sg;

namespace {
thread_local char g_err[512] = "";
hd_status sfail(hd_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    hd::set_error_message(g_err);  // also reported by hd_last_error()
    return st;
}
hd_status hipfail(hipError_t e, const char *what) {
    return sfail(HD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}
size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

struct hd_surrogate {
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    Weights wt{};
    unsigned char *wbuf = nullptr;  // weight copies
    int step = 0;
    // workspace (grown on demand)
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    long long ws_px = 0;
    uint16_t *act[5] = {};
    uint16_t *dz[2] = {};
    float *y = nullptr, *dy = nullptr, *partials = nullptr;
    double *red = nullptr;  // chunk sums of the partial reduction
    double *loss_part = nullptr;
    size_t partial_floats = 0;
    size_t loss_cap = 0;  // loss partials the workspace holds
    // fallback scratch (device) and the host side of its tables (pinned, reused: a call
    // waits for the previous call's table upload before overwriting it)
    unsigned char *fb = nullptr;
    size_t fb_bytes = 0;
    unsigned char *host_tab = nullptr;
    size_t host_tab_bytes = 0;
    hipEvent_t tab_done = nullptr;
    bool tab_pending = false;
    // the last forward or training step: pixels, and the activations it kept (bit l - 1: A_l)
    long long last_px = 0;
    int kept = 0;
};

namespace {

constexpr int kWgradBlocks = 512;

int tiles16(int B, int H, int W) { return B * ((H + 15) / 16) * ((W + 15) / 16); }
// workgroups of the last layer's forward (one loss partial each): 256-column blocks per row
int loss_blocks(int B, int H, int W) { return ((W + 255) / 256) * H * B; }

// Workspace for a batch of B images of H x W. Growing it frees the old one and allocates
// the new one in stream order on `st` (calls on one object are ordered by the caller).
hd_status ensure_ws(hd_surrogate *s, int B, int H, int W, hipStream_t st) {
    const long long npx = (long long)B * H * W;
    const size_t pf_need = (size_t)std::max<long long>(
        std::max<long long>((long long)tiles16(B, H, W) * (9 * C + 1), (long long)kWgradBlocks * LAYER32),
        (long long)kWgradBlocks * (9 * C + C));
    const size_t nblk = (size_t)loss_blocks(B, H, W);
    if (npx <= s->ws_px && pf_need <= s->partial_floats && nblk <= s->loss_cap && s->ws) return HD_OK;
    if (s->ws) {
        hipError_t e = hipFreeAsync(s->ws, st);
        if (e != hipSuccess) return hipfail(e, "workspace free");
        s->ws = nullptr;
    }
    const long long px = std::max(npx, s->ws_px);
    const size_t act_b = r256((size_t)px * C * 2);
    const size_t f_b = r256((size_t)px * 4);
    const size_t pf = std::max(pf_need, s->partial_floats);
    const size_t lcap = std::max(nblk, s->loss_cap);
    const size_t lp_b = r256(lcap * 8);
    // chunk sums: the widest reduction is a 32-channel layer (LAYER32 entries)
    const size_t red_b = r256((size_t)REDUCE_CHUNKS * LAYER32 * 8);
    const size_t total = 7 * act_b + 2 * f_b + r256(pf * 4) + lp_b + red_b;
    hipError_t e = hipMallocAsync((void **)&s->ws, total, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->ws = nullptr;
        s->ws_px = 0;
        return sfail(HD_ERR_NOMEM, "surrogate workspace (%zu bytes): %s", total, hipGetErrorString(e));
    }
    unsigned char *p = s->ws;
    for (int i = 0; i < 5; ++i, p += act_b) s->act[i] = (uint16_t *)p;
    for (int i = 0; i < 2; ++i, p += act_b) s->dz[i] = (uint16_t *)p;
    s->y = (float *)p;
    p += f_b;
    s->dy = (float *)p;
    p += f_b;
    s->partials = (float *)p;
    p += r256(pf * 4);
    s->loss_part = (double *)p;
    p += lp_b;
    s->red = (double *)p;
    s->ws_bytes = total;
    s->ws_px = px;
    s->partial_floats = pf;
    s->loss_cap = lcap;
    return HD_OK;
}

hd_status check_batch(const void *in, int n_img, int h, int w, int64_t pitch, int64_t img_stride,
                      int32_t dt, int max_value) {
    if (!in) return sfail(HD_ERR_NULL, "input is NULL");
    if (dt != HD_U8 && dt != HD_U16) return sfail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    // n_img and h are launch-grid dimensions (at most 65535 each)
    // pitch and image stride bounded so that every offset below fits in int64
    if (n_img < 1 || h < 1 || w < 1 || n_img > 65535 || h > 65535 || w > 65535 || pitch < w ||
        pitch > (1LL << 32) || img_stride < (int64_t)(h - 1) * pitch + w || img_stride > (1LL << 48))
        return sfail(HD_ERR_DIMS, "bad batch geometry %d x %d x %d (pitch %lld, image stride %lld)", n_img,
                     h, w, (long long)pitch, (long long)img_stride);
    if ((long long)n_img * h * w > (1LL << 31))
        return sfail(HD_ERR_DIMS, "batch too large for one call (%lld pixels)", (long long)n_img * h * w);
    if (max_value < 1 || max_value > (dt == HD_U8 ? 255 : 65535))
        return sfail(HD_ERR_MAXVAL, "max_value %d", max_value);
    return HD_OK;
}

// Forward through layer 5 (activations kept in s->act).
hd_status forward_body(hd_surrogate *s, const void *in, int eb, int B, int H, int W, long long pitch,
                       long long istride, float mval, hipStream_t st) {
    hipError_t e = launch_conv1_fwd(in, eb, pitch, istride, B, H, W, mval, s->wt.w1r, s->params + OFF_B1,
                                    s->act[0], st);
    if (e != hipSuccess) return hipfail(e, "conv1 launch");
    for (int l = 0; l < 4; ++l) {
        e = launch_conv32(true, s->act[l], B, H, W, s->wt.wf[l], s->params + OFF_W2 + l * LAYER32 + 9 * C * C,
                          nullptr, s->act[l + 1], st);
        if (e != hipSuccess) return hipfail(e, "conv32 launch");
    }
    return HD_OK;
}

}  // namespace

extern "C" {

int32_t surrogate_num_params(void) { return N_PARAMS; }

hd_status surrogate_create(hd_surrogate **out, const float *init_params) {
    if (!out) return sfail(HD_ERR_NULL, "out is NULL");
    *out = nullptr;
    hd_surrogate *s = new (std::nothrow) hd_surrogate();
    if (!s) return sfail(HD_ERR_NOMEM, "host allocation");
    const size_t pb = r256((size_t)N_PARAMS * 4);
    unsigned char *base = nullptr;
    hipError_t e = hipMalloc((void **)&base, 4 * pb);
    if (e != hipSuccess) {
        delete s;
        (void)hipGetLastError();
        return sfail(HD_ERR_NOMEM, "parameter buffers: %s", hipGetErrorString(e));
    }
    s->params = (float *)base;
    s->m = (float *)(base + pb);
    s->v = (float *)(base + 2 * pb);
    s->grad = (float *)(base + 3 * pb);
    const size_t wb = r256(9 * C * 4) * 2 + 8 * r256(9 * C * C * 2);
    e = hipMalloc((void **)&s->wbuf, wb);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete s;
        (void)hipGetLastError();
        return sfail(HD_ERR_NOMEM, "weight buffers: %s", hipGetErrorString(e));
    }
    unsigned char *p = s->wbuf;
    s->wt.w1r = (float *)p;
    p += r256(9 * C * 4);
    s->wt.w6r = (float *)p;
    p += r256(9 * C * 4);
    for (int l = 0; l < 4; ++l, p += r256(9 * C * C * 2)) s->wt.wf[l] = (uint16_t *)p;
    for (int l = 0; l < 4; ++l, p += r256(9 * C * C * 2)) s->wt.wb[l] = (uint16_t *)p;
    std::vector<float> zeros((size_t)N_PARAMS, 0.0f);
    e = hipMemcpy(s->params, init_params ? init_params : zeros.data(), (size_t)N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->m, zeros.data(), (size_t)N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->v, zeros.data(), (size_t)N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_adam_prep(s->params, s->m, s->v, nullptr, 0, 0, 0, 0, 0, s->wt, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(s->wbuf);
        (void)hipFree(base);
        delete s;
        return hipfail(e, "parameter upload");
    }
    *out = s;
    return HD_OK;
}

void surrogate_destroy(hd_surrogate *s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    if (s->ws) (void)hipFree(s->ws);
    if (s->fb) (void)hipFree(s->fb);
    if (s->host_tab) (void)hipHostFree(s->host_tab);
    if (s->tab_done) (void)hipEventDestroy(s->tab_done);
    if (s->wbuf) (void)hipFree(s->wbuf);
    if (s->params) (void)hipFree(s->params);
    delete s;
}

hd_status surrogate_get_state(hd_surrogate *s, float *params, float *m, float *v, int32_t *step) {
    if (!s) return sfail(HD_ERR_NULL, "surrogate is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && params) e = hipMemcpy(params, s->params, (size_t)N_PARAMS * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && m) e = hipMemcpy(m, s->m, (size_t)N_PARAMS * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && v) e = hipMemcpy(v, s->v, (size_t)N_PARAMS * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hipfail(e, "state download");
    if (step) *step = s->step;
    return HD_OK;
}

hd_status surrogate_get_activation(hd_surrogate *s, int32_t layer, uint16_t *host, int64_t count) {
    if (!s) return sfail(HD_ERR_NULL, "surrogate is NULL");
    if (!host) return sfail(HD_ERR_NULL, "host is NULL");
    if (layer < 1 || layer > 5) return sfail(HD_ERR_ARG, "layer %d outside 1..5", layer);
    if (!(s->kept & (1 << (layer - 1))))
        return sfail(HD_ERR_ARG, "the last call did not keep activation %d", layer);
    if (count != s->last_px * C)
        return sfail(HD_ERR_ARG, "count %lld != %lld (pixels of the last call x 32)", (long long)count,
                     s->last_px * C);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host, s->act[layer - 1], (size_t)count * 2, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hipfail(e, "activation download");
    return HD_OK;
}

hd_status surrogate_set_state(hd_surrogate *s, const float *params, const float *m, const float *v,
                              int32_t step) {
    if (!s) return sfail(HD_ERR_NULL, "surrogate is NULL");
    if (step < 0) return sfail(HD_ERR_ARG, "step %d < 0", step);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && params) e = hipMemcpy(s->params, params, (size_t)N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && m) e = hipMemcpy(s->m, m, (size_t)N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && v) e = hipMemcpy(s->v, v, (size_t)N_PARAMS * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_adam_prep(s->params, s->m, s->v, nullptr, 0, 0, 0, 0, 0, s->wt, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hipfail(e, "state upload");
    s->step = step;
    return HD_OK;
}

hd_status surrogate_forward(hd_surrogate *s, const void *in, int32_t n_img, int32_t h, int32_t w,
                            int64_t pitch, int64_t img_stride, int32_t dt, int32_t max_value, float *out,
                            int64_t out_pitch, int64_t out_img_stride, void *stream) {
    if (!s) return sfail(HD_ERR_NULL, "surrogate is NULL");
    hd_status st = check_batch(in, n_img, h, w, pitch, img_stride, dt, max_value);
    if (st != HD_OK) return st;
    if (!out) return sfail(HD_ERR_NULL, "out is NULL");
    if (out_pitch < w || out_pitch > (1LL << 32) || out_img_stride < (int64_t)(h - 1) * out_pitch + w ||
        out_img_stride > (1LL << 48))
        return sfail(HD_ERR_DIMS, "bad output geometry");
    if ((st = ensure_ws(s, n_img, h, w, (hipStream_t)stream)) != HD_OK) return st;
    const int eb = dt == HD_U8 ? 1 : 2;
    hipStream_t sm = (hipStream_t)stream;
    s->last_px = (long long)n_img * h * w;
    if (hd::surrogate_fused_inference()) {
        s->kept = 0;  // no activation leaves the chip
        const hipError_t e = launch_stream_forward(in, eb, pitch, img_stride, n_img, h, w, (float)max_value, s->wt,
                                                   s->params, out, out_pitch, out_img_stride, sm);
        if (e != hipSuccess) return hipfail(e, "one-launch forward");
        return HD_OK;
    }
    s->kept = 0x1f;
    if ((st = forward_body(s, in, eb, n_img, h, w, pitch, img_stride, (float)max_value, sm)) != HD_OK) return st;
    hipError_t e = launch_conv6_fwd(s->act[4], in, eb, pitch, img_stride, n_img, h, w, (float)max_value,
                                    s->wt.w6r, s->params + OFF_B6, out, out_pitch, out_img_stride, nullptr,
                                    nullptr, nullptr, sm);
    if (e != hipSuccess) return hipfail(e, "conv6 launch");
    return HD_OK;
}

hd_status surrogate_train_step(hd_surrogate *s, const void *in, int32_t n_img, int32_t h, int32_t w,
                               int64_t pitch, int64_t img_stride, int32_t dt, int32_t max_value,
                               const float *target, float lr, float *loss_out, float *grad_out,
                               int32_t apply_update, void *stream) {
    if (!s) return sfail(HD_ERR_NULL, "surrogate is NULL");
    hd_status st = check_batch(in, n_img, h, w, pitch, img_stride, dt, max_value);
    if (st != HD_OK) return st;
    if (!target) return sfail(HD_ERR_NULL, "target is NULL");
    if (!(lr >= 0.0f)) return sfail(HD_ERR_ARG, "learning rate must be >= 0");
    if ((st = ensure_ws(s, n_img, h, w, (hipStream_t)stream)) != HD_OK) return st;
    const int eb = dt == HD_U8 ? 1 : 2;
    const float mval = (float)max_value;
    const int B = n_img, H = h, W = w;
    s->last_px = (long long)B * H * W;
    s->kept = 0x1f;
    const long long npx = (long long)B * H * W;
    hipStream_t sm = (hipStream_t)stream;
    hipError_t e;
    float *grad = grad_out ? grad_out : s->grad;
    if ((st = forward_body(s, in, eb, B, H, W, pitch, img_stride, mval, sm)) != HD_OK) return st;
    const int nlb = loss_blocks(B, H, W);
    e = launch_conv6_fwd(s->act[4], in, eb, pitch, img_stride, B, H, W, mval, s->wt.w6r, s->params + OFF_B6,
                         s->y, W, (long long)H * W, target, s->dy, s->loss_part, sm);
    if (e != hipSuccess) return hipfail(e, "conv6 launch");
    if (loss_out && (e = launch_reduce_loss(s->loss_part, nlb, npx, loss_out, sm)) != hipSuccess)
        return hipfail(e, "loss reduce launch");
    // layer 6 backward
    e = launch_conv6_bwd(s->dy, s->act[4], B, H, W, s->wt.w6r, s->dz[0], s->partials, sm);
    if (e == hipSuccess)
        e = launch_reduce_partials(s->partials, conv6_bwd_blocks(B, H, W), 9 * C + 1, grad + OFF_W6, s->red, sm);
    if (e != hipSuccess) return hipfail(e, "layer-6 backward launch");
    int cur = 0;
    const int nwb = std::min(kWgradBlocks, tiles16(B, H, W));
    for (int l = 3; l >= 0; --l) {  // layers 5..2: weights l (0-based among the four)
        e = launch_conv32_wgrad(s->dz[cur], s->act[l], B, H, W, nwb, s->partials, sm);
        if (e == hipSuccess) e = launch_reduce_partials(s->partials, nwb, LAYER32, grad + OFF_W2 + l * LAYER32, s->red, sm);
        if (e == hipSuccess)
            e = launch_conv32(false, s->dz[cur], B, H, W, s->wt.wb[l], nullptr, s->act[l], s->dz[cur ^ 1], sm);
        if (e != hipSuccess) return hipfail(e, "32-channel backward launch");
        cur ^= 1;
    }
    e = launch_conv1_wgrad(s->dz[cur], in, eb, pitch, img_stride, B, H, W, mval, nwb, s->partials, sm);
    if (e == hipSuccess) e = launch_reduce_partials(s->partials, nwb, 9 * C + C, grad + OFF_W1, s->red, sm);
    if (e != hipSuccess) return hipfail(e, "layer-1 backward launch");
    if (apply_update) {
        s->step += 1;
        e = launch_adam_prep(s->params, s->m, s->v, grad, s->step, lr, 0.9f, 0.999f, 1e-8f, s->wt, sm);
        if (e != hipSuccess) return hipfail(e, "adam launch");
    }
    return HD_OK;
}

hd_status surrogate_denoise(hd_surrogate *s, const hd_slice *slices, int32_t n, int32_t dt,
                            int32_t max_value, int32_t smax, int32_t win_h, int32_t win_w, float p_max,
                            float r_lo, float r_hi, float d_hi, int32_t check_smax, float threshold,
                            int32_t *n_fallback_out, float *tile_scores_out, void *stream) {
    if (!s) return sfail(HD_ERR_NULL, "surrogate is NULL");
    if (!slices || n < 1) return sfail(HD_ERR_ARG, "no slices");
    if (!(p_max > 0.0f) || !(r_hi > 0.0f) || !(r_lo >= 0.0f) || !(threshold >= 0.0f) || !(d_hi >= 0.0f))
        return sfail(HD_ERR_ARG,
                     "calibration must satisfy p_max > 0, r_hi > 0, r_lo >= 0, d_hi >= 0, threshold >= 0");
    if (smax <= 1 || smax % 2 == 0 || smax > HD_SMAX_LIMIT) return sfail(HD_ERR_SMAX, "SMAX must be an odd integer > 1");
    const bool deviation = d_hi > 0.0f;
    if (deviation && (check_smax <= 1 || check_smax % 2 == 0 || check_smax > smax))
        return sfail(HD_ERR_SMAX, "check_smax %d must be odd, > 1 and <= smax", check_smax);
    if (win_h < 1 || win_w < 1 || win_h % 2 == 0 || win_w % 2 == 0 || win_h > HD_WIN_LIMIT || win_w > HD_WIN_LIMIT)
        return sfail(HD_ERR_WINDOW, "bad Wiener window");
    const int eb = dt == HD_U8 ? 1 : (dt == HD_U16 ? 2 : 0);
    if (!eb) return sfail(HD_ERR_DTYPE, "unknown dtype");
    hipStream_t sm = (hipStream_t)stream;
    hd_status st;
    // 1. surrogate forward, slice by slice, straight into the outputs
    for (int i = 0; i < n; ++i) {
        const hd_slice &q = slices[i];
        if (!q.out) return sfail(HD_ERR_NULL, "slice %d: out is NULL", i);
        // bounds that keep the image strides below in int64 (the full geometry check follows)
        if (q.h < 1 || q.h > 65535 || q.in_pitch > (1LL << 32) || q.out_pitch > (1LL << 32))
            return sfail(HD_ERR_DIMS, "slice %d: bad geometry %d x %d (pitches %lld, %lld)", i, q.h, q.w,
                         (long long)q.in_pitch, (long long)q.out_pitch);
        st = surrogate_forward(s, q.in, 1, q.h, q.w, q.in_pitch, (int64_t)q.h * q.in_pitch, dt, max_value,
                               q.out, q.out_pitch, (int64_t)q.h * q.out_pitch, stream);
        if (st != HD_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "slice %d: %s", i, g_err);
            return sfail(st, "%s", msg);
        }
    }
    // 2. tables: slices with their stage tiles (64 x 32) and check tiles (64 x 64)
    std::vector<hd::SliceDesc> tab((size_t)n);
    std::vector<int> check_begin((size_t)n);
    int nt = 0, nc = 0;
    size_t a_off = 0, p_off = 0;
    std::vector<size_t> a_offs((size_t)n), p_offs((size_t)n);
    for (int i = 0; i < n; ++i) {
        const hd_slice &q = slices[i];
        const int64_t ap = ((int64_t)q.w * eb + 15) / 16 * 16 / eb;
        a_offs[(size_t)i] = a_off;
        a_off += r256((size_t)q.h * ap * eb);
        p_offs[(size_t)i] = p_off;
        if (deviation) p_off += r256((size_t)q.h * q.w * 4);
        hd::SliceDesc &d = tab[(size_t)i];
        d.in = q.in;
        d.amf = nullptr;
        d.out = q.out;
        d.in_pitch = q.in_pitch;
        d.amf_pitch = ap;
        d.out_pitch = q.out_pitch;
        d.h = q.h;
        d.w = q.w;
        d.tiles_x = (q.w + hd::TILE_X - 1) / hd::TILE_X;
        d.tile_begin = nt;
        nt += d.tiles_x * ((q.h + hd::TILE_Y - 1) / hd::TILE_Y);
        check_begin[(size_t)i] = nc;
        nc += ((q.w + 63) / 64) * ((q.h + 63) / 64);
    }
    // scratch: [a images][proxy images][table][check_begin][proxy pointers][flags nt][list nt][count]
    //          [partials nt][nu2 n][scores nc]
    const size_t tab_b = r256(sizeof(hd::SliceDesc) * (size_t)n);
    const size_t cb_b = r256(4 * (size_t)n);
    const size_t pp_b = r256(sizeof(float *) * (size_t)n);
    const size_t fl_b = r256(4 * (size_t)nt);
    const size_t part_b = r256(8 * (size_t)nt);
    const size_t nu_b = r256(8 * (size_t)n);
    const size_t sc_b = r256(4 * (size_t)nc);
    const size_t need = a_off + p_off + tab_b + cb_b + pp_b + 2 * fl_b + 256 + part_b + nu_b + sc_b;
    hipError_t e;
    if (need > s->fb_bytes) {
        // regrown in stream order, like the workspace
        if (s->fb) {
            if ((e = hipFreeAsync(s->fb, sm)) != hipSuccess) return hipfail(e, "fallback scratch free");
            s->fb = nullptr;
            s->fb_bytes = 0;
        }
        e = hipMallocAsync((void **)&s->fb, need, sm);
        if (e != hipSuccess || !s->fb) {
            (void)hipGetLastError();
            s->fb = nullptr;
            return sfail(HD_ERR_NOMEM, "fallback scratch (%zu bytes): %s", need, hipGetErrorString(e));
        }
        s->fb_bytes = need;
    }
    unsigned char *p = s->fb;
    for (int i = 0; i < n; ++i) tab[(size_t)i].amf = p + a_offs[(size_t)i];
    p += a_off;
    unsigned char *proxy_base = p;
    p += p_off;
    hd::SliceDesc *d_tab = (hd::SliceDesc *)p;
    p += tab_b;
    int *d_cb = (int *)p;
    p += cb_b;
    float **d_proxies = (float **)p;
    p += pp_b;
    int *d_flags = (int *)p;
    p += fl_b;
    int *d_list = (int *)p;
    p += fl_b;
    int *d_count = (int *)p;
    p += 256;
    unsigned long long *d_part = (unsigned long long *)p;
    p += part_b;
    double *d_nu2 = (double *)p;
    p += nu_b;
    float *d_scores = tile_scores_out ? tile_scores_out : (float *)p;
    // 3. the plain-output proxy: the plain hybrid with the AMF stopped at check_smax (the
    //    ordinary batched call, into the proxy images)
    if (deviation) {
        std::vector<hd_slice> ps((size_t)n);
        for (int i = 0; i < n; ++i) {
            ps[(size_t)i] = slices[i];
            ps[(size_t)i].out = (float *)(proxy_base + p_offs[(size_t)i]);
            ps[(size_t)i].out_pitch = slices[i].w;
        }
        if ((st = hybrid_denoise_batched(ps.data(), n, dt, max_value, check_smax, win_h, win_w, -1.0, 0, stream)) !=
            HD_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "plain-output proxy: %s", hd_last_error());
            return sfail(st, "%s", msg);
        }
    }
    // 4. the tables, through the object's pinned host buffer (in stream order; the buffer is
    //    reused once the previous call's upload has completed)
    const size_t hb = tab_b + cb_b + pp_b;
    if (s->tab_pending && (e = hipEventSynchronize(s->tab_done)) != hipSuccess) return hipfail(e, "table reuse");
    s->tab_pending = false;
    if (hb > s->host_tab_bytes) {
        if (s->host_tab) (void)hipHostFree(s->host_tab);
        s->host_tab = nullptr;
        s->host_tab_bytes = 0;
        if ((e = hipHostMalloc((void **)&s->host_tab, hb, hipHostMallocDefault)) != hipSuccess) {
            (void)hipGetLastError();
            s->host_tab = nullptr;
            return sfail(HD_ERR_NOMEM, "pinned table buffer: %s", hipGetErrorString(e));
        }
        s->host_tab_bytes = hb;
    }
    if (!s->tab_done && (e = hipEventCreateWithFlags(&s->tab_done, hipEventDisableTiming)) != hipSuccess)
        return hipfail(e, "table event");
    memcpy(s->host_tab, tab.data(), sizeof(hd::SliceDesc) * (size_t)n);
    memcpy(s->host_tab + tab_b, check_begin.data(), 4 * (size_t)n);
    float **hp = (float **)(s->host_tab + tab_b + cb_b);
    for (int i = 0; i < n; ++i) hp[i] = (float *)(proxy_base + p_offs[(size_t)i]);
    if ((e = hipMemcpyAsync(d_tab, s->host_tab, hb, hipMemcpyHostToDevice, sm)) != hipSuccess ||
        (e = hipEventRecord(s->tab_done, sm)) != hipSuccess)
        return hipfail(e, "fallback table upload");
    s->tab_pending = true;
    // flags and the list count start at zero (kernels: no memset nodes if the caller captures)
    if ((e = hd::launch_zero_u32((unsigned int *)d_count, 1, sm)) != hipSuccess ||
        (e = hd::launch_zero_u32((unsigned int *)d_flags, nt, sm)) != hipSuccess)
        return hipfail(e, "fallback scratch clear");
    hd::SliceSet set{};
    set.one = tab[0];
    set.many = n > 1 ? d_tab : nullptr;
    set.n = n;
    // 5. per-tile check -> flags + list of failing stage tiles
    e = launch_tile_check(set, nc, d_cb, eb, (float)max_value, p_max, r_lo, r_hi,
                          deviation ? (const float *const *)d_proxies : nullptr, d_hi, threshold, d_scores, d_flags,
                          d_list, d_count, sm);
    if (e != hipSuccess) return hipfail(e, "tile check launch");
    // 6. plain path on the failing tiles: AMF with the Wiener ring, noise power over the
    //    failing tiles of each slice, Wiener apply into the outputs
    set.list = d_list;
    set.list_count = d_count;
    set.flags = d_flags;
    e = hd::launch_amf_stage(set, nt, eb, smax, 0, win_h, win_w, d_part, hd::SELECT_AUTO, false, sm);
    if (e == hipSuccess) e = hd::launch_noise_reduce(set, d_part, win_h, win_w, d_nu2, sm);
    if (e == hipSuccess)
        e = hd::launch_wiener_stage(set, nt, eb, max_value, win_h, win_w, true, d_nu2, -1.0, nullptr, false, sm);
    if (e != hipSuccess) return hipfail(e, "fallback launch");
    if (n_fallback_out && (e = hipMemcpyAsync(n_fallback_out, d_count, 4, hipMemcpyDeviceToDevice, sm)) != hipSuccess)
        return hipfail(e, "fallback count copy");
    return HD_OK;
}

}  // extern "C"

// Internal declarations of the learned-surrogate kernels (6-layer 3x3 conv, 32 channels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hd_internal.h"

namespace hd {
namespace sg {

constexpr int C = 32;
// flat fp32 parameter vector: W1 [9][32], b1, W2..W5 [9][32][32] + bias, W6 [9][32], b6
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = 9 * C;
constexpr int OFF_W2 = OFF_B1 + C;
constexpr int LAYER32 = 9 * C * C + C;  // weights + bias of one 32 -> 32 layer
constexpr int OFF_W6 = OFF_W2 + 4 * LAYER32;
constexpr int OFF_B6 = OFF_W6 + 9 * C;
constexpr int N_PARAMS = OFF_B6 + 1;  // 37601

// Device copies of the weights in the form each kernel reads them.
struct Weights {
    float *w1r;         // [9][32] bf16-rounded W1 (fp32 storage)
    float *w6r;         // [9][32] bf16-rounded W6
    uint16_t *wf[4];    // layers 2..5, bf16, forward layout [t][co][ci]
    uint16_t *wb[4];    // layers 2..5, bf16, backward-data layout [t][ci][co] = W[8 - t][co][ci]
};

hipError_t launch_conv1_fwd(const void *g, int eb, long long pitch, long long img_stride, int B, int H, int W,
                            float mval, const float *w1r, const float *b1, uint16_t *a1, hipStream_t s);
hipError_t launch_conv32(bool fwd, const uint16_t *in, int B, int H, int W, const uint16_t *wt,
                         const float *bias, const uint16_t *mask, uint16_t *out, hipStream_t s);
hipError_t launch_conv6_fwd(const uint16_t *a5, const void *g, int eb, long long pitch, long long img_stride,
                            int B, int H, int W, float mval, const float *w6r, const float *b6, float *y,
                            long long y_pitch, long long y_img_stride, const float *target, float *dy,
                            double *loss_partials, hipStream_t s);
// Inference in one launch (the row-streaming kernel), bit-identical to conv1 + 4 x conv32 +
// conv6; no activation is stored.
hipError_t launch_stream_forward(const void *g, int eb, long long pitch, long long img_stride, int B, int H, int W,
                                 float mval, const Weights &wt, const float *params, float *y, long long y_pitch,
                                 long long y_img_stride, hipStream_t s);
int conv6_bwd_blocks(int B, int H, int W);
hipError_t launch_conv6_bwd(const float *dy, const uint16_t *a5, int B, int H, int W, const float *w6r,
                            uint16_t *dz5, float *partials, hipStream_t s);
hipError_t launch_conv32_wgrad(const uint16_t *dz, const uint16_t *a_prev, int B, int H, int W, int nblocks,
                               float *partials, hipStream_t s);
hipError_t launch_conv1_wgrad(const uint16_t *dz, const void *g, int eb, long long pitch, long long img_stride,
                              int B, int H, int W, float mval, int nblocks, float *partials, hipStream_t s);
// sum of nblocks partial rows of n floats into grad (double, fixed order), through red:
// at most REDUCE_CHUNKS x n doubles of scratch
constexpr int REDUCE_CHUNKS = 64;
hipError_t launch_reduce_partials(const float *partials, int nblocks, int n, float *grad, double *red,
                                  hipStream_t s);
hipError_t launch_reduce_loss(const double *partials, int n, long long npx, float *loss, hipStream_t s);
hipError_t launch_adam_prep(float *w, float *m, float *v, const float *grad, int step, float lr, float b1,
                            float b2, float eps, const Weights &wt, hipStream_t s);
// proxies: device array of one dense float32 image per slice (the plain output proxy), or
// null for no deviation term; d_hi: the deviation bound (root mean square).
hipError_t launch_tile_check(const SliceSet &set, int n_check, const int *check_begin, int eb, float mval,
                             float p_max, float r_lo, float r_hi, const float *const *proxies, float d_hi,
                             float threshold, float *scores, int *flags, int *list, int *count, hipStream_t s);

}  // namespace sg
}  // namespace hd

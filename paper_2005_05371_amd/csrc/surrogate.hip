// Learned surrogate of the hybrid filter on gfx950: a 6-layer 3x3 convolutional network,
// 32 channels, ReLU, residual output, with bf16 weights / activations and fp32
// accumulation. Every inference layer runs on the matrix cores: the 32 -> 32 layers
// (forward, backward-data, backward-weight) with v_mfma_f32_16x16x32_bf16, layer 1 with
// v_mfma_f32_16x16x4f32 (its input x = g / M is fp32), layer 6 with the bf16 instruction and
// the taps as the rows of A. The training forms of layer 6 and the layer-1 / layer-6
// gradients are plain vector code. Inference runs either one launch per layer (the
// training forward, activations stored) or the whole network in one row-streaming launch
// (network_stream_kernel), bit-identical.
//
// Network: x = g / M; Z_l[p, co] = sum_t sum_ci X[p + off_t, ci] W_l[t, co, ci] + b_l[co]
// (t = ky * 3 + kx, off_t = (ky - 1, kx - 1), zero padding at the image border);
// A_l = relu(Z_l), l = 1..5; y = x + Z_6. Loss: mean over pixels of (y - target)^2.
// Stored in bf16 (round to nearest even): the weights the layers use, the activations
// A_1..A_5 and the gradients dZ_1..dZ_5. Everything else is fp32.
//
// Layout: activations NHWC, [image][row][col][32] bf16 (64 bytes per pixel).
// Parameters (fp32 master copy, flat): W1 [9][32] (tap, co), b1 [32], W2..W5 [9][32][32]
// (tap, co, ci) each followed by its bias [32], W6 [9][32] (tap, ci), b6 [1].
//
// MFMA use (16x16x32 bf16: lane l holds row l % 16 of A and column l % 16 of B, with k
// elements 8 * (l / 16) .. + 8; C gives lane l column l % 16, rows 4 * (l / 16) .. + 4):
//  * forward / backward-data: C[co][px] += W[t][co][ci] x X[px + off_t][ci], M = 16 output
//    channels, N = 16 pixels of one row, K = the 32 input channels of one tap; per 16
//    pixels 9 taps x 2 channel halves = 18 instructions. The weight operands stay in
//    registers for the whole (persistent) workgroup; pixel operands are 16-byte LDS reads
//    (NHWC), and the next tile's input is loaded into registers while the MFMAs run.
//  * backward-weight: C[co][ci] += sum_px dZ[px][co] x X[px + off_t][ci], K = 32 pixels
//    (two 8-pixel halves of two rows); both operands staged channel-major in LDS, so that
//    each is one 16-byte read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "surrogate_internal.h"
#include "tile_io.h"

namespace hd {
namespace sg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// pixel stride in LDS tiles: 32 channels + 8 pad (80 bytes) spreads the rows over banks
constexpr int CP = 40;
constexpr int TS = 16;  // output tile side (16 x 16 pixels)
constexpr int HS = TS + 2;

// Stage a (TS + 2)^2 NHWC bf16 tile with a 1-pixel zero border into LDS (stride CP).
__device__ __forceinline__ void stage_act(uint16_t *lds, const uint16_t *__restrict__ act, int H, int W,
                                          int b, int y0, int x0) {
    for (int i = threadIdx.x; i < HS * HS * 4; i += 256) {
        const int px = i >> 2, part = i & 3;
        const int ly = px / HS, lx = px - ly * HS;
        const int gy = y0 + ly - 1, gx = x0 + lx - 1;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *(const uint4 *)(act + (((long long)b * H + gy) * W + gx) * C + part * 8);
        *(uint4 *)(lds + px * CP + part * 8) = v;
    }
}

// Workgroup barrier that orders LDS only: the global loads and stores in flight are not
// waited for (the kernel using it exchanges nothing through global memory within a
// workgroup; registers loaded from global memory are waited for where they are used). A
// plain __syncthreads() would also drain every outstanding global access, including the
// input rows loaded ahead, at each of its many barriers.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Tile index t -> image b and the tile's top-left pixel (y0, x0), 16 x 16 tiles.
__device__ __forceinline__ void tile_at(int t, int ntx, int nty, int &b, int &y0, int &x0) {
    const int per = ntx * nty;
    b = t / per;
    const int r = t - b * per;
    const int ty = r / ntx;
    y0 = ty * TS;
    x0 = (r - ty * ntx) * TS;
}

// A SIDE x SIDE NHWC bf16 region at (y0 - RING, x0 - RING) (zero outside the image) in
// registers, 16-byte pieces spread over the workgroup: fetched from global memory ahead of
// use, then put into LDS (stride CP), so that a persistent workgroup's next loads are in
// flight while it computes.
template <int SIDE, int RING>
struct RegionRegs {
    static constexpr int PER = (SIDE * SIDE * 4 + 255) / 256;
    uint4 v[PER];
    __device__ __forceinline__ void fetch(const uint16_t *__restrict__ act, int H, int W, int b, int y0, int x0) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            uint4 q = make_uint4(0, 0, 0, 0);
            if (i < SIDE * SIDE * 4) {
                const int px = i >> 2, part = i & 3;
                const int ly = px / SIDE, lx = px - ly * SIDE;
                const int gy = y0 + ly - RING, gx = x0 + lx - RING;
                if (gy >= 0 && gy < H && gx >= 0 && gx < W)
                    q = *(const uint4 *)(act + (((long long)b * H + gy) * W + gx) * C + part * 8);
            }
            v[k] = q;
        }
    }
    __device__ __forceinline__ void put(uint16_t *lds) const {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            if (i < SIDE * SIDE * 4) *(uint4 *)(lds + (i >> 2) * CP + (i & 3) * 8) = v[k];
        }
    }
};

// bf16(relu(acc + bias)) of four channels starting at co, packed; zero when !inside.
__device__ __forceinline__ uint2 relu_pack4(const f32x4 &acc, const float *bias, int co, bool inside) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = inside ? fmaxf(acc[i] + bias[co + i], 0.0f) : 0.0f;
    return make_uint2((uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16),
                      (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16));
}

// ---- layer 1 (1 -> 32) on the matrix cores, fp32 operands ---------------------------------
// v_mfma_f32_16x16x4f32: M = 16 output channels, N = 16 pixels, K = 4 taps; the 9 taps in
// three steps (taps 9..11 weigh zero). Lane (q = l / 16, l16 = l % 16) holds
// A[l16][q] = W1[4i + q][h * 16 + l16] and B[q][l16] = x of pixel l16 shifted by tap 4i + q;
// D gives lane l the channels h * 16 + 4q .. + 4 of pixel l16. Z1 = bias + that sum.
struct Layer1W {
    float w[3][2];
    __device__ __forceinline__ void load(const float *__restrict__ w1r) {
        const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) w[i][h] = 4 * i + q < 9 ? w1r[(4 * i + q) * C + h * 16 + l16] : 0.0f;
    }
};

// Layer-1 sums (bias not added) over an R x R pixel region (row-major index j) whose input
// is the (R + 2) x (R + 2) fp32 LDS region s_x: store(j, acc0, acc1) gets channels
// 4q .. + 4 (acc0) and 16 + 4q .. + 4 (acc1) of pixel j, for every j of the 16-pixel blocks
// (j >= R * R included: the store skips them).
template <int R, typename Store>
__device__ __forceinline__ void conv1_region(const float *s_x, const Layer1W &wa, Store store) {
    constexpr int NPX = R * R, NB = (NPX + 15) / 16, SI = R + 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, q = lane >> 4;
    for (int blk = wv; blk < NB; blk += 4) {
        const int j = blk * 16 + l16, c = j < NPX ? j : NPX - 1;
        const float *px = s_x + (c / R) * SI + c % R;
        f32x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int t = 4 * i + q, tt = t < 9 ? t : 8;
            const float xb = t < 9 ? px[(tt / 3) * SI + tt % 3] : 0.0f;
            a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.w[i][0], xb, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa.w[i][1], xb, a1, 0, 0, 0);
        }
        store(j, a0, a1);
    }
}

// ---- layer 6 (32 -> 1) on the matrix cores --------------------------------------------------
// A rows = the 9 taps (rows 9..15 zero), K = the 32 channels, N = 16 pixels of the A5 region:
// C[t][p] = sum_ci W6[t][ci] A5[p][ci] is what region pixel p adds to the output pixel
// p - off_t, so one MFMA per 16 region pixels gives the terms of all nine taps. The output:
// y = x + (b6 + C[0][p + off_0] + ... + C[8][p + off_8]), the terms added in tap order.
struct Layer6W {
    bf16x8 w;
    __device__ __forceinline__ void load(const float *__restrict__ w6r) {
        const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = (__bf16)(l16 < 9 ? w6r[l16 * C + q * 8 + e] : 0.0f);
    }
};

// Tap terms of every pixel of an S x S region (row-major, LDS stride CP, zero outside the
// image) into s_c[t * S * S + j].
template <int S>
__device__ __forceinline__ void conv6_taps(const uint16_t *s_in, const Layer6W &wa, float *s_c) {
    constexpr int NPX = S * S, NB = (NPX + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, q = lane >> 4;
    for (int blk = wv; blk < NB; blk += 4) {
        const int j = blk * 16 + l16, c = j < NPX ? j : NPX - 1;
        const bf16x8 xb = *(const bf16x8 *)(s_in + c * CP + q * 8);
        const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa.w, xb, f32x4{0, 0, 0, 0}, 0, 0, 0);
        if (j < NPX)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * q + r < 9) s_c[(4 * q + r) * NPX + j] = acc[r];
    }
}

// b6 plus the nine tap terms of output pixel (ty, tx), whose region pixel is (ty + 1, tx + 1).
template <int S>
__device__ __forceinline__ float conv6_sum(const float *s_c, float b6v, int ty, int tx) {
    float z = b6v;
#pragma unroll
    for (int t = 0; t < 9; ++t) z += s_c[t * S * S + (ty + t / 3) * S + tx + t % 3];
    return z;
}

// ---- layer 1: 1 -> 32 ----------------------------------------------------------------------
// Persistent over 16 x 16 tiles (blockIdx.x, + gridDim.x, ...); the next tile's input region
// is loaded while the current one is computed (two LDS buffers).
template <typename T>
__global__ __launch_bounds__(256) void conv1_fwd_kernel(const T *__restrict__ g, long long pitch,
                                                        long long img_stride, int B, int H, int W,
                                                        float mval, const float *__restrict__ w1r,
                                                        const float *__restrict__ b1,
                                                        uint16_t *__restrict__ a1, int ntx, int nty) {
    __shared__ float s_tab[sizeof(T) == 1 ? 256 : 1];  // 8-bit data: g / M for every g
    __shared__ float s_x[2][HS * HS];
    constexpr int NR = (HS * HS + 255) / 256;  // region values per thread
    const int q = (threadIdx.x & 63) >> 4;
    Layer1W wa;
    wa.load(w1r);
    float bv[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) bv[h][r] = b1[h * 16 + 4 * q + r];
    if (sizeof(T) == 1) s_tab[threadIdx.x] = (float)threadIdx.x / mval;
    const int ntiles = ntx * nty * B;
    int raw[NR];  // this thread's values of the next region, -1 outside the image
    auto fetch = [&](int t) {
        int b, y0, x0;
        tile_at(t, ntx, nty, b, y0, x0);
        const T *gb = g + (long long)b * img_stride;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            const int ly = i / HS, lx = i - ly * HS;
            const int gy = y0 + ly - 1, gx = x0 + lx - 1;
            raw[k] = (i < HS * HS && gy >= 0 && gy < H && gx >= 0 && gx < W) ? (int)gb[(long long)gy * pitch + gx]
                                                                            : -1;
        }
    };
    int t = blockIdx.x;
    if (t < ntiles) fetch(t);
    __syncthreads();  // s_tab
    for (int buf = 0; t < ntiles; t += gridDim.x, buf ^= 1) {
        float *sx = s_x[buf];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + 256 * k;
            if (i < HS * HS) sx[i] = raw[k] < 0 ? 0.0f : (sizeof(T) == 1 ? s_tab[raw[k]] : (float)raw[k] / mval);
        }
        // the region is complete, and every thread is past its reads of the other buffer
        // (the previous tile's), which the next iteration fills
        __syncthreads();
        int b, y0, x0;
        tile_at(t, ntx, nty, b, y0, x0);
        if (t + (int)gridDim.x < ntiles) fetch(t + (int)gridDim.x);
        conv1_region<TS>(sx, wa, [&](int j, const f32x4 &s0, const f32x4 &s1) {
            const int gy = y0 + j / TS, gx = x0 + j % TS;
            if (gy >= H || gx >= W) return;
            uint16_t *o = a1 + (((long long)b * H + gy) * W + gx) * C;
            *(uint2 *)(o + 4 * q) = relu_pack4(s0, bv[0], 0, true);
            *(uint2 *)(o + 16 + 4 * q) = relu_pack4(s1, bv[1], 0, true);
        });
    }
}

// ---- 32 -> 32 on the matrix cores --------------------------------------------------------
// FWD: out = bf16(relu(Z + bias)). BWD: out = bf16(Z * (mask > 0)), no bias (backward-data:
// the weights passed are W'[t][ci][co] = W[8 - t][co][ci], input = dZ of the next layer,
// mask = the activation the gradient flows into).
template <bool FWD>
__global__ __launch_bounds__(256) void conv32_mfma_kernel(const uint16_t *__restrict__ in, int B, int H, int W,
                                                          const uint16_t *__restrict__ wt,
                                                          const float *__restrict__ bias,
                                                          const uint16_t *__restrict__ mask,
                                                          uint16_t *__restrict__ out, int ntx, int nty) {
    // Persistent: each workgroup loops over 16 x 16 tiles (blockIdx.x, + gridDim.x, ...),
    // loading the layer's MFMA weight operands once, and fetches the next tile's input
    // region into registers while the MFMAs of the current one run.
    __shared__ __align__(16) uint16_t s_in[HS * HS * CP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, kq = lane >> 4;  // kq: which 8 of the 32 k-elements
    const int ntiles = ntx * nty * B;
    // weight operands for all taps and both output-channel halves (A: rows = out channels)
    bf16x8 wa[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            wa[t][h] = *(const bf16x8 *)(wt + ((t * C) + h * 16 + l16) * C + kq * 8);
    float bv[2][4];
    if constexpr (FWD) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[h][i] = bias[h * 16 + kq * 4 + i];
    }
    RegionRegs<HS, 1> nxt;
    int t = blockIdx.x, b, y0, x0;
    if (t < ntiles) {
        tile_at(t, ntx, nty, b, y0, x0);
        nxt.fetch(in, H, W, b, y0, x0);
    }
    for (; t < ntiles; t += gridDim.x) {
        nxt.put(s_in);
        __syncthreads();
        tile_at(t, ntx, nty, b, y0, x0);
        if (t + (int)gridDim.x < ntiles) {  // in flight during the MFMAs
            int nb, ny0, nx0;
            tile_at(t + (int)gridDim.x, ntx, nty, nb, ny0, nx0);
            nxt.fetch(in, H, W, nb, ny0, nx0);
        }
        for (int rr = 0; rr < TS / 4; ++rr) {
            const int row = wv * (TS / 4) + rr;  // output row in the tile
            f32x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
            for (int tp = 0; tp < 9; ++tp) {
                const int ky = tp / 3, kx = tp % 3;
                // B: column = pixel l16 of the row, k = input channels kq*8 .. +8
                const bf16x8 xb = *(const bf16x8 *)(s_in + ((row + ky) * HS + l16 + kx) * CP + kq * 8);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[tp][0], xb, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[tp][1], xb, acc1, 0, 0, 0);
            }
            const int gy = y0 + row, gx = x0 + l16;
            if (gy >= H || gx >= W) continue;
            const long long pix = ((long long)b * H + gy) * W + gx;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const f32x4 acc = h ? acc1 : acc0;
                const int co = h * 16 + kq * 4;  // 4 consecutive output channels of this pixel
                float v[4];
                if constexpr (FWD) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[i] + bv[h][i], 0.0f);
                } else {
                    const uint2 m = *(const uint2 *)(mask + pix * C + co);
                    const uint16_t mk[4] = {(uint16_t)(m.x & 0xffff), (uint16_t)(m.x >> 16),
                                            (uint16_t)(m.y & 0xffff), (uint16_t)(m.y >> 16)};
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = from_bf16(mk[i]) > 0.0f ? acc[i] : 0.0f;
                }
                const uint2 o = make_uint2((uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16),
                                           (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16));
                *(uint2 *)(out + pix * C + co) = o;
            }
        }
        __syncthreads();  // every wave is done with s_in before the next tile is put
    }
}

// The MFMA A operands of one 32 -> 32 layer (rows = output channels), all taps.
struct LayerW {
    bf16x8 w[9][2];
    __device__ __forceinline__ void load(const uint16_t *__restrict__ wt) {
        const int lane = threadIdx.x & 63, l16 = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) w[t][h] = *(const bf16x8 *)(wt + ((t * C) + h * 16 + l16) * C + kq * 8);
    }
};

// ---- inference: the whole network in one row-streaming launch ----------------------------
// A workgroup owns NS_W output columns x NS_H output rows of one image and sweeps down its
// rows. Each step computes one row of every layer, layer l two rows behind layer l - 1
// (x: row s, A_l: row s - 2l, the tap terms C: row s - 11, y: row s - 13), from four-row
// LDS rings of the previous layer's rows: a step reads three rows of each ring while the
// new row goes into the fourth slot, so one barrier per step separates the writes from the
// next step's reads. The x ring keeps 16 rows (the output adds x of its own row, 13 rows
// back), and the input is loaded NS_XAHEAD rows ahead of its use, so that no step waits on
// global memory. A ring row covers the columns the next layer needs (A_l:
// [-(6 - l), NS_W + 6 - l) around the strip) and holds zeros outside the image, which is
// the next layer's zero padding. Wave w keeps the weights of the 32 -> 32 layer w + 2 in
// registers and computes that layer's row, two 16-pixel blocks at a time; layer 1's blocks
// and the tap-term blocks are shared out over the waves, and wave 3 also adds up the output
// row. No activation leaves the chip: per pixel the launch reads the input and writes y.
// Every per-pixel operation is the per-layer kernels' own, so the output is bit-identical
// to theirs.
constexpr int NS_W = 48;                // output columns of a strip
constexpr int NS_H = 48;                // output rows of a workgroup
constexpr int NS_XW = NS_W + 12;        // x ring row: columns [-6, NS_W + 6)
constexpr int NS_CW = NS_W + 2;         // tap-term row: columns [-1, NS_W + 1)
constexpr int NS_NB = 4;                // 16-pixel blocks of every ring row
constexpr int NS_XROWS = 16;            // rows of the x ring
constexpr int NS_XAHEAD = 4;            // input rows in flight ahead of their use
__host__ __device__ constexpr int ns_width(int l) { return NS_W + 2 * (6 - l); }  // A_l ring row
// A_l ring: 4 rows of ns_rowpx(l) pixels (64 bytes each; the row padded to a multiple of 4
// pixels, so that every row starts at a multiple of 4 pixels)
__host__ __device__ constexpr int ns_rowpx(int l) { return (ns_width(l) + 3) & ~3; }
__host__ __device__ constexpr int ns_ring_px(int l) { return 4 * ns_rowpx(l); }
__host__ __device__ constexpr int ns_base_px(int l) {
    int b = 0;
    for (int i = 1; i < l; ++i) b += ns_ring_px(i);
    return b;
}
constexpr int NS_ACT_PX = ns_base_px(6);
static_assert(ns_width(1) <= 16 * NS_NB && NS_CW > 16 * (NS_NB - 1), "every ring row is four blocks");
__device__ __forceinline__ int ns_slot(int r) { return (r + 12) & 3; }  // ring slot of row r >= -12
__device__ __forceinline__ int ns_xslot(int r) { return (r + 16) & (NS_XROWS - 1); }  // x ring, r >= -16
// Element offset, within its ring row, of the 16-byte chunk c (channels 8c .. 8c + 7) of
// column j: the chunks of a pixel are rotated by (j >> 2) & 3, so that the same chunk of 16
// consecutive columns falls in 16 different 16-byte bank groups (at a bare 64-byte pixel
// stride every fourth pixel shares one; rows start at multiples of 4 pixels).
__device__ __forceinline__ int ns_off(int j, int c) { return j * C + ((c ^ ((j >> 2) & 3)) << 3); }
// element offset of ring row r of layer l
__device__ __forceinline__ int ns_row(int l, int r) { return (ns_base_px(l) + ns_slot(r) * ns_rowpx(l)) * C; }

struct NetPtrs {
    const float *w1r, *b1;
    const uint16_t *wf[4];  // layers 2..5, forward layout
    const float *bias[4];   // layers 2..5
    const float *w6r, *b6;
};

template <typename T>
__global__ __launch_bounds__(256) void network_stream_kernel(const T *__restrict__ g, long long pitch,
                                                             long long img_stride, int H, int W, float mval,
                                                             NetPtrs P, float *__restrict__ y, long long y_pitch,
                                                             long long y_img_stride) {
    __shared__ __align__(16) uint16_t s_act[NS_ACT_PX * C];
    __shared__ float s_x[NS_XROWS * NS_XW];
    __shared__ float s_c[4 * 9 * NS_CW];
    const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wave-uniform
    const int b = blockIdx.z, x0 = blockIdx.x * NS_W, Y0 = blockIdx.y * NS_H;
    const int L = wv + 2;  // this wave's 32 -> 32 layer
    const int wL = ns_width(L);
    // per-lane LDS offsets within a ring row: this wave's layer reads (block pair p, tap
    // column kx), its writes (block, channel half), layer 1's and the tap terms' block wv
    int rd0[NS_NB / 2][3], rd1[NS_NB / 2][3], wr[NS_NB][2];
#pragma unroll
    for (int p = 0; p < NS_NB / 2; ++p) {
        const int j0 = 32 * p + l16, j1 = j0 + 16;
        const int c0 = j0 < wL ? j0 : wL - 1, c1 = j1 < wL ? j1 : wL - 1;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            rd0[p][kx] = ns_off(c0 + kx, q);
            rd1[p][kx] = ns_off(c1 + kx, q);
        }
    }
#pragma unroll
    for (int blk = 0; blk < NS_NB; ++blk)
#pragma unroll
        for (int h = 0; h < 2; ++h) wr[blk][h] = ns_off(16 * blk + l16, 2 * h + (q >> 1)) + (q & 1) * 4;
    const int jw = wv * 16 + l16;  // layer 1's and the tap terms' column
    const int wr1[2] = {wr[wv][0], wr[wv][1]};
    const int rdc = ns_off(jw < NS_CW ? jw : NS_CW - 1, q);
    LayerW wl;
    wl.load(P.wf[wv]);
    float bl[2][4], b1v[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bl[h][r] = P.bias[wv][h * 16 + 4 * q + r];
            b1v[h][r] = P.b1[h * 16 + 4 * q + r];
        }
    Layer1W w1;
    w1.load(P.w1r);
    Layer6W w6;
    w6.load(P.w6r);
    const float b6v = P.b6[0];
    const T *gb = g + (long long)b * img_stride;
    // raw input of row r, column threadIdx.x - 6 (threads < NS_XW; -1 outside the image),
    // loaded NS_XAHEAD steps ahead of its conversion and store
    const int xend = Y0 + NS_H + 6;  // x rows [Y0 - 6, xend)
    auto load_x = [&](int r) -> int {
        const int gx = x0 - 6 + (int)threadIdx.x;
        return (threadIdx.x < NS_XW && r >= 0 && r < H && r < xend && gx >= 0 && gx < W)
                   ? (int)gb[(long long)r * pitch + gx]
                   : -1;
    };
    int rx[NS_XAHEAD];
#pragma unroll
    for (int k = 0; k < NS_XAHEAD; ++k) rx[k] = load_x(Y0 - 6 + k);
    for (int s = Y0 - 6; s <= Y0 + NS_H + 12; ++s) {
        const int q1 = s - 2, qL = s - 2 * L, qc = s - 11, qy = s - 13;
        // x row s
        if (s < xend) {
            if (threadIdx.x < NS_XW)
                s_x[ns_xslot(s) * NS_XW + threadIdx.x] =
                    rx[0] < 0 ? 0.0f : (float)rx[0] / mval;  // as the per-layer kernel (and its 8-bit table)
#pragma unroll
            for (int k = 0; k + 1 < NS_XAHEAD; ++k) rx[k] = rx[k + 1];
            rx[NS_XAHEAD - 1] = load_x(s + NS_XAHEAD);
        }
        // layer 1 row q1: block wv
        if (q1 >= Y0 - 5 && q1 < Y0 + NS_H + 5) {
            const bool row_in = q1 >= 0 && q1 < H;
            const int j = wv * 16 + l16, jc = j < ns_width(1) ? j : ns_width(1) - 1;
            f32x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
            if (row_in) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int t = 4 * i + q, tt = t < 9 ? t : 8;
                    const float xb = t < 9 ? s_x[ns_xslot(q1 - 1 + tt / 3) * NS_XW + jc + tt % 3] : 0.0f;
                    a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(w1.w[i][0], xb, a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(w1.w[i][1], xb, a1, 0, 0, 0);
                }
            }
            const int gx = x0 - 5 + j;
            const bool inside = row_in && gx >= 0 && gx < W;
            if (j < ns_width(1)) {
                uint16_t *row = s_act + ns_row(1, q1);
                *(uint2 *)(row + wr1[0]) = relu_pack4(a0, b1v[0], 0, inside);
                *(uint2 *)(row + wr1[1]) = relu_pack4(a1, b1v[1], 0, inside);
            }
        }
        // this wave's layer L, row qL: blocks (0, 1) then (2, 3)
        if (qL >= Y0 - (6 - L) && qL < Y0 + NS_H + (6 - L)) {
            const bool row_in = qL >= 0 && qL < H;
            const uint16_t *rin[3] = {s_act + ns_row(L - 1, qL - 1), s_act + ns_row(L - 1, qL),
                                      s_act + ns_row(L - 1, qL + 1)};
            uint16_t *rout = s_act + ns_row(L, qL);
#pragma unroll
            for (int pb = 0; pb < NS_NB; pb += 2) {
                const int j0 = pb * 16 + l16, j1 = j0 + 16;
                f32x4 a00 = {0, 0, 0, 0}, a01 = {0, 0, 0, 0}, a10 = {0, 0, 0, 0}, a11 = {0, 0, 0, 0};
                if (row_in) {
                    // all 18 operand reads first (in flight together), then the MFMAs
                    bf16x8 xa[9], xc[9];
#pragma unroll
                    for (int t = 0; t < 9; ++t) {
                        xa[t] = *(const bf16x8 *)(rin[t / 3] + rd0[pb / 2][t % 3]);
                        xc[t] = *(const bf16x8 *)(rin[t / 3] + rd1[pb / 2][t % 3]);
                    }
                    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs
#pragma unroll
                    for (int t = 0; t < 9; ++t) {
                        a00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl.w[t][0], xa[t], a00, 0, 0, 0);
                        a01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl.w[t][1], xa[t], a01, 0, 0, 0);
                        a10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl.w[t][0], xc[t], a10, 0, 0, 0);
                        a11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl.w[t][1], xc[t], a11, 0, 0, 0);
                    }
                }
                const int gx0 = x0 - (6 - L) + j0, gx1 = gx0 + 16;
                const bool in0 = row_in && gx0 >= 0 && gx0 < W, in1 = row_in && gx1 >= 0 && gx1 < W;
                if (j0 < wL) {
                    *(uint2 *)(rout + wr[pb][0]) = relu_pack4(a00, bl[0], 0, in0);
                    *(uint2 *)(rout + wr[pb][1]) = relu_pack4(a01, bl[1], 0, in0);
                }
                if (j1 < wL) {
                    *(uint2 *)(rout + wr[pb + 1][0]) = relu_pack4(a10, bl[0], 0, in1);
                    *(uint2 *)(rout + wr[pb + 1][1]) = relu_pack4(a11, bl[1], 0, in1);
                }
            }
        }
        // tap terms of A5 row qc: block wv
        if (qc >= Y0 - 1 && qc < Y0 + NS_H + 1) {
            const int j = jw;
            const bf16x8 xb = *(const bf16x8 *)(s_act + ns_row(5, qc) + rdc);
            const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w6.w, xb, f32x4{0, 0, 0, 0}, 0, 0, 0);
            if (j < NS_CW)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (4 * q + r < 9) s_c[(ns_slot(qc) * 9 + 4 * q + r) * NS_CW + j] = acc[r];
        }
        // output row qy
        if (wv == 3 && qy >= Y0 && qy < Y0 + NS_H && qy < H && lane < NS_W) {
            const int gx = x0 + lane;
            if (gx < W) {
                float z = b6v;
#pragma unroll
                for (int t = 0; t < 9; ++t) z += s_c[(ns_slot(qy - 1 + t / 3) * 9 + t) * NS_CW + lane + t % 3];
                // x of the output pixel: the ring's value is g / M as the per-layer kernel
                // computes it
                const float xv = s_x[ns_xslot(qy) * NS_XW + lane + 6];
                y[(long long)b * y_img_stride + (long long)qy * y_pitch + gx] = xv + z;
            }
        }
        lds_barrier();
    }
}

// ---- layer 6: 32 -> 1, residual output, fused loss gradient --------------------------------
template <typename T>
__global__ __launch_bounds__(256) void conv6_fwd_kernel(const uint16_t *__restrict__ a5, const T *__restrict__ g,
                                                        long long pitch, long long img_stride, int B, int H,
                                                        int W, float mval, const float *__restrict__ w6r,
                                                        const float *__restrict__ b6, float *__restrict__ y,
                                                        long long y_pitch, long long y_img_stride,
                                                        const float *__restrict__ target,
                                                        float *__restrict__ dy,
                                                        double *__restrict__ loss_partials) {
    __shared__ float sw[9 * C];
    __shared__ double s_red[4];
    for (int i = threadIdx.x; i < 9 * C; i += 256) sw[i] = w6r[i];
    __syncthreads();
    const long long npx = (long long)B * H * W;
    // grid: (column blocks, rows, images)
    const int x = blockIdx.x * 256 + threadIdx.x, yy0 = blockIdx.y, b = blockIdx.z;
    const long long p = ((long long)b * H + yy0) * W + x;
    double l2 = 0.0;
    if (x < W) {
        float z = b6[0];
        for (int t = 0; t < 9; ++t) {
            const int yy = yy0 + t / 3 - 1, xx = x + t % 3 - 1;
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const uint4 *src = (const uint4 *)(a5 + (((long long)b * H + yy) * W + xx) * C);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = src[q];
                const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    z = fmaf(from_bf16((uint16_t)(wd[k] & 0xffff)), sw[t * C + q * 8 + 2 * k], z);
                    z = fmaf(from_bf16((uint16_t)(wd[k] >> 16)), sw[t * C + q * 8 + 2 * k + 1], z);
                }
            }
        }
        const float xv = (float)g[(long long)b * img_stride + (long long)yy0 * pitch + x] / mval;
        const float yv = xv + z;
        y[(long long)b * y_img_stride + (long long)yy0 * y_pitch + x] = yv;
        if (target) {
            const float d = yv - target[p];
            dy[p] = 2.0f * d / (float)npx;
            l2 = (double)d * (double)d;
        }
    }
    if (!target) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l2 += __shfl_down(l2, off, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = l2;
    __syncthreads();
    if (threadIdx.x == 0)
        loss_partials[blockIdx.x + gridDim.x * ((long long)blockIdx.y + gridDim.y * (long long)blockIdx.z)] =
            s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

// Inference form of layer 6 (no loss): persistent over 16 x 16 tiles, the A5 region of the
// next tile loaded into registers while the current one is computed; the tap terms on the
// matrix cores (conv6_taps), then one thread per output pixel.
template <typename T>
__global__ __launch_bounds__(256) void conv6_infer_kernel(const uint16_t *__restrict__ a5, const T *__restrict__ g,
                                                          long long pitch, long long img_stride, int B, int H,
                                                          int W, float mval, const float *__restrict__ w6r,
                                                          const float *__restrict__ b6, float *__restrict__ y,
                                                          long long y_pitch, long long y_img_stride, int ntx,
                                                          int nty) {
    __shared__ __align__(16) uint16_t s_in[HS * HS * CP];
    __shared__ float s_c[9 * HS * HS];
    const int ntiles = ntx * nty * B;
    const int ty = threadIdx.x / TS, tx = threadIdx.x % TS;
    const float b6v = b6[0];
    Layer6W w6;
    w6.load(w6r);
    RegionRegs<HS, 1> nxt;
    int t = blockIdx.x, b, y0, x0;
    if (t < ntiles) {
        tile_at(t, ntx, nty, b, y0, x0);
        nxt.fetch(a5, H, W, b, y0, x0);
    }
    for (; t < ntiles; t += gridDim.x) {
        nxt.put(s_in);  // the previous tile's readers of s_in passed the barrier below
        __syncthreads();
        tile_at(t, ntx, nty, b, y0, x0);
        if (t + (int)gridDim.x < ntiles) {
            int nb, ny0, nx0;
            tile_at(t + (int)gridDim.x, ntx, nty, nb, ny0, nx0);
            nxt.fetch(a5, H, W, nb, ny0, nx0);
        }
        conv6_taps<HS>(s_in, w6, s_c);
        __syncthreads();
        const int gy = y0 + ty, gx = x0 + tx;
        if (gy < H && gx < W) {
            const float xv = (float)g[(long long)b * img_stride + (long long)gy * pitch + gx] / mval;
            y[(long long)b * y_img_stride + (long long)gy * y_pitch + gx] = xv + conv6_sum<HS>(s_c, b6v, ty, tx);
        }
    }
}

// Layer 6 backward over one 16 x 16 tile: dZ5 = bf16((sum_t dY[q - off_t] W6[t][ci]) *
// (A5[q][ci] > 0)), and the tile's partial dW6[t][ci] = sum_p dY[p] A5[p + off_t][ci],
// db6 = sum_p dY[p].
__global__ __launch_bounds__(256) void conv6_bwd_kernel(const float *__restrict__ dy, const uint16_t *__restrict__ a5,
                                                        int B, int H, int W, const float *__restrict__ w6r,
                                                        uint16_t *__restrict__ dz5, float *__restrict__ partials) {
    __shared__ __align__(16) uint16_t s_a[HS * HS * CP];
    __shared__ float s_dy[HS * HS];
    __shared__ float sw[9 * C];
    const int x0 = blockIdx.x * TS, y0 = blockIdx.y * TS, b = blockIdx.z;
    for (int i = threadIdx.x; i < 9 * C; i += 256) sw[i] = w6r[i];
    stage_act(s_a, a5, H, W, b, y0, x0);
    for (int i = threadIdx.x; i < HS * HS; i += 256) {
        const int ly = i / HS, lx = i - ly * HS, gy = y0 + ly - 1, gx = x0 + lx - 1;
        s_dy[i] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? dy[((long long)b * H + gy) * W + gx] : 0.0f;
    }
    __syncthreads();
    {
        const int ly = threadIdx.x / TS, lx = threadIdx.x % TS;
        const int gy = y0 + ly, gx = x0 + lx;
        if (gy < H && gx < W) {
            uint32_t packed[C / 2];
#pragma unroll
            for (int ci = 0; ci < C; ci += 2) {
                float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    // q - off_t: the output pixel whose window reads q through tap t
                    const float dv = s_dy[(ly + 1 - (t / 3 - 1)) * HS + (lx + 1 - (t % 3 - 1))];
                    d0 = fmaf(dv, sw[t * C + ci], d0);
                    d1 = fmaf(dv, sw[t * C + ci + 1], d1);
                }
                const uint16_t *ac = s_a + ((ly + 1) * HS + lx + 1) * CP;
                d0 = from_bf16(ac[ci]) > 0.0f ? d0 : 0.0f;
                d1 = from_bf16(ac[ci + 1]) > 0.0f ? d1 : 0.0f;
                packed[ci / 2] = (uint32_t)to_bf16(d0) | ((uint32_t)to_bf16(d1) << 16);
            }
            uint4 *dst = (uint4 *)(dz5 + (((long long)b * H + gy) * W + gx) * C);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dst[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
        }
    }
    // partial weight gradient of this tile: thread j handles (t, ci) = j and j + 256
    const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    for (int j = threadIdx.x; j < 9 * C + 1; j += 256) {
        float acc = 0.0f;
        if (j < 9 * C) {
            const int t = j / C, ci = j % C, ky = t / 3, kx = t % 3;
            for (int ly = 0; ly < TS; ++ly)
                for (int lx = 0; lx < TS; ++lx)
                    acc = fmaf(s_dy[(ly + 1) * HS + lx + 1], from_bf16(s_a[((ly + ky) * HS + lx + kx) * CP + ci]), acc);
        } else {
            for (int i = 0; i < TS * TS; ++i) acc += s_dy[(i / TS + 1) * HS + i % TS + 1];
        }
        partials[blk * (9 * C + 1) + j] = acc;
    }
}

// Partial weight / bias gradient of a 32 -> 32 layer over the tiles this workgroup owns
// (tiles blockIdx.x, + gridDim.x, ...): wave w accumulates taps w, w + 4, w + 8 on the
// matrix cores, M = 16 out channels, N = 16 in channels, K = 32 pixels (the 8 pixels of
// k-group q: tile row 2s + q / 2, columns (q & 1) * 8 .. + 8). Both operands are staged
// channel-major so that every operand is one 16-byte LDS read: dZ as [channel][pixel], and
// the input region as three copies [kx][channel][row * 16 + col] = A[row][col + kx], one
// per horizontal tap offset (rows padded by 8 elements, which spreads 16 consecutive
// channels over all banks).
constexpr int WG_DZS = TS * TS + 8;  // dZ row (one channel) in elements
constexpr int WG_AS = HS * TS + 8;   // input copy row (one channel) in elements
__global__ __launch_bounds__(256) void conv32_wgrad_kernel(const uint16_t *__restrict__ dz,
                                                           const uint16_t *__restrict__ a_prev, int B,
                                                           int H, int W, int ntx, int nty,
                                                           float *__restrict__ partials) {
    __shared__ __align__(16) uint16_t s_a[3 * C * WG_AS];
    __shared__ __align__(16) uint16_t s_dz[C * WG_DZS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l16 = lane & 15, kq = lane >> 4;
    constexpr int NTW = 3;  // taps per wave (wave 0: 0,4,8; wave 1: 1,5; ...)
    f32x4 acc[NTW][2][2];
#pragma unroll
    for (int i = 0; i < NTW; ++i)
#pragma unroll
        for (int hc = 0; hc < 2; ++hc)
#pragma unroll
            for (int hi = 0; hi < 2; ++hi) acc[i][hc][hi] = f32x4{0, 0, 0, 0};
    float bacc = 0.0f;  // bias gradient: thread co < 32
    const int ntiles = ntx * nty * B;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int b, y0, x0;
        tile_at(tile, ntx, nty, b, y0, x0);
        __syncthreads();  // previous tile's operands are consumed
        for (int i = threadIdx.x; i < HS * HS * 4; i += 256) {
            const int px = i >> 2, part = i & 3;
            const int ly = px / HS, lx = px - ly * HS;
            const int gy = y0 + ly - 1, gx = x0 + lx - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gy >= 0 && gy < H && gx >= 0 && gx < W)
                v = *(const uint4 *)(a_prev + (((long long)b * H + gy) * W + gx) * C + part * 8);
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int c = lx - kx;
                if (c < 0 || c >= TS) continue;
                uint16_t *dst = s_a + (kx * C + part * 8) * WG_AS + ly * TS + c;
#pragma unroll
                for (int j = 0; j < 8; ++j) dst[j * WG_AS] = (uint16_t)(wd[j >> 1] >> (16 * (j & 1)));
            }
        }
        for (int i = threadIdx.x; i < TS * TS * 4; i += 256) {
            const int px = i >> 2, part = i & 3;
            const int gy = y0 + px / TS, gx = x0 + px % TS;
            uint4 v = make_uint4(0, 0, 0, 0);  // pixels outside the image contribute nothing
            if (gy < H && gx < W) v = *(const uint4 *)(dz + (((long long)b * H + gy) * W + gx) * C + part * 8);
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
            uint16_t *dst = s_dz + part * 8 * WG_DZS + px;
#pragma unroll
            for (int j = 0; j < 8; ++j) dst[j * WG_DZS] = (uint16_t)(wd[j >> 1] >> (16 * (j & 1)));
        }
        __syncthreads();
        if (threadIdx.x < C)
            for (int i = 0; i < TS * TS; ++i) bacc += from_bf16(s_dz[threadIdx.x * WG_DZS + i]);
        for (int s = 0; s < TS * TS / 32; ++s) {
            const int row = 2 * s + (kq >> 1), col0 = (kq & 1) * 8;
            bf16x8 da[2];
#pragma unroll
            for (int hc = 0; hc < 2; ++hc)
                da[hc] = *(const bf16x8 *)(s_dz + (hc * 16 + l16) * WG_DZS + row * TS + col0);
#pragma unroll
            for (int i = 0; i < NTW; ++i) {
                const int t = wv + 4 * i;
                if (t >= 9) break;
                const int ky = t / 3, kx = t % 3;
#pragma unroll
                for (int hi = 0; hi < 2; ++hi) {
                    const bf16x8 xb = *(const bf16x8 *)(s_a + (kx * C + hi * 16 + l16) * WG_AS + (row + ky) * TS + col0);
#pragma unroll
                    for (int hc = 0; hc < 2; ++hc)
                        acc[i][hc][hi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(da[hc], xb, acc[i][hc][hi], 0, 0, 0);
                }
            }
        }
    }
    // partials[block][t][co][ci] then [block][9 * 1024 + co] for the bias
    float *dst = partials + (long long)blockIdx.x * (9 * C * C + C);
#pragma unroll
    for (int i = 0; i < NTW; ++i) {
        const int t = wv + 4 * i;
        if (t >= 9) break;
#pragma unroll
        for (int hc = 0; hc < 2; ++hc)
#pragma unroll
            for (int hi = 0; hi < 2; ++hi)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = hc * 16 + kq * 4 + e, ci = hi * 16 + l16;
                    dst[(t * C + co) * C + ci] = acc[i][hc][hi][e];
                }
    }
    if (threadIdx.x < C) dst[9 * C * C + threadIdx.x] = bacc;
}

// Partial gradient of layer 1 over the owned tiles: dW1[t][co] = sum_p dZ1[p][co] x[p + off_t],
// db1[co] = sum_p dZ1[p][co]; thread j handles entries j and j + 256 of the 320.
template <typename T>
__global__ __launch_bounds__(256) void conv1_wgrad_kernel(const uint16_t *__restrict__ dz, const T *__restrict__ g,
                                                          long long pitch, long long img_stride, int B, int H,
                                                          int W, float mval, int ntx, int nty,
                                                          float *__restrict__ partials) {
    __shared__ __align__(16) uint16_t s_dz[TS * TS * CP];
    __shared__ float s_x[HS * HS];
    float acc[2] = {0.0f, 0.0f};
    const int ntiles = ntx * nty * B;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tx = tile % ntx, ty = (tile / ntx) % nty, b = tile / (ntx * nty);
        const int x0 = tx * TS, y0 = ty * TS;
        __syncthreads();
        for (int i = threadIdx.x; i < TS * TS * 4; i += 256) {
            const int px = i >> 2, part = i & 3;
            const int gy = y0 + px / TS, gx = x0 + px % TS;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gy < H && gx < W) v = *(const uint4 *)(dz + (((long long)b * H + gy) * W + gx) * C + part * 8);
            *(uint4 *)(s_dz + px * CP + part * 8) = v;
        }
        for (int i = threadIdx.x; i < HS * HS; i += 256) {
            const int ly = i / HS, lx = i - ly * HS, gy = y0 + ly - 1, gx = x0 + lx - 1;
            s_x[i] = (gy >= 0 && gy < H && gx >= 0 && gx < W)
                         ? (float)g[(long long)b * img_stride + (long long)gy * pitch + gx] / mval
                         : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int j = threadIdx.x + 256 * k;
            if (j >= 9 * C + C) break;
            float a = 0.0f;
            if (j < 9 * C) {
                const int t = j / C, co = j % C, ky = t / 3, kx = t % 3;
                for (int i = 0; i < TS * TS; ++i)
                    a = fmaf(from_bf16(s_dz[i * CP + co]), s_x[(i / TS + ky) * HS + i % TS + kx], a);
            } else {
                for (int i = 0; i < TS * TS; ++i) a += from_bf16(s_dz[i * CP + (j - 9 * C)]);
            }
            acc[k] += a;
        }
    }
    float *dst = partials + (long long)blockIdx.x * (9 * C + C);
    for (int k = 0; k < 2; ++k) {
        const int j = threadIdx.x + 256 * k;
        if (j < 9 * C + C) dst[j] = acc[k];
    }
}

// grad[off + j] = sum over blocks of partials[block][j] in double, in a fixed order: chunk c
// (blocks c * per .. c * per + per - 1, in block order) into red[c][j], then the chunks in
// order. Both stages spread over many workgroups (one thread per entry and chunk).
__global__ void reduce_partials_chunk_kernel(const float *__restrict__ partials, int nblocks, int n, int per,
                                             double *__restrict__ red) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
    if (j >= n) return;
    const int b0 = c * per, b1 = min(nblocks, b0 + per);
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += (double)partials[(long long)b * n + j];
    red[(long long)c * n + j] = s;
}
__global__ void reduce_chunks_kernel(const double *__restrict__ red, int chunks, int n, float *__restrict__ grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += red[(long long)c * n + j];
    grad[j] = (float)s;
}

__global__ void reduce_loss_kernel(const double *__restrict__ partials, int n, long long npx,
                                   float *__restrict__ loss) {
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += partials[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s[0] / (double)npx);
}

// Adam on the fp32 master parameters, then the layer copies: W1 / W6 rounded to bf16
// values (kept as fp32 for the vector kernels), W2..W5 as bf16 in the forward layout
// [t][co][ci] and the backward-data layout [t][ci][co] with the tap mirrored (8 - t).
__global__ void adam_prep_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                 const float *__restrict__ grad, int step, float lr, float b1, float b2,
                                 float eps, Weights wt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N_PARAMS) return;
    float wj = w[j];
    if (grad) {
        const float gj = grad[j];
        const float mj = b1 * m[j] + (1.0f - b1) * gj;
        const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
        m[j] = mj;
        v[j] = vj;
        const float mh = mj / (1.0f - powf(b1, (float)step));
        const float vh = vj / (1.0f - powf(b2, (float)step));
        wj -= lr * mh / (sqrtf(vh) + eps);
        w[j] = wj;
    }
    const uint16_t hb = to_bf16(wj);
    if (j < OFF_B1) {
        wt.w1r[j] = from_bf16(hb);
    } else if (j >= OFF_W6 && j < OFF_B6) {
        wt.w6r[j - OFF_W6] = from_bf16(hb);
    } else {
        for (int l = 0; l < 4; ++l) {
            const int o = OFF_W2 + l * (9 * C * C + C);
            if (j >= o && j < o + 9 * C * C) {
                const int k = j - o, t = k / (C * C), co = (k / C) % C, ci = k % C;
                wt.wf[l][k] = hb;
                wt.wb[l][((8 - t) * C + ci) * C + co] = hb;
            }
        }
    }
}

// ---- per-tile check ------------------------------------------------------------------------
// One workgroup per 64 x 64 check tile of a slice: impulse fraction (pixels at 0 or M), the
// mean squared residual (x - y)^2 over the other pixels and, with a proxy of the plain
// output (proxies != null: dense float32 images, one per slice), the mean squared
// deviation (y - proxy)^2 over all pixels; score = max(frac / p_max, res / r_hi,
// r_lo / res, dev / d_hi2) (infinite when res == 0). Failing tiles (score >= threshold)
// append the stage tiles (64 x 32) they cover to the fallback list.
template <typename T>
__global__ __launch_bounds__(256) void tile_check_kernel(SliceSet set, int n_check_x_total,
                                                         const int *__restrict__ check_begin,
                                                         float mval, float p_max, float r_lo, float r_hi,
                                                         const float *const *__restrict__ proxies, float d_hi2,
                                                         float threshold, float *__restrict__ scores,
                                                         int *__restrict__ flags, int *__restrict__ list,
                                                         int *__restrict__ count) {
    __shared__ float s_imp[4], s_res[4], s_cnt[4], s_dev[4];
    const int ct = blockIdx.x;  // global check-tile index
    int si = 0;
    if (set.n > 1) {
        int lo = 0, hi = set.n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (check_begin[mid] <= ct) lo = mid;
            else hi = mid - 1;
        }
        si = lo;
    }
    const SliceDesc sd = slice_desc(set, si);
    const int lct = ct - (set.n > 1 ? check_begin[si] : 0);
    const int ncx = (sd.w + 63) / 64;
    const int cy = lct / ncx, cx = lct % ncx;
    const T *gimg = (const T *)sd.in;
    const float *prox = proxies ? proxies[si] : nullptr;
    float imp = 0.0f, res = 0.0f, cnt = 0.0f, dev = 0.0f;
    for (int i = threadIdx.x; i < 64 * 64; i += 256) {
        const int yy = cy * 64 + i / 64, xx = cx * 64 + i % 64;
        if (yy >= sd.h || xx >= sd.w) continue;
        const float gv = (float)gimg[(long long)yy * sd.in_pitch + xx];
        const float yv = sd.out[(long long)yy * sd.out_pitch + xx];
        cnt += 1.0f;
        if (gv == 0.0f || gv == mval) {
            imp += 1.0f;
        } else {
            const float d = gv / mval - yv;
            res += d * d;
        }
        if (prox) {
            const float e = yv - prox[(long long)yy * sd.w + xx];
            dev += e * e;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        imp += __shfl_down(imp, off, 64);
        res += __shfl_down(res, off, 64);
        cnt += __shfl_down(cnt, off, 64);
        dev += __shfl_down(dev, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_imp[threadIdx.x >> 6] = imp;
        s_res[threadIdx.x >> 6] = res;
        s_cnt[threadIdx.x >> 6] = cnt;
        s_dev[threadIdx.x >> 6] = dev;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const float ti = s_imp[0] + s_imp[1] + s_imp[2] + s_imp[3];
    const float tr = s_res[0] + s_res[1] + s_res[2] + s_res[3];
    const float tc = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    const float td = s_dev[0] + s_dev[1] + s_dev[2] + s_dev[3];
    const float frac = ti / tc;
    const float rmean = (tc > ti) ? tr / (tc - ti) : 0.0f;
    float score = fmaxf(frac / p_max, rmean / r_hi);
    score = rmean > 0.0f ? fmaxf(score, r_lo / rmean) : __builtin_huge_valf();
    if (prox) score = fmaxf(score, (td / tc) / d_hi2);
    scores[ct] = score;
    const int fail = !(score < threshold);
    // the stage tiles (64 x 32) covered by this check tile
    const int stx = sd.tiles_x;
    for (int k = 0; k < 2; ++k) {
        const int sy = cy * 2 + k;
        if (sy * TILE_Y >= sd.h) break;
        const int st = sd.tile_begin + sy * stx + cx;
        flags[st] = fail;
        if (fail) list[atomicAdd(count, 1)] = st;
    }
}

}  // namespace

// Persistent grid of a kernel: as many workgroups as the device holds at once, at
// most one per tile. The occupancy is looked up on the first launch of each kernel (one
// cache per kernel, on the device current then); the grid size affects only the speed,
// never the result.
template <auto Kernel>
static int persistent_grid(int ntiles) {
    static std::atomic<int> resident{0};
    int g = resident.load();
    if (g == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, Kernel, 256, 0) != hipSuccess || per < 1 || cus < 1) {
            (void)hipGetLastError();
            g = 1024;
        } else {
            g = cus * per;
            resident.store(g);
        }
    }
    return g < ntiles ? g : ntiles;
}

hipError_t launch_conv1_fwd(const void *g, int eb, long long pitch, long long img_stride, int B, int H, int W,
                            float mval, const float *w1r, const float *b1, uint16_t *a1, hipStream_t s) {
    const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS, ntiles = ntx * nty * B;
    if (eb == 1)
        hipLaunchKernelGGL(conv1_fwd_kernel<uint8_t>, dim3(persistent_grid<conv1_fwd_kernel<uint8_t>>(ntiles)), dim3(256),
                           0, s, (const uint8_t *)g, pitch, img_stride, B, H, W, mval, w1r, b1, a1, ntx, nty);
    else
        hipLaunchKernelGGL(conv1_fwd_kernel<uint16_t>, dim3(persistent_grid<conv1_fwd_kernel<uint16_t>>(ntiles)),
                           dim3(256), 0, s, (const uint16_t *)g, pitch, img_stride, B, H, W, mval, w1r, b1, a1,
                           ntx, nty);
    return hipGetLastError();
}

hipError_t launch_conv32(bool fwd, const uint16_t *in, int B, int H, int W, const uint16_t *wt,
                         const float *bias, const uint16_t *mask, uint16_t *out, hipStream_t s) {
    const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS;
    const int ntiles = ntx * nty * B;
    if (fwd)
        hipLaunchKernelGGL(conv32_mfma_kernel<true>, dim3(persistent_grid<conv32_mfma_kernel<true>>(ntiles)), dim3(256), 0,
                           s, in, B, H, W, wt, bias, mask, out, ntx, nty);
    else
        hipLaunchKernelGGL(conv32_mfma_kernel<false>, dim3(persistent_grid<conv32_mfma_kernel<false>>(ntiles)), dim3(256),
                           0, s, in, B, H, W, wt, bias, mask, out, ntx, nty);
    return hipGetLastError();
}

hipError_t launch_conv6_fwd(const uint16_t *a5, const void *g, int eb, long long pitch, long long img_stride,
                            int B, int H, int W, float mval, const float *w6r, const float *b6, float *y,
                            long long y_pitch, long long y_img_stride, const float *target, float *dy,
                            double *loss_partials, hipStream_t s) {
    if (!target) {
        const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS, ntiles = ntx * nty * B;
        if (eb == 1)
            hipLaunchKernelGGL(conv6_infer_kernel<uint8_t>, dim3(persistent_grid<conv6_infer_kernel<uint8_t>>(ntiles)),
                               dim3(256), 0, s, a5, (const uint8_t *)g, pitch, img_stride, B, H, W, mval, w6r, b6, y,
                               y_pitch, y_img_stride, ntx, nty);
        else
            hipLaunchKernelGGL(conv6_infer_kernel<uint16_t>, dim3(persistent_grid<conv6_infer_kernel<uint16_t>>(ntiles)),
                               dim3(256), 0, s, a5, (const uint16_t *)g, pitch, img_stride, B, H, W, mval, w6r, b6,
                               y, y_pitch, y_img_stride, ntx, nty);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((W + 255) / 256), (unsigned)H, (unsigned)B);
    if (eb == 1)
        hipLaunchKernelGGL(conv6_fwd_kernel<uint8_t>, grid, dim3(256), 0, s, a5, (const uint8_t *)g, pitch,
                           img_stride, B, H, W, mval, w6r, b6, y, y_pitch, y_img_stride, target, dy,
                           loss_partials);
    else
        hipLaunchKernelGGL(conv6_fwd_kernel<uint16_t>, grid, dim3(256), 0, s, a5, (const uint16_t *)g, pitch,
                           img_stride, B, H, W, mval, w6r, b6, y, y_pitch, y_img_stride, target, dy,
                           loss_partials);
    return hipGetLastError();
}

hipError_t launch_stream_forward(const void *g, int eb, long long pitch, long long img_stride, int B, int H, int W,
                                 float mval, const Weights &wt, const float *params, float *y, long long y_pitch,
                                 long long y_img_stride, hipStream_t s) {
    NetPtrs P;
    P.w1r = wt.w1r;
    P.b1 = params + OFF_B1;
    for (int l = 0; l < 4; ++l) {
        P.wf[l] = wt.wf[l];
        P.bias[l] = params + OFF_W2 + l * LAYER32 + 9 * C * C;
    }
    P.w6r = wt.w6r;
    P.b6 = params + OFF_B6;
    const dim3 grid((unsigned)((W + NS_W - 1) / NS_W), (unsigned)((H + NS_H - 1) / NS_H), (unsigned)B);
    if (eb == 1)
        hipLaunchKernelGGL(network_stream_kernel<uint8_t>, grid, dim3(256), 0, s, (const uint8_t *)g, pitch, img_stride,
                           H, W, mval, P, y, y_pitch, y_img_stride);
    else
        hipLaunchKernelGGL(network_stream_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t *)g, pitch,
                           img_stride, H, W, mval, P, y, y_pitch, y_img_stride);
    return hipGetLastError();
}

int conv6_bwd_blocks(int B, int H, int W) { return ((W + TS - 1) / TS) * ((H + TS - 1) / TS) * B; }

hipError_t launch_conv6_bwd(const float *dy, const uint16_t *a5, int B, int H, int W, const float *w6r,
                            uint16_t *dz5, float *partials, hipStream_t s) {
    const dim3 grid((W + TS - 1) / TS, (H + TS - 1) / TS, B);
    hipLaunchKernelGGL(conv6_bwd_kernel, grid, dim3(256), 0, s, dy, a5, B, H, W, w6r, dz5, partials);
    return hipGetLastError();
}

hipError_t launch_conv32_wgrad(const uint16_t *dz, const uint16_t *a_prev, int B, int H, int W, int nblocks,
                               float *partials, hipStream_t s) {
    const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS;
    hipLaunchKernelGGL(conv32_wgrad_kernel, dim3(nblocks), dim3(256), 0, s, dz, a_prev, B, H, W, ntx, nty,
                       partials);
    return hipGetLastError();
}

hipError_t launch_conv1_wgrad(const uint16_t *dz, const void *g, int eb, long long pitch, long long img_stride,
                              int B, int H, int W, float mval, int nblocks, float *partials, hipStream_t s) {
    const int ntx = (W + TS - 1) / TS, nty = (H + TS - 1) / TS;
    if (eb == 1)
        hipLaunchKernelGGL(conv1_wgrad_kernel<uint8_t>, dim3(nblocks), dim3(256), 0, s, dz, (const uint8_t *)g,
                           pitch, img_stride, B, H, W, mval, ntx, nty, partials);
    else
        hipLaunchKernelGGL(conv1_wgrad_kernel<uint16_t>, dim3(nblocks), dim3(256), 0, s, dz,
                           (const uint16_t *)g, pitch, img_stride, B, H, W, mval, ntx, nty, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float *partials, int nblocks, int n, float *grad, double *red,
                                  hipStream_t s) {
    const int per = (nblocks + REDUCE_CHUNKS - 1) / REDUCE_CHUNKS;
    const int chunks = (nblocks + per - 1) / per;
    hipLaunchKernelGGL(reduce_partials_chunk_kernel, dim3((n + 255) / 256, chunks), dim3(256), 0, s, partials,
                       nblocks, n, per, red);
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((n + 255) / 256), dim3(256), 0, s, red, chunks, n, grad);
    return hipGetLastError();
}

hipError_t launch_reduce_loss(const double *partials, int n, long long npx, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(reduce_loss_kernel, dim3(1), dim3(256), 0, s, partials, n, npx, loss);
    return hipGetLastError();
}

hipError_t launch_adam_prep(float *w, float *m, float *v, const float *grad, int step, float lr, float b1,
                            float b2, float eps, const Weights &wt, hipStream_t s) {
    hipLaunchKernelGGL(adam_prep_kernel, dim3((N_PARAMS + 255) / 256), dim3(256), 0, s, w, m, v, grad, step, lr,
                       b1, b2, eps, wt);
    return hipGetLastError();
}

hipError_t launch_tile_check(const SliceSet &set, int n_check, const int *check_begin, int eb, float mval,
                             float p_max, float r_lo, float r_hi, const float *const *proxies, float d_hi,
                             float threshold, float *scores, int *flags, int *list, int *count, hipStream_t s) {
    const float d_hi2 = d_hi * d_hi;
    if (eb == 1)
        hipLaunchKernelGGL(tile_check_kernel<uint8_t>, dim3(n_check), dim3(256), 0, s, set, n_check, check_begin,
                           mval, p_max, r_lo, r_hi, proxies, d_hi2, threshold, scores, flags, list, count);
    else
        hipLaunchKernelGGL(tile_check_kernel<uint16_t>, dim3(n_check), dim3(256), 0, s, set, n_check,
                           check_begin, mval, p_max, r_lo, r_hi, proxies, d_hi2, threshold, scores, flags, list,
                           count);
    return hipGetLastError();
}

}  // namespace sg
}  // namespace hd

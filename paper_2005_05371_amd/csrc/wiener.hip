// Adaptive Wiener filter (local mean / variance form) for gfx950.
//
// The hybrid de-noiser applies a Wiener filter to the AMF output (arXiv 2005.05371,
// Sec. IV and Fig. 4; Alg. 1, procedure parallelHybrid). This library uses the local
// form: for the AMF output a, over a win_h x win_w window (symmetric padding),
//   S1 = sum a, S2 = sum a^2 (exact integers), N = win_h * win_w,
//   mu = S1 / N, s2 = (N * S2 - S1^2) / N^2 (population variance),
//   nu2 = caller value, or mean of s2 over the image = sum(N * S2 - S1^2) / (N^2 * H * W),
//   out = (mu + (a - mu) * max(s2 - nu2, 0) / max(s2, nu2)) / max_value, mu when both are 0.
//
// Kernels: one 64 x 16 tile per workgroup, the tile plus its window halo staged in LDS,
// separable window sums (rows, then columns) in exact integers. The noise estimate is a
// global dependency; the partials kernel adds each block's exact integer sum into a
// 128-bit accumulator (atomic adds of integers: the result does not depend on the order),
// and the apply kernel, launched after it on the same stream, reads it.
#include "hd_internal.h"

namespace hd {
namespace {

constexpr int TX = 64;
constexpr int TY = 16;
constexpr int NT = 256;
constexpr int RPT = TY / (NT / TX);  // 4 output rows per thread
constexpr int RMAX = 7;              // largest window radius (side 15)
constexpr int LH_MAX = TY + 2 * RMAX;
constexpr int LW_MAX = TX + 2 * RMAX;

template <typename T>
struct Sq;  // square-sum type: 8-bit data fits 32 bits for any accepted window
template <>
struct Sq<uint8_t> { using type = uint32_t; };
template <>
struct Sq<uint16_t> { using type = unsigned long long; };

// Stage the tile + halo and compute, for each of the thread's RPT pixels, the window
// sums s1 (exact) and the variance numerator num = N * S2 - S1^2 (exact).
template <typename T>
struct WienerTile {
    uint32_t a[LH_MAX * LW_MAX];
    uint32_t h1[LH_MAX * TX];
    typename Sq<T>::type h2[LH_MAX * TX];
};

template <typename T>
__device__ __forceinline__ void tile_moments(WienerTile<T> &sm, const T *__restrict__ a, int H, int W,
                                             long long ap, int wh, int ww, int x0, int y0,
                                             uint32_t s1[RPT], unsigned long long num[RPT],
                                             uint32_t centre[RPT]) {
    using S2T = typename Sq<T>::type;
    const int rh = wh >> 1, rw = ww >> 1;
    const int lw = TX + 2 * rw, lh = TY + 2 * rh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int ly = wv; ly < lh; ly += NT / 64) {
        const T *src = a + (long long)mirror(y0 + ly - rh, H) * ap;
        uint32_t *dst = sm.a + ly * lw;
        for (int lx = lane; lx < lw; lx += 64) dst[lx] = src[mirror(x0 + lx - rw, W)];
    }
    __syncthreads();
    // horizontal sums over ww columns for every staged row, one column per lane
    for (int ly = wv; ly < lh; ly += NT / 64) {
        const uint32_t *row = sm.a + ly * lw + lane;
        uint32_t t1 = 0;
        S2T t2 = 0;
        for (int dx = 0; dx < ww; ++dx) {
            const uint32_t v = row[dx];
            t1 += v;
            t2 += (S2T)v * v;
        }
        sm.h1[ly * TX + lane] = t1;
        sm.h2[ly * TX + lane] = t2;
    }
    __syncthreads();
    const unsigned long long n = (unsigned long long)(wh * ww);
    const int rb = wv * RPT;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        uint32_t t1 = 0;
        unsigned long long t2 = 0;
        for (int dy = 0; dy < wh; ++dy) {
            t1 += sm.h1[(rb + j + dy) * TX + lane];
            t2 += (unsigned long long)sm.h2[(rb + j + dy) * TX + lane];
        }
        s1[j] = t1;
        num[j] = n * t2 - (unsigned long long)t1 * t1;
        centre[j] = sm.a[(rb + j + rh) * lw + lane + rw];
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <typename T>
__global__ __launch_bounds__(NT) void wiener_partials_kernel(const T *__restrict__ a, int H, int W,
                                                             long long ap, int wh, int ww,
                                                             NoiseAcc *__restrict__ acc) {
    __shared__ WienerTile<T> sm;
    __shared__ unsigned long long s_wsum[NT / 64];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    uint32_t s1[RPT], ctr[RPT];
    unsigned long long num[RPT];
    tile_moments<T>(sm, a, H, W, ap, wh, ww, x0, y0, s1, num, ctr);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long t = 0;
    const bool col_ok = (x0 + lane) < W;
#pragma unroll
    for (int j = 0; j < RPT; ++j)
        if (col_ok && (y0 + wv * RPT + j) < H) t += num[j];
    t = wave_sum_u64(t);
    if (lane == 0) s_wsum[wv] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int i = 0; i < NT / 64; ++i) b += s_wsum[i];
        if (b) {
            const unsigned long long old = atomicAdd(&acc->lo, b);
            if (old + b < old) atomicAdd(&acc->hi, 1ull);  // carry into the high word
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void wiener_apply_kernel(const T *__restrict__ a, float *__restrict__ out,
                                                          int H, int W, long long ap, long long op,
                                                          int wh, int ww, float mf,
                                                          const NoiseAcc *__restrict__ acc,
                                                          double noise_var, double *__restrict__ nu2_out) {
    __shared__ WienerTile<T> sm;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const double n = (double)(wh * ww);
    double nu2 = noise_var;
    if (acc) {
        const double total = (double)acc->hi * 18446744073709551616.0 + (double)acc->lo;
        nu2 = total / (n * n * (double)H * (double)W);
    }
    if (nu2_out && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *nu2_out = nu2;
    uint32_t s1[RPT], ctr[RPT];
    unsigned long long num[RPT];
    tile_moments<T>(sm, a, H, W, ap, wh, ww, x0, y0, s1, num, ctr);
    const float nu2f = (float)nu2;
    const float nf = (float)(wh * ww);
    const float inv_n2 = (float)(1.0 / (n * n));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool col_ok = (x0 + lane) < W;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int y = y0 + wv * RPT + j;
        if (!col_ok || y >= H) continue;
        // true divisions keep flat regions exact: S1 / N = a and a / M round once
        const float mu = (float)s1[j] / nf;
        const float var = (float)num[j] * inv_n2;
        const float den = fmaxf(var, nu2f);
        const float gain = den > 0.0f ? fmaxf(var - nu2f, 0.0f) / den : 0.0f;
        out[(long long)y * op + x0 + lane] = (mu + ((float)ctr[j] - mu) * gain) / mf;
    }
}

__global__ void zero_acc_kernel(NoiseAcc *acc, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        acc[i].lo = 0;
        acc[i].hi = 0;
    }
}

}  // namespace

hipError_t launch_zero_acc(NoiseAcc *acc, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_acc_kernel, dim3((n + 255) / 256), dim3(256), 0, s, acc, n);
    return hipGetLastError();
}

hipError_t launch_wiener_partials(const void *a, int h, int w, long long pitch, int dt_bytes,
                                  int win_h, int win_w, NoiseAcc *acc, hipStream_t s) {
    const dim3 grid((w + TX - 1) / TX, (h + TY - 1) / TY);
    if (dt_bytes == 1)
        hipLaunchKernelGGL(wiener_partials_kernel<uint8_t>, grid, dim3(NT), 0, s,
                           (const uint8_t *)a, h, w, pitch, win_h, win_w, acc);
    else
        hipLaunchKernelGGL(wiener_partials_kernel<uint16_t>, grid, dim3(NT), 0, s,
                           (const uint16_t *)a, h, w, pitch, win_h, win_w, acc);
    return hipGetLastError();
}

hipError_t launch_wiener_apply(const void *a, float *out, int h, int w, long long a_pitch,
                               long long out_pitch, int dt_bytes, int max_value, int win_h,
                               int win_w, const NoiseAcc *acc, double noise_var,
                               double *nu2_out, hipStream_t s) {
    const dim3 grid((w + TX - 1) / TX, (h + TY - 1) / TY);
    const float mf = (float)max_value;  // exact: max_value <= 65535
    if (dt_bytes == 1)
        hipLaunchKernelGGL(wiener_apply_kernel<uint8_t>, grid, dim3(NT), 0, s,
                           (const uint8_t *)a, out, h, w, a_pitch, out_pitch, win_h, win_w, mf,
                           acc, noise_var, nu2_out);
    else
        hipLaunchKernelGGL(wiener_apply_kernel<uint16_t>, grid, dim3(NT), 0, s,
                           (const uint16_t *)a, out, h, w, a_pitch, out_pitch, win_h, win_w, mf,
                           acc, noise_var, nu2_out);
    return hipGetLastError();
}

}  // namespace hd

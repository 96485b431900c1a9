// Image degradation on the device (the paper's degradImage, Alg. 1 step 3, which the paper
// names without defining): additive Gaussian noise of standard deviation sigma, rounded
// half-to-even and clipped to [0, M], then salt and pepper (probability `density`, 0 or M
// with one half each).
//
// Random numbers come from the counter-based generator Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC 2011): pixel p (row-major index) of stream s draws the block with counter
// (p mod 2^32, p div 2^32, s, 0) under key (seed mod 2^32, seed div 2^32). Words r0, r1
// feed a Box-Muller Gaussian in double precision, r2 decides the impulse, r3 its sign.
// No state: every pixel is independent, any launch shape gives the same image.
#include "tile_io.h"

namespace hd {
namespace {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {  // the key advances by the Weyl constants between rounds
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32->64 multiply each (v_mad_u64_u32) gives both halves
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x, m1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(m1 >> 32) ^ c.y ^ k0, (uint32_t)m1, (uint32_t)(m0 >> 32) ^ c.w ^ k1, (uint32_t)m0);
    }
    return c;
}

// One pixel of the degradation: the Gaussian value rounded and clipped, then the impulse.
// The rounded Gaussian stage rint(x + sigma z) is defined in double precision. It is first
// evaluated in single precision; only a value within `margin` of a rounding boundary (a
// half-integer), where the two could round differently, is recomputed in double. margin
// bounds the single-precision error of x + sigma z (|z| <= 6.7 for u1 >= 2^-32), so the
// result is the double-precision one.
__device__ __forceinline__ int degrade_pixel(float xv, uint4 r, int max_value, double sigma, double thr,
                                             float margin) {
    // ln u1 to a few ulps relative: for u1 >= 1/2 as log1p of the exact integer complement
    // (u1 = 1 - m 2^-32), below as the log of u1 itself
    const float ln_u1 = r.x >= 0x80000000u ? log1pf(-(float)(0xFFFFFFFFu - r.x) * 2.3283064365386963e-10f)
                                           : logf(((float)r.x + 1.0f) * 2.3283064365386963e-10f);
    const float u2f = (float)r.y * 2.3283064365386963e-10f;
    const float zf = sqrtf(-2.0f * ln_u1) * cospif(2.0f * u2f);
    const float pf = xv + (float)sigma * zf;
    const float fr = pf - floorf(pf);
    float g = rintf(pf);
    if (fabsf(fr - 0.5f) <= margin || !(fabsf(pf) < 1e30f)) {
        const double u1 = ((double)r.x + 1.0) * (1.0 / 4294967296.0);  // (0, 1], exact
        const double u2 = (double)r.y * (1.0 / 4294967296.0);          // [0, 1), exact
        const double two_pi = 2.0 * 3.141592653589793;
        const double z = __dmul_rn(sqrt(-2.0 * log(u1)), cos(__dmul_rn(two_pi, u2)));
        // x + sigma z rounded as written (no fused multiply-add), then half-to-even
        const double pre = __dadd_rn((double)xv, __dmul_rn(sigma, z));
        g = (float)fmin(fmax(rint(pre), -1.0), (double)max_value + 1.0);
    }
    int gi = (int)fminf(fmaxf(g, 0.0f), (float)max_value);
    if ((double)r.z < thr) gi = (r.w & 1u) ? max_value : 0;
    return gi;
}

// Each thread takes PPT consecutive pixels of the row-major image (independent generator
// blocks, so their arithmetic overlaps); the pixel index is split into row and column once
// per thread.
constexpr int PPT = 4;

template <typename T>
__global__ __launch_bounds__(256) void degrade_kernel(const T *__restrict__ clean, T *noisy, int h, int w,
                                                      long long cpitch, long long npitch, int max_value,
                                                      double sigma, double thr, uint32_t k0, uint32_t k1,
                                                      uint32_t stream_id, float margin) {
    const unsigned long long n = (unsigned long long)h * (unsigned)w;
    for (unsigned long long p0 = ((unsigned long long)blockIdx.x * 256 + threadIdx.x) * PPT; p0 < n;
         p0 += (unsigned long long)gridDim.x * 256 * PPT) {
        unsigned long long y0 = p0 / (unsigned)w;
        int x0 = (int)(p0 - y0 * (unsigned)w);
        long long ci[PPT], ni[PPT];
        float xv[PPT];
        {
            long long y = (long long)y0;
            int x = x0;
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                ci[j] = y * cpitch + x;
                ni[j] = y * npitch + x;
                xv[j] = p0 + j < n ? (float)clean[ci[j]] : 0.0f;
                if (++x == w) { x = 0; ++y; }
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const unsigned long long p = p0 + j;
            const uint4 r = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)(p >> 32), stream_id, 0u), k0, k1);
            const int g = degrade_pixel(xv[j], r, max_value, sigma, thr, margin);
            if (p < n) noisy[ni[j]] = (T)g;
        }
    }
}

}  // namespace

hipError_t launch_degrade(const void *clean, void *noisy, int h, int w, long long cpitch, long long npitch,
                          int eb, int max_value, double sigma, double density, unsigned long long seed,
                          uint32_t stream_id, hipStream_t s) {
    const unsigned long long quads = ((unsigned long long)h * (unsigned)w + PPT - 1) / PPT;
    const unsigned int blocks = (unsigned int)((quads + 255) / 256 < (1u << 20) ? (quads + 255) / 256 : (1u << 20));
    const double thr = floor(density * 4294967296.0);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    // single-precision error bound of x + sigma z: z to ~1e-6 relative (log, cos of an
    // angle rounded to 24 bits, sqrt), the product and sum to a few ulps; |z| <= 6.7.
    // Four times that bound.
    const float margin = (float)(4.0 * (1e-6 * sigma * 6.7 + 1.2e-7 * ((double)max_value + sigma * 6.7)) + 1e-6);
    if (eb == 1)
        hipLaunchKernelGGL(degrade_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, (const uint8_t *)clean,
                           (uint8_t *)noisy, h, w, cpitch, npitch, max_value, sigma, thr, k0, k1, stream_id, margin);
    else
        hipLaunchKernelGGL(degrade_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, (const uint16_t *)clean,
                           (uint16_t *)noisy, h, w, cpitch, npitch, max_value, sigma, thr, k0, k1, stream_id, margin);
    return hipGetLastError();
}

}  // namespace hd

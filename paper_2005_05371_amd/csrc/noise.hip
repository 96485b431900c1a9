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
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

template <typename T>
__global__ __launch_bounds__(256) void degrade_kernel(const T *__restrict__ clean, T *noisy, int h, int w,
                                                      long long cpitch, long long npitch, int max_value,
                                                      double sigma, double thr, uint32_t k0, uint32_t k1,
                                                      uint32_t stream_id) {
    const long long n = (long long)h * w;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const int y = (int)(p / w), x = (int)(p - (long long)y * w);
        const uint4 r = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)(p >> 32), stream_id, 0u), k0, k1);
        const double u1 = ((double)r.x + 1.0) * (1.0 / 4294967296.0);  // (0, 1], exact
        const double u2 = (double)r.y * (1.0 / 4294967296.0);          // [0, 1), exact
        const double two_pi = 2.0 * 3.141592653589793;
        const double z = __dmul_rn(sqrt(-2.0 * log(u1)), cos(__dmul_rn(two_pi, u2)));
        // x + sigma z rounded as written (no fused multiply-add), then half-to-even
        const double pre = __dadd_rn((double)clean[(long long)y * cpitch + x], __dmul_rn(sigma, z));
        double g = rint(pre);
        g = fmin(fmax(g, 0.0), (double)max_value);
        if ((double)r.z < thr) g = (r.w & 1u) ? (double)max_value : 0.0;
        noisy[(long long)y * npitch + x] = (T)g;
    }
}

}  // namespace

hipError_t launch_degrade(const void *clean, void *noisy, int h, int w, long long cpitch, long long npitch,
                          int eb, int max_value, double sigma, double density, unsigned long long seed,
                          uint32_t stream_id, hipStream_t s) {
    const long long n = (long long)h * w;
    const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    const double thr = floor(density * 4294967296.0);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (eb == 1)
        hipLaunchKernelGGL(degrade_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, (const uint8_t *)clean,
                           (uint8_t *)noisy, h, w, cpitch, npitch, max_value, sigma, thr, k0, k1, stream_id);
    else
        hipLaunchKernelGGL(degrade_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, (const uint16_t *)clean,
                           (uint16_t *)noisy, h, w, cpitch, npitch, max_value, sigma, thr, k0, k1, stream_id);
    return hipGetLastError();
}

}  // namespace hd

// Internal declarations shared by the HIP translation units of libhybrid_denoise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

// Symmetric (half-sample) mirror of i into [0, n), period 2n: ... c b a | a b c | c b a ...
__host__ __device__ __forceinline__ int mirror(int i, int n) {
    if ((unsigned)i < (unsigned)n) return i;
    const int p = 2 * n;
    int m = i % p;
    if (m < 0) m += p;
    return (m < n) ? m : (p - 1 - m);
}

// 128-bit accumulator of the Wiener variance numerators of one image:
// word 0 = low 64 bits, word 1 = carries out of the low word. Exact and independent of
// the order in which blocks add into it.
struct NoiseAcc {
    unsigned long long lo;
    unsigned long long hi;
};

// ---- launchers (all asynchronous on `s`) -------------------------------------------
// AMF of one image. dt_bytes: 1 (uint8) or 2 (uint16).
hipError_t launch_amf(const void *in, void *out, int h, int w, long long in_pitch,
                      long long out_pitch, int dt_bytes, int smax, int keep, hipStream_t s);

// Zero `n` noise accumulators.
hipError_t launch_zero_acc(NoiseAcc *acc, int n, hipStream_t s);

// Sum of the exact local-variance numerators (N * S2 - S1^2) of `a` into *acc.
hipError_t launch_wiener_partials(const void *a, int h, int w, long long pitch, int dt_bytes,
                                  int win_h, int win_w, NoiseAcc *acc, hipStream_t s);

// Wiener apply. nu2 from `acc` (acc != nullptr) or `noise_var` (acc == nullptr).
// nu2_out (device double*, may be null) receives the nu2 used.
hipError_t launch_wiener_apply(const void *a, float *out, int h, int w, long long a_pitch,
                               long long out_pitch, int dt_bytes, int max_value, int win_h,
                               int win_w, const NoiseAcc *acc, double noise_var,
                               double *nu2_out, hipStream_t s);

}  // namespace hd

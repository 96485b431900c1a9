// Device helpers shared by the stage kernels: work-item -> slice/tile mapping and
// staging of an image region (with symmetric padding) into LDS.
#pragma once

#include "hd_internal.h"

namespace hd {

// Integer type of S2 and of N * S2 - S1^2: 32 bits for 8-bit data (N * S2 <= 225 * 225 *
// 255^2 < 2^32), 64 bits for 16-bit data.
template <typename T>
struct SqT;
template <>
struct SqT<uint8_t> { using type = uint32_t; };
template <>
struct SqT<uint16_t> { using type = unsigned long long; };

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum of a 128-bit (lo, hi) value over the workgroup; every thread receives the total.
__device__ __forceinline__ void block_sum_u128(unsigned long long &lo, unsigned long long &hi,
                                               unsigned long long *s_lo, unsigned long long *s_hi) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long ol = __shfl_down(lo, off, 64), oh = __shfl_down(hi, off, 64);
        const unsigned long long sl = lo + ol;
        hi += oh + (sl < lo);
        lo = sl;
    }
    if (lane == 0) {
        s_lo[wv] = lo;
        s_hi[wv] = hi;
    }
    __syncthreads();
    unsigned long long tl = 0, th = 0;
    for (int k = 0; k < STAGE_THREADS / 64; ++k) {
        const unsigned long long sl = tl + s_lo[k];
        th += s_hi[k] + (sl < tl);
        tl = sl;
    }
    lo = tl;
    hi = th;
    __syncthreads();
}

// Minimum and maximum of (mn, mx) over the workgroup; every thread receives them.
__device__ __forceinline__ void block_minmax(float &mn, float &mx, unsigned long long *s_a,
                                             unsigned long long *s_b) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, off, 64));
        mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    }
    if (lane == 0) {
        s_a[wv] = __float_as_uint(mn);
        s_b[wv] = __float_as_uint(mx);
    }
    __syncthreads();
    for (int k = 0; k < STAGE_THREADS / 64; ++k) {
        mn = fminf(mn, __uint_as_float((uint32_t)s_a[k]));
        mx = fmaxf(mx, __uint_as_float((uint32_t)s_b[k]));
    }
    __syncthreads();
}

// Largest 16-bit sample value v with N * v^2 < 2^32 (N >= 1): at or below it, S2 of an
// N-sample window fits 32 bits.
__host__ __device__ inline uint32_t narrow_max_u16(uint32_t n) {
    uint32_t v = (uint32_t)__builtin_sqrt(4294967295.0 / (double)n);
    if (v > 65535u) v = 65535u;
    while (v > 0 && (unsigned long long)n * v * v > 0xffffffffull) --v;
    while (v < 65535u && (unsigned long long)n * (v + 1) * (v + 1) <= 0xffffffffull) ++v;
    return v;
}

// Constants of the Wiener output for one slice (window N = wh * ww, max value mf, noise
// power nu2).
struct WienerConst {
    uint32_t n, magic;  // S1 / N = mulhi(S1, magic) for S1 < 2^32 / N
    float rcp_n, inv_n2, nu2f, mf, rcp_m;
    uint32_t narrow_max;  // 16-bit data: sample maximum that keeps S2 in 32 bits
};

// The window and max-value constants, computed once on the host and passed to the kernels
// (a 64-bit integer division and three divisions per lane otherwise); nu2f is set in the
// kernel from the slice's noise power. N = 0 (no Wiener window) gives zeros.
__host__ __device__ inline WienerConst wiener_const(int wh, int ww, float mf) {
    WienerConst c{};
    c.n = (uint32_t)(wh * ww);
    if (c.n == 0) return c;
    c.magic = (uint32_t)((0x100000000ull + c.n - 1) / c.n);
    c.rcp_n = 1.0f / (float)c.n;
    c.inv_n2 = (float)(1.0 / ((double)c.n * (double)c.n));
    c.mf = mf;
    c.rcp_m = 1.0f / mf;
    c.narrow_max = narrow_max_u16(c.n);
    return c;
}
__device__ __forceinline__ WienerConst with_noise(WienerConst c, double nu2d) {
    c.nu2f = (float)nu2d;
    return c;
}

// 24 x 24-bit unsigned multiply, low 32 bits, at full rate. HIP's __umul24 returns int;
// this keeps the product unsigned, so that widening it to 64 bits does not sign-extend a
// product >= 2^31.
__device__ __forceinline__ uint32_t umul24(uint32_t a, uint32_t b) {
    return (uint32_t)__umul24(a, b);
}

// N * S2 - S1^2 of one window (N = window size <= 225). For 8-bit data every operand is
// below 2^24 (S1 <= 225 * 255, S2 <= 225 * 255^2) and both products below 2^32, so 24-bit
// multiplies are exact (full rate; 32-bit integer multiplies issue at a quarter of it).
//
// For 16-bit data the result needs 64 bits, but its factors stay small: N <= 225 < 2^8,
// S1 <= 225 * 65535 < 2^24 and S2 <= 225 * 65535^2 < 2^40. N * S2 is taken as two 24-bit
// products (S2's bits 0..23 and 24..39) and S1^2 as the low and high words of one
// 24 x 24-bit product: full-rate multiplies instead of quarter-rate 64-bit ones.
template <typename S2T>
__device__ __forceinline__ S2T window_num(S2T nwin, uint32_t s1, S2T s2) {
    if constexpr (sizeof(S2T) == 4) {
        return umul24(nwin, s2) - umul24(s1, s1);
    } else {
        const uint32_t n = (uint32_t)nwin;
        const uint64_t ns2 = ((uint64_t)umul24(n, (uint32_t)(s2 >> 24)) << 24) +
                             (uint64_t)umul24(n, (uint32_t)s2 & 0xFFFFFFu);
        const uint32_t a = s1 & 0xFFFFFFu;  // s1 < 2^24: the mask only tells the compiler
        return ns2 - (uint64_t)a * a;
    }
}

// v^2 of one sample. For 16-bit data (64-bit sums) v^2 < 2^32 is the low word of a
// full-rate 24-bit multiply, not a quarter-rate 64-bit product; 8-bit samples are left
// to the compiler, which already multiplies them at full rate.
template <typename S2T>
__device__ __forceinline__ S2T square_u16(uint32_t v) {
    if constexpr (sizeof(S2T) == 8) return (S2T)umul24(v, v);
    else return v * v;
}

// Adaptive Wiener output of one pixel (normalised by the max value) from the exact window
// sums S1 and num = N * S2 - S1^2 and the pixel's AMF value av:
//   mu = S1 / N, var = num / N^2, out = (mu + (av - mu) * max(var - nu2, 0) / max(var, nu2)) / M.
// Every kernel that writes Wiener output goes through this function, so all paths agree
// to the bit.
// The part that does not depend on the noise power: mu, var and av - mu.
struct WienerPrep {
    float mu, var, d;
};
// u32 -> float in one conversion instruction. For a value that comes from the high word of
// a 64-bit product or shift, the compiler widens the conversion into the 64-bit sequence
// (normalise, sticky bit, convert, scale: five more instructions); an empty asm statement
// on the value hides where it came from.
__device__ __forceinline__ float u32_to_float(uint32_t x) {
    asm("" : "+v"(x));
    return (float)x;
}
template <typename NumT>
__device__ __forceinline__ WienerPrep wiener_prep(uint32_t s1, NumT num, float av, const WienerConst &c) {
    float numf;
    if constexpr (sizeof(NumT) == 4) numf = (float)num;
    else numf = u32_to_float((uint32_t)(num >> 32)) * 4294967296.0f + (float)(uint32_t)num;
    // mu = S1 / N: exact integer quotient plus the remainder's share, so a flat window
    // gives its value exactly
    const uint32_t q = __umulhi(s1, c.magic);
    const float mu = u32_to_float(q) + (float)(s1 - umul24(q, c.n)) * c.rcp_n;  // q < 2^16, N <= 225
    return WienerPrep{mu, numf * c.inv_n2, av - mu};
}
__device__ __forceinline__ float wiener_finish(const WienerPrep &p, const WienerConst &c) {
    const float den = fmaxf(p.var, c.nu2f);
    const float gain = den > 0.0f ? fmaxf(p.var - c.nu2f, 0.0f) * __builtin_amdgcn_rcpf(den) : 0.0f;
    const float y = p.mu + p.d * gain;
    // y / max_value: reciprocal product plus one fma correction step
    const float q0 = y * c.rcp_m;
    return fmaf(fmaf(-q0, c.mf, y), c.rcp_m, q0);
}
template <typename NumT>
__device__ __forceinline__ float wiener_pixel(uint32_t s1, NumT num, float av, const WienerConst &c) {
    return wiener_finish(wiener_prep<NumT>(s1, num, av, c), c);
}

// Sum and sum of squares of the WW bytes (WW = 3, 5 or 7) starting at byte b of an LDS
// buffer, from the aligned dwords around them: byte reads at odd addresses would be merged
// by the compiler into misaligned wider LDS reads, which are slow. One byte-wise alignment
// and 4-byte dot products give the sums. Reads up to 3 bytes past the window's last byte.
template <int WW>
__device__ __forceinline__ void byte_window_sums(const unsigned char *base, int b, uint32_t &t1, uint32_t &t2) {
    static_assert(WW == 3 || WW == 5 || WW == 7, "window width");
    const int off = b & 3;
    const uint32_t *dw = (const uint32_t *)(base + (b - off));
    const uint32_t d0 = dw[0], d1 = dw[1];
    const uint32_t wa = __builtin_amdgcn_alignbyte(d1, d0, (uint32_t)off);  // bytes b .. b + 3
    if constexpr (WW == 3) {
        const uint32_t w3 = wa & 0x00ffffffu;
        t1 = __builtin_amdgcn_udot4(w3, 0x01010101u, 0u, false);
        t2 = __builtin_amdgcn_udot4(w3, w3, 0u, false);
    } else if constexpr (WW == 5) {
        const uint32_t e = (d1 >> (8 * off)) & 0xffu;  // byte b + 4
        t1 = __builtin_amdgcn_udot4(wa, 0x01010101u, e, false);
        t2 = __builtin_amdgcn_udot4(wa, wa, e * e, false);
    } else {
        const uint32_t wb = __builtin_amdgcn_alignbyte(dw[2], d1, (uint32_t)off) & 0x00ffffffu;  // b + 4 .. b + 6
        t1 = __builtin_amdgcn_udot4(wa, 0x01010101u, __builtin_amdgcn_udot4(wb, 0x01010101u, 0u, false), false);
        t2 = __builtin_amdgcn_udot4(wa, wa, __builtin_amdgcn_udot4(wb, wb, 0u, false), false);
    }
}

// Sum, sum of squares and maximum of the WW 16-bit samples (WW = 3, 5 or 7) starting at
// element e of an LDS buffer of uint16_t, from the aligned dwords around them: one
// half-word alignment, then 2-element dot products. The sum of squares is exact only while
// WW * max^2 < 2^32 (the caller checks the maximum). Reads up to one element past the last.
template <int WW, bool TRACK_MAX = true>
__device__ __forceinline__ void u16_window_sums(const uint16_t *base, int e, uint32_t &t1, uint32_t &t2,
                                                uint32_t &mx) {
    static_assert(WW == 3 || WW == 5 || WW == 7, "window width");
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    constexpr int P = WW / 2;  // element pairs; one single element after them
    const uint32_t *dw = (const uint32_t *)(base + (e & ~1));
    const uint32_t sh = (uint32_t)(e & 1) * 16u;
    uint32_t d[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i) d[i] = dw[i];
    const uint32_t last = (d[P] >> sh) & 0xffffu;
    uint32_t s1 = last, s2 = last * last, m = last;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const uint32_t pr = __builtin_amdgcn_alignbit(d[i + 1], d[i], sh);  // elements e + 2i, e + 2i + 1
        const u16x2 v = __builtin_bit_cast(u16x2, pr);
        s1 = __builtin_amdgcn_udot2(v, (u16x2){1, 1}, s1, false);
        s2 = __builtin_amdgcn_udot2(v, v, s2, false);
        if constexpr (TRACK_MAX) m = max(m, max(pr & 0xffffu, pr >> 16));
    }
    t1 = s1;
    t2 = s2;
    mx = m;
}

// N * S2 - S1^2 (64 bits) from a 32-bit S2 (16-bit data whose window maximum keeps N * max^2
// below 2^32): two 32 x 32 -> 64-bit multiply-adds.
__device__ __forceinline__ unsigned long long window_num_narrow(uint32_t n, uint32_t s1, uint32_t s2) {
    return (unsigned long long)n * s2 - (unsigned long long)s1 * s1;
}

// Contrast stretch of one output value to the slice's range [lo, hi]: (y - lo) / (hi - lo),
// unchanged when the slice is constant (hi == lo). The stand-alone and the resident paths
// both go through it.
__device__ __forceinline__ float stretch_pixel(float y, float lo, float hi) {
    return hi > lo ? (y - lo) / (hi - lo) : y;
}
// (min, max) of float outputs packed in 64 bits, max in the high word.
__device__ __forceinline__ unsigned long long pack_range(float mn, float mx) {
    return ((unsigned long long)__float_as_uint(mx) << 32) | (unsigned long long)__float_as_uint(mn);
}
__device__ __forceinline__ float range_lo(unsigned long long r) { return __uint_as_float((uint32_t)r); }
__device__ __forceinline__ float range_hi(unsigned long long r) { return __uint_as_float((uint32_t)(r >> 32)); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2). Give each
// XCD a contiguous run of tiles so that vertically and horizontally adjacent tiles, which
// share halo rows, mostly hit the same L2.
__device__ __forceinline__ int xcd_remap(int b, int g) {
    const int x = b & 7, i = b >> 3;
    const int q = g >> 3, r = g & 7;
    return x * q + min(x, r) + i;
}

// Index of the slice holding global tile `t` (binary search over ascending tile_begin).
__device__ __forceinline__ int slice_index(const SliceSet &set, int t) {
    if (set.n == 1) return 0;
    int lo = 0, hi = set.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (set.many[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Tile range and size of slice i.
struct SliceExtent {
    int tile_begin, ntiles, h, w;
};
__device__ __forceinline__ SliceExtent slice_extent(const SliceSet &set, int i) {
    SliceExtent e;
    e.tile_begin = set.n == 1 ? set.one.tile_begin : set.many[i].tile_begin;
    e.h = set.n == 1 ? set.one.h : set.many[i].h;
    e.w = set.n == 1 ? set.one.w : set.many[i].w;
    const int tx = set.n == 1 ? set.one.tiles_x : set.many[i].tiles_x;
    e.ntiles = tx * ((e.h + TILE_Y - 1) / TILE_Y);
    return e;
}

// Descriptor of slice i by value (kernel argument for a single slice, else the table).
__device__ __forceinline__ SliceDesc slice_desc(const SliceSet &set, int i) {
    SliceDesc d;
    if (set.n == 1) {
        d = set.one;
    } else {
        d = set.many[i];
    }
    return d;
}

// Exact i / d for 0 <= i < 4096, 1 <= d <= 16 with m = ceil(65536 / d).
// lt / tx for 0 <= lt, 1 <= tx (a tile's row in its slice): a single-precision reciprocal
// estimate, exact after one correction each way while lt < 2^22; exact division above
__device__ __forceinline__ int div_tiles(int lt, int tx) {
    if (lt >= (1 << 22)) return lt / tx;
    int q = (int)((float)lt * __builtin_amdgcn_rcpf((float)tx));
    q -= (q * tx > lt) ? 1 : 0;
    q += ((q + 1) * tx <= lt) ? 1 : 0;
    return q;
}
__device__ __forceinline__ int div_small(int i, int m) { return (i * m) >> 16; }

// Geometry of a staged region: element (r, c) of the region lives at lds[r * lpt + off + c].
struct Staged {
    int off;
    int lpt;
};

// Stage rows [gy0, gy0 + rows) x columns [gx0, gx0 + cols) of `img` (h x w, pitch in
// elements, mirrored outside the image) into LDS; region element (r, c) lands at
// lds[r * lpt + off + c]. With `aligned` (image base and row pitch in bytes multiples of
// 16) the region is covered by 16-byte chunks of the image row: chunks inside the row take
// one 16-byte load each, the in-image elements of a chunk that straddles the row end are
// loaded one by one, and the columns outside the image are then copied inside LDS from
// their mirror columns (one reflection; a region that needs more, on images narrower than
// the window radius, loads every element through the mirror instead). Rows outside the
// image are read from their mirror rows directly. Without `aligned`, element by element.
// With ODD_PITCH the LDS row pitch is an odd number of 16-byte chunks (one chunk of padding
// when needed), so that rows 1 to 7 apart start in different LDS banks: the per-pixel
// window reads of scattered pixels then conflict less. All threads of the workgroup must
// call it (it may synchronise them).
//
// THREADS is the workgroup size. With vmax set (16-bit data), *vmax receives this thread's
// maximum over the elements it loaded, a superset of the region's elements (whole 16-byte
// chunks); the region's maximum is the maximum over the workgroup.
template <typename T, bool ODD_PITCH = false, int THREADS = STAGE_THREADS>
__device__ __forceinline__ Staged stage_region(T *lds, const T *__restrict__ img, int h, int w,
                                               long long pitch, int gy0, int gx0, int rows,
                                               int cols, bool aligned, uint32_t *vmax = nullptr) {
    constexpr int EB = sizeof(T);
    constexpr int PER = 16 / EB;
    const int tid = threadIdx.x;
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    auto pkmax = [](uint32_t a, uint32_t b) {
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
    };
    uint32_t mx = 0;  // packed pair of 16-bit maxima (chunk loads) or a plain maximum
    Staged g;
    // columns outside the image that one reflection maps into the region
    const int lo_out = max(0, -gx0), hi_out = max(0, gx0 + cols - w);
    const bool one_reflect = lo_out <= w && hi_out <= w && (lo_out == 0 || lo_out <= gx0 + cols) &&
                             (hi_out == 0 || 2 * w - (gx0 + cols) >= gx0);
    if (aligned && one_reflect) {
        const int b0 = gx0 * EB;
        const int ab = b0 & ~15;  // floor to a chunk boundary (also for negative b0)
        const int off_b = b0 - ab;
        const int nch = (off_b + cols * EB + 15) >> 4;
        const int pch = ODD_PITCH ? (nch | 1) : nch;  // row pitch in chunks
        g.off = off_b / EB;
        g.lpt = pch * PER;
        const int total = rows * nch;
        const int m = (65536 + nch - 1) / nch;
        const int wb = w * EB;
#pragma unroll 2
        for (int i = tid; i < total; i += THREADS) {
            const int r = div_small(i, m);
            const int c = i - r * nch;
            const int cb = ab + c * 16;
            const T *row = img + (long long)mirror(gy0 + r, h) * pitch;
            if (cb >= 0 && cb + 16 <= wb) {
                const uint4 v = *(const uint4 *)((const char *)row + cb);
                ((uint4 *)lds)[r * pch + c] = v;
                if (vmax) mx = pkmax(mx, pkmax(pkmax(v.x, v.y), pkmax(v.z, v.w)));
            } else if (cb < wb && cb + 16 > 0) {
                const int gx = cb / EB;  // exact: cb is a multiple of 16
                for (int e = max(0, -gx); e < PER && gx + e < w; ++e) {
                    const T v = row[gx + e];
                    lds[r * g.lpt + c * PER + e] = v;
                    if (vmax) mx = pkmax(mx, (uint32_t)v);
                }
            }
        }
        if (lo_out > 0 || hi_out > 0) {
            __syncthreads();
            // out-of-image columns from their mirror columns, which lie in the region
            const int nout = lo_out + hi_out;
            for (int i = tid; i < rows * nout; i += THREADS) {
                const int r = i / nout, k = i - r * nout;
                const int gx = k < lo_out ? gx0 + k : w + (k - lo_out);
                T *lr = lds + r * g.lpt + g.off;
                lr[gx - gx0] = lr[mirror(gx, w) - gx0];
            }
        }
    } else {
        g.off = 0;
        g.lpt = (ODD_PITCH ? (((cols * EB + 15) / 16) | 1) : (cols * EB + 15) / 16) * PER;
        const int total = rows * cols;
        // i / cols = mulhi(i, ceil(2^32 / cols)), exact for i < 2^16 and cols < 2^8
        const uint32_t mc = (uint32_t)((0x100000000ull + cols - 1) / cols);
#pragma unroll 4
        for (int i = tid; i < total; i += THREADS) {
            const int r = (int)__umulhi((uint32_t)i, mc);
            const int c = i - r * cols;
            const T v = img[(long long)mirror(gy0 + r, h) * pitch + mirror(gx0 + c, w)];
            lds[r * g.lpt + c] = v;
            if (vmax) mx = max(mx, (uint32_t)v);
        }
    }
    if (vmax) *vmax = max(mx & 0xffffu, mx >> 16);
    return g;
}

// Exact i / d for 0 <= i < 4096, 1 <= d <= 255 with m = ceil(2^20 / d).
__device__ __forceinline__ int div_region(int i, int m) { return (i * m) >> 20; }
__host__ __device__ __forceinline__ int div_region_magic(int d) { return ((1 << 20) + d - 1) / d; }

// Store rows x cols of an LDS tile (element (r, c) at lds[r * lpt + c]) to the image at
// (gy0, gx0), clipped to h x w. When the tile row is full and the image rows are 16-byte
// aligned, each lane gathers 16 bytes from LDS and issues one 16-byte store.
template <typename T>
__device__ __forceinline__ void store_region(T *__restrict__ img, int h, int w, long long pitch,
                                             int gy0, int gx0, const T *lds, int lpt, int rows,
                                             int cols, bool aligned) {
    constexpr int EB = sizeof(T);
    constexpr int PER = 16 / EB;  // elements per 16-byte chunk
    const int tid = threadIdx.x;
    const int rows_in = min(rows, h - gy0);
    if (aligned && gx0 + cols <= w && ((gx0 * EB) & 15) == 0 && (cols % PER) == 0) {
        const int nch = cols / PER;
        const int m = (65536 + nch - 1) / nch;
        const int total = rows_in * nch;
        for (int i = tid; i < total; i += STAGE_THREADS) {
            const int r = div_small(i, m);
            const int c = i - r * nch;
            const T *src = lds + r * lpt + c * PER;
            uint32_t wd[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (EB == 1)
                    wd[q] = (uint32_t)src[4 * q] | ((uint32_t)src[4 * q + 1] << 8) |
                            ((uint32_t)src[4 * q + 2] << 16) | ((uint32_t)src[4 * q + 3] << 24);
                else
                    wd[q] = (uint32_t)src[2 * q] | ((uint32_t)src[2 * q + 1] << 16);
            }
            *(uint4 *)((char *)img + ((long long)(gy0 + r) * pitch + gx0) * EB + c * 16) =
                make_uint4(wd[0], wd[1], wd[2], wd[3]);
        }
    } else {
        const int lane = tid & 63, wv = tid >> 6;
        const int cols_in = min(cols, w - gx0);
        for (int r = wv; r < rows_in; r += STAGE_THREADS / 64) {
            T *dst = img + (long long)(gy0 + r) * pitch + gx0;
            for (int c = lane; c < cols_in; c += 64) dst[c] = lds[r * lpt + c];
        }
    }
}

}  // namespace hd

// Stage 2 of the hybrid de-noiser on gfx950: adaptive Wiener filter (local mean /
// variance form) of the AMF output, and the per-slice noise power reduction.
//
// The hybrid applies a Wiener filter to the AMF output (arXiv 2005.05371, Sec. IV and
// Fig. 4; Alg. 1, procedure parallelHybrid). For the AMF output a, over a win_h x win_w
// window with symmetric padding:
//   S1 = sum a, S2 = sum a^2 (exact integers), N = win_h * win_w,
//   mu = S1 / N, s2 = (N * S2 - S1^2) / N^2 (population variance),
//   nu2 = caller value, or the mean of s2 over the slice = sum(N * S2 - S1^2) / (N^2 h w),
//   out = (mu + (a - mu) * max(s2 - nu2, 0) / max(s2, nu2)) / max_value, mu when both are 0.
//
// Kernels: one 64 x 32 tile per workgroup (256 threads, 8 pixels per thread in one
// column); the tile plus its window halo is staged in LDS with 16-byte loads; row sums
// over win_w, then a sliding column sum over win_h, all in exact integers. The noise
// reduction sums the exact per-tile partials of each slice (128-bit, fixed order).
#include <type_traits>

#include "tile_io.h"

namespace hd {
namespace {

constexpr int NT = STAGE_THREADS;
constexpr int RPT = TILE_Y / (NT / 64);  // 8 rows per thread

// Any window size: row sums through LDS (h1 / h2), then a sliding column sum.
template <typename T, bool APPLY>
__global__ __launch_bounds__(NT) void wiener_stage_kernel(SliceSet set, int total_tiles, int wh,
                                                          int ww, float mf,
                                                          const double *__restrict__ nu2,
                                                          double noise_var,
                                                          unsigned long long *__restrict__ partials,
                                                          int aligned,
                                                          unsigned long long *__restrict__ ranges,
                                                          WienerConst wcb) {
    using S2T = typename SqT<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long s_wsum[NT / 64], s_wsum2[NT / 64];

    int tile;
    if (set.list) {
        if ((int)blockIdx.x >= *set.list_count) return;
        tile = set.list[blockIdx.x];
    } else {
        tile = xcd_remap(blockIdx.x, total_tiles);
    }
    const int si = slice_index(set, tile);
    const SliceDesc sd = slice_desc(set, si);
    const int H = sd.h, W = sd.w;
    const int lt = tile - sd.tile_begin;
    const int ty = div_tiles(lt, sd.tiles_x);
    const int x0 = (lt - ty * sd.tiles_x) * TILE_X;
    const int y0 = ty * TILE_Y;
    const int rh = wh >> 1, rw = ww >> 1;
    const int rows = TILE_Y + 2 * rh, cols = TILE_X + 2 * rw;
    const int nch_max = (15 + cols * (int)sizeof(T) + 15) / 16;

    T *s_a = (T *)smem;
    uint32_t *h1 = (uint32_t *)(smem + rows * nch_max * 16);
    S2T *h2 = (S2T *)(smem + rows * nch_max * 16 + rows * TILE_X * 4);

    const Staged st = stage_region<T>(s_a, (const T *)sd.amf, H, W, sd.amf_pitch, y0 - rh, x0 - rw,
                                      rows, cols, aligned != 0);
    __syncthreads();
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ uint32_t s_wmax[NT / 64];
    // 1. row sums over win_w of every staged row, for each tile column: S1 in 32 bits; S2 in
    //    32 bits for 8-bit data, and for 16-bit data first in 32 bits too, checked against
    //    the tile's maximum (a tile whose samples could overflow them redoes them in 64)
    uint32_t *h2n = (uint32_t *)h2;
    uint32_t tmax = 0;
    auto hsums_narrow = [&](auto wwc) {
        constexpr int WW = decltype(wwc)::value;
        for (int r = wv; r < rows; r += NT / 64) {
            uint32_t t1 = 0, t2 = 0;
            if constexpr (WW > 0 && sizeof(T) == 1) {
                byte_window_sums<WW>((const unsigned char *)s_a, r * st.lpt + st.off + lane, t1, t2);
            } else if constexpr (WW > 0) {
                uint32_t m = 0;
                u16_window_sums<WW>((const uint16_t *)s_a, r * st.lpt + st.off + lane, t1, t2, m);
                tmax = max(tmax, m);
            } else {
                const T *row = s_a + r * st.lpt + st.off + lane;
                for (int dx = 0; dx < ww; ++dx) {
                    const uint32_t v = row[dx];
                    t1 += v;
                    t2 += umul24(v, v);  // v^2 < 2^32; the sum is checked against the maximum below
                    tmax = max(tmax, v);
                }
            }
            h1[r * TILE_X + lane] = t1;
            h2n[r * TILE_X + lane] = t2;
        }
    };
    if (ww == 3) hsums_narrow(std::integral_constant<int, 3>{});
    else if (ww == 5) hsums_narrow(std::integral_constant<int, 5>{});
    else if (ww == 7) hsums_narrow(std::integral_constant<int, 7>{});
    else hsums_narrow(std::integral_constant<int, 0>{});
    bool wide = false;
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) tmax = max(tmax, (uint32_t)__shfl_xor((int)tmax, off, 64));
        if (lane == 0) s_wmax[wv] = tmax;
    }
    __syncthreads();
    if constexpr (sizeof(T) == 2) {
        uint32_t vmax = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) vmax = max(vmax, s_wmax[i]);
        wide = vmax > wcb.narrow_max;  // uniform across the workgroup
        if (wide) {
            // samples too large for 32-bit S2: the row sums of squares again, in 64 bits
            unsigned long long *h2w = (unsigned long long *)h2;
            for (int r = wv; r < rows; r += NT / 64) {
                const T *row = s_a + r * st.lpt + st.off + lane;
                unsigned long long t2 = 0;
                for (int dx = 0; dx < ww; ++dx) t2 += square_u16<unsigned long long>(row[dx]);
                h2w[r * TILE_X + lane] = t2;
            }
            __syncthreads();
        }
    }

    // 2. exact window sums slide down the column: S1 in 32 bits; S2 in 32 bits (8-bit data,
    //    and 16-bit tiles whose maximum allows it) or 64 bits; N * S2 - S1^2 in 32 bits for
    //    8-bit data (N * S2 <= 225 * 225 * 255^2 < 2^32), 64 bits for 16-bit data
    const uint32_t nwin = (uint32_t)(wh * ww);
    const int gx = x0 + lane;
    const int j0 = wv * RPT;
    const bool col_ok = gx < W;
    const int rows_ok = min(RPT, H - (y0 + j0));
    auto columns = [&](auto s2tag) {
        using C2 = decltype(s2tag);  // type of the S2 sums in LDS
        using NumT = typename std::conditional<sizeof(T) == 1, uint32_t, unsigned long long>::type;
        const C2 *hh = (const C2 *)h2;
        auto num_of = [&](uint32_t a1, C2 a2) -> NumT {
            if constexpr (sizeof(T) == 1) return window_num<uint32_t>(nwin, a1, a2);
            else if constexpr (sizeof(C2) == 4) return window_num_narrow(nwin, a1, a2);
            else return window_num<unsigned long long>((unsigned long long)nwin, a1, a2);
        };
        uint32_t s1 = 0;
        C2 s2 = 0;
        for (int dy = 0; dy < wh; ++dy) {
            s1 += h1[(j0 + dy) * TILE_X + lane];
            s2 += hh[(j0 + dy) * TILE_X + lane];
        }
        if constexpr (APPLY) {
            const WienerConst wc = with_noise(wcb, nu2 ? nu2[si] : noise_var);
            float *orow = sd.out + (long long)(y0 + j0) * sd.out_pitch + gx;
            const T *arow = s_a + (j0 + rh) * st.lpt + st.off + lane + rw;
            float mn = __builtin_inff(), mx = -__builtin_inff();
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (j > 0) {  // slide the column window down by one row
                    s1 += h1[(j0 + j + wh - 1) * TILE_X + lane] - h1[(j0 + j - 1) * TILE_X + lane];
                    s2 += hh[(j0 + j + wh - 1) * TILE_X + lane] - hh[(j0 + j - 1) * TILE_X + lane];
                }
                if (col_ok && j < rows_ok) {
                    const float y = wiener_pixel<NumT>(s1, num_of(s1, s2), (float)arow[j * st.lpt], wc);
                    orow[(long long)j * sd.out_pitch] = y;
                    mn = fminf(mn, y);
                    mx = fmaxf(mx, y);
                }
            }
            if (ranges) {  // the tile's output range, for the contrast stretch
                block_minmax(mn, mx, s_wsum, s_wsum2);
                if (tid == 0) ranges[tile] = pack_range(mn, mx);
            }
        } else {
            unsigned long long t = 0;
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (j > 0) {
                    s1 += h1[(j0 + j + wh - 1) * TILE_X + lane] - h1[(j0 + j - 1) * TILE_X + lane];
                    s2 += hh[(j0 + j + wh - 1) * TILE_X + lane] - hh[(j0 + j - 1) * TILE_X + lane];
                }
                if (col_ok && j < rows_ok) t += (unsigned long long)num_of(s1, s2);
            }
            t = wave_sum_u64(t);
            if (lane == 0) s_wsum[wv] = t;
            __syncthreads();
            if (tid == 0) {
                unsigned long long b = 0;
                for (int i = 0; i < NT / 64; ++i) b += s_wsum[i];
                partials[tile] = b;
            }
        }
    };
    if (sizeof(T) == 2 && wide) columns((unsigned long long)0);
    else columns((uint32_t)0);
}

// Square 3 / 5 / 7 windows, one wave per tile: lane = tile column. The lane walks down
// its column over the TILE_Y + WIN - 1 region rows, forms each row's horizontal sums once
// and keeps the last WIN of them in registers (a ring whose indices the unrolled loop
// fixes), so an output pixel costs (TILE_Y + WIN - 1) / TILE_Y row sums. 16-bit sums of
// squares are 32-bit when the staged region's maximum keeps them below 2^32 (the tile's
// maximum from the staging loads), 64-bit otherwise.
template <typename T, bool APPLY, int WIN, typename S2T>
__device__ __forceinline__ void column_pass(const T *s_a, const Staged &st, const SliceDesc &sd, int si, int tile,
                                            int y0, int gx, const double *__restrict__ nu2, double noise_var,
                                            unsigned long long *__restrict__ partials,
                                            unsigned long long *__restrict__ ranges, const WienerConst &wcb) {
    constexpr int R = WIN / 2, ROWS = TILE_Y + 2 * R;
    constexpr uint32_t nwin = (uint32_t)(WIN * WIN);
    const int lane = threadIdx.x;
    const bool col_ok = gx < sd.w;
    const int rows_ok = min(TILE_Y, sd.h - y0);
    const T *col = s_a + st.off + lane;
    uint32_t r1[WIN];
    S2T r2[WIN];
    uint32_t s1 = 0;
    S2T s2 = 0;
    float mn = __builtin_inff(), mx = -__builtin_inff();
    unsigned long long t = 0, sum_s2 = 0, sum_s1sq = 0;
    WienerConst wc = wcb;
    if constexpr (APPLY) wc = with_noise(wcb, nu2 ? nu2[si] : noise_var);
    float *ocol = sd.out + (long long)y0 * sd.out_pitch + gx;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        uint32_t t1;
        S2T t2;
        if constexpr (sizeof(T) == 1) {
            byte_window_sums<WIN>((const unsigned char *)s_a, i * st.lpt + st.off + lane, t1, t2);
        } else if constexpr (sizeof(S2T) == 4) {
            uint32_t unused;
            u16_window_sums<WIN, false>((const uint16_t *)s_a, i * st.lpt + st.off + lane, t1, t2, unused);
        } else {
            t1 = 0;
            t2 = 0;
#pragma unroll
            for (int dx = 0; dx < WIN; ++dx) {
                const uint32_t v = col[i * st.lpt + dx];
                t1 += v;
                t2 += square_u16<S2T>(v);
            }
        }
        s1 += t1;
        s2 += t2;
        if (i >= WIN) {
            s1 -= r1[i % WIN];
            s2 -= r2[i % WIN];
        }
        r1[i % WIN] = t1;
        r2[i % WIN] = t2;
        if (i >= WIN - 1) {
            const int j = i - (WIN - 1);  // output row of this window position
            if (col_ok && j < rows_ok) {
                if constexpr (sizeof(T) == 1) {
                    const uint32_t num = window_num<uint32_t>(nwin, s1, s2);
                    if constexpr (APPLY) {
                        const float y = wiener_pixel<uint32_t>(s1, num, (float)col[(j + R) * st.lpt + R], wc);
                        ocol[(long long)j * sd.out_pitch] = y;
                        mn = fminf(mn, y);
                        mx = fmaxf(mx, y);
                    } else {
                        t += num;
                    }
                } else if constexpr (APPLY) {
                    unsigned long long num;
                    if constexpr (sizeof(S2T) == 4) num = window_num_narrow(nwin, s1, s2);
                    else num = (unsigned long long)nwin * s2 - (unsigned long long)s1 * s1;
                    const float y =
                        wiener_pixel<unsigned long long>(s1, num, (float)col[(j + R) * st.lpt + R], wc);
                    ocol[(long long)j * sd.out_pitch] = y;
                    mn = fminf(mn, y);
                    mx = fmaxf(mx, y);
                } else {
                    // sum of N * S2 - S1^2 over the column as N * (sum S2) - (sum S1^2): two
                    // 64-bit accumulations per pixel instead of two 64-bit multiply-adds
                    // (s1 < 2^24, so s1^2 is one 24-bit product's low and high words)
                    sum_s2 += (unsigned long long)s2;
                    const uint32_t a = s1 & 0xFFFFFFu;
                    sum_s1sq += (unsigned long long)a * a;
                }
            }
        }
    }
    if constexpr (APPLY) {
        if (ranges) {  // the tile's output range, for the contrast stretch
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                mn = fminf(mn, __shfl_xor(mn, off, 64));
                mx = fmaxf(mx, __shfl_xor(mx, off, 64));
            }
            if (lane == 0) ranges[tile] = pack_range(mn, mx);
        }
    } else {
        if constexpr (sizeof(T) == 2) t = (unsigned long long)nwin * sum_s2 - sum_s1sq;  // exact mod 2^64
        t = wave_sum_u64(t);
        if (lane == 0) partials[tile] = t;
    }
}

template <typename T, bool APPLY, int WIN>
__global__ __launch_bounds__(64) void wiener_column_kernel(SliceSet set, int total_tiles,
                                                           const double *__restrict__ nu2, double noise_var,
                                                           unsigned long long *__restrict__ partials, int aligned,
                                                           unsigned long long *__restrict__ ranges, WienerConst wcb) {
    constexpr int R = WIN / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    int tile;
    if (set.list) {
        if ((int)blockIdx.x >= *set.list_count) return;
        tile = set.list[blockIdx.x];
    } else {
        tile = xcd_remap(blockIdx.x, total_tiles);
    }
    const int si = slice_index(set, tile);
    const SliceDesc sd = slice_desc(set, si);
    const int lt = tile - sd.tile_begin;
    const int ty = div_tiles(lt, sd.tiles_x);
    const int x0 = (lt - ty * sd.tiles_x) * TILE_X;
    const int y0 = ty * TILE_Y;
    T *s_a = (T *)smem;
    uint32_t vmax = 0;
    const Staged st = stage_region<T, false, 64>(s_a, (const T *)sd.amf, sd.h, sd.w, sd.amf_pitch, y0 - R, x0 - R,
                                                 TILE_Y + 2 * R, TILE_X + 2 * R, aligned != 0,
                                                 sizeof(T) == 2 ? &vmax : nullptr);
    __syncthreads();
    const int gx = x0 + (int)threadIdx.x;
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off, 64));
        if (vmax > wcb.narrow_max) {  // uniform across the wave
            column_pass<T, APPLY, WIN, unsigned long long>(s_a, st, sd, si, tile, y0, gx, nu2, noise_var, partials,
                                                           ranges, wcb);
            return;
        }
    }
    column_pass<T, APPLY, WIN, uint32_t>(s_a, st, sd, si, tile, y0, gx, nu2, noise_var, partials, ranges, wcb);
}

// One workgroup per slice: exact 128-bit sum of the slice's tile partials, then
// nu2 = sum / (N^2 h w) in double.
__global__ __launch_bounds__(256) void noise_reduce_kernel(SliceSet set,
                                                           const unsigned long long *__restrict__ partials,
                                                           int wh, int ww, double *__restrict__ nu2) {
    __shared__ unsigned long long s_lo[256], s_hi[256];
    const int si = blockIdx.x;
    const SliceDesc sd = slice_desc(set, si);
    const int ntiles = sd.tiles_x * ((sd.h + TILE_Y - 1) / TILE_Y);
    __shared__ unsigned long long s_px[256];
    unsigned long long lo = 0, hi = 0, px = 0;
    for (int i = threadIdx.x; i < ntiles; i += 256) {
        if (set.flags && !set.flags[sd.tile_begin + i]) continue;
        const unsigned long long p = partials[sd.tile_begin + i];
        lo += p;
        hi += (lo < p);
        const int ty = i / sd.tiles_x, tx = i - ty * sd.tiles_x;
        px += (unsigned long long)min(TILE_Y, sd.h - ty * TILE_Y) * min(TILE_X, sd.w - tx * TILE_X);
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    s_px[threadIdx.x] = px;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
            const unsigned long long a = s_lo[threadIdx.x], b = s_lo[threadIdx.x + stride];
            const unsigned long long sum = a + b;
            s_lo[threadIdx.x] = sum;
            s_hi[threadIdx.x] += s_hi[threadIdx.x + stride] + (sum < a);
            s_px[threadIdx.x] += s_px[threadIdx.x + stride];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = (double)(wh * ww);
        const double total = (double)s_hi[0] * 18446744073709551616.0 + (double)s_lo[0];
        // mean over the slice's pixels (over the flagged tiles' pixels when flags are set)
        const double npx = set.flags ? (double)s_px[0] : (double)sd.h * (double)sd.w;
        nu2[si] = npx > 0 ? total / (n * n * npx) : 0.0;
    }
}

// Range (min, max) of every 64 x 32 tile of the float outputs (one workgroup per tile).
__global__ __launch_bounds__(256) void tile_range_kernel(SliceSet set, int total_tiles,
                                                         unsigned long long *__restrict__ tile_ranges) {
    __shared__ unsigned long long s_a[4], s_b[4];
    const int tile = xcd_remap(blockIdx.x, total_tiles);
    const SliceDesc sd = slice_desc(set, slice_index(set, tile));
    const int lt = tile - sd.tile_begin;
    const int ty = div_tiles(lt, sd.tiles_x);
    const int x = (lt - ty * sd.tiles_x) * TILE_X + (threadIdx.x & 63);
    const int y0 = ty * TILE_Y + (threadIdx.x >> 6) * RPT;
    float mn = __builtin_inff(), mx = -__builtin_inff();
    if (x < sd.w)
        for (int j = 0; j < RPT && y0 + j < sd.h; ++j) {
            const float v = sd.out[(long long)(y0 + j) * sd.out_pitch + x];
            mn = fminf(mn, v);
            mx = fmaxf(mx, v);
        }
    block_minmax(mn, mx, s_a, s_b);
    if (threadIdx.x == 0) tile_ranges[tile] = pack_range(mn, mx);
}

// One workgroup per slice: the slice's output range from its tiles' ranges.
__global__ __launch_bounds__(256) void range_reduce_kernel(SliceSet set,
                                                           const unsigned long long *__restrict__ tile_ranges,
                                                           unsigned long long *__restrict__ slice_ranges) {
    __shared__ unsigned long long s_a[4], s_b[4];
    const int si = blockIdx.x;
    const SliceExtent e = slice_extent(set, si);
    float mn = __builtin_inff(), mx = -__builtin_inff();
    for (int i = threadIdx.x; i < e.ntiles; i += 256) {
        const unsigned long long r = tile_ranges[e.tile_begin + i];
        mn = fminf(mn, range_lo(r));
        mx = fmaxf(mx, range_hi(r));
    }
    block_minmax(mn, mx, s_a, s_b);
    if (threadIdx.x == 0) slice_ranges[si] = pack_range(mn, mx);
}

// Contrast stretch in place: one workgroup per 64 x 32 tile of the outputs.
__global__ __launch_bounds__(256) void stretch_kernel(SliceSet set, int total_tiles,
                                                      const unsigned long long *__restrict__ slice_ranges) {
    const int tile = xcd_remap(blockIdx.x, total_tiles);
    const int si = slice_index(set, tile);
    const SliceDesc sd = slice_desc(set, si);
    const int lt = tile - sd.tile_begin;
    const int ty = div_tiles(lt, sd.tiles_x);
    const int x = (lt - ty * sd.tiles_x) * TILE_X + (threadIdx.x & 63);
    const int y0 = ty * TILE_Y + (threadIdx.x >> 6) * RPT;
    const unsigned long long r = slice_ranges[si];
    const float lo = range_lo(r), hi = range_hi(r);
    if (x >= sd.w) return;
    for (int j = 0; j < RPT && y0 + j < sd.h; ++j) {
        float *p = sd.out + (long long)(y0 + j) * sd.out_pitch + x;
        *p = stretch_pixel(*p, lo, hi);
    }
}

// Descriptors of the paper's image partitions: `parts` horizontal strips, strip i = rows
// [floor(i h / parts), floor((i + 1) h / parts)), each an image of its own (AMF input `in`,
// AMF output `out`), tiles numbered strip after strip.
__global__ void strip_table_kernel(SliceDesc *table, const unsigned char *in, unsigned char *out, int h,
                                   int w, long long in_pitch, long long out_pitch, int eb, int parts) {
    const int i = threadIdx.x;
    if (i >= parts) return;
    const int tx = (w + TILE_X - 1) / TILE_X;
    int begin = 0;
    for (int j = 0; j < i; ++j) {
        const int hj = (int)((long long)(j + 1) * h / parts) - (int)((long long)j * h / parts);
        begin += tx * ((hj + TILE_Y - 1) / TILE_Y);
    }
    const int r0 = (int)((long long)i * h / parts), r1 = (int)((long long)(i + 1) * h / parts);
    SliceDesc d;
    d.in = in + (long long)r0 * in_pitch * eb;
    d.amf = out + (long long)r0 * out_pitch * eb;
    d.out = nullptr;
    d.in_pitch = in_pitch;
    d.amf_pitch = out_pitch;
    d.out_pitch = 0;
    d.h = r1 - r0;
    d.w = w;
    d.tiles_x = tx;
    d.tile_begin = begin;
    table[i] = d;
}

__global__ void fill_f64_kernel(double *p, double v) {
    if (threadIdx.x == 0) *p = v;
}

__global__ __launch_bounds__(256) void zero_u32_kernel(unsigned int *p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

hipError_t launch_strip_table(SliceDesc *table, const void *in, void *out, int h, int w,
                              long long in_pitch, long long out_pitch, int eb, int parts, hipStream_t s) {
    hipLaunchKernelGGL(strip_table_kernel, dim3(1), dim3(256), 0, s, table, (const unsigned char *)in,
                       (unsigned char *)out, h, w, in_pitch, out_pitch, eb, parts);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const SliceSet &set, int total_tiles, unsigned long long *tile_ranges,
                              hipStream_t s) {
    hipLaunchKernelGGL(tile_range_kernel, dim3(total_tiles), dim3(256), 0, s, set, total_tiles, tile_ranges);
    return hipGetLastError();
}

hipError_t launch_stretch(const SliceSet &set, int total_tiles, const unsigned long long *tile_ranges,
                          unsigned long long *slice_ranges, hipStream_t s) {
    hipLaunchKernelGGL(range_reduce_kernel, dim3(set.n), dim3(256), 0, s, set, tile_ranges, slice_ranges);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stretch_kernel, dim3(total_tiles), dim3(256), 0, s, set, total_tiles, slice_ranges);
    return hipGetLastError();
}

hipError_t launch_noise_reduce(const SliceSet &set, const unsigned long long *partials,
                               int wh, int ww, double *nu2, hipStream_t s) {
    hipLaunchKernelGGL(noise_reduce_kernel, dim3(set.n), dim3(256), 0, s, set, partials, wh, ww, nu2);
    return hipGetLastError();
}

hipError_t launch_wiener_stage(const SliceSet &set, int total_tiles, int eb, int max_value,
                               int wh, int ww, bool apply, const double *nu2, double noise_var,
                               unsigned long long *partials, bool aligned, hipStream_t s,
                               unsigned long long *ranges) {
    const dim3 grid(total_tiles), block(NT);
    const int smem = wiener_smem_bytes(eb, wh, ww);
    const float mf = (float)max_value;  // exact: max_value <= 65535
    const WienerConst wcb = wiener_const(wh, ww, mf);
    const int al = aligned ? 1 : 0;
    if (wh == ww && (wh == 3 || wh == 5 || wh == 7)) {
        // square 3 / 5 / 7 windows: one wave per tile, row sums in registers, LDS for the
        // region only (the row-sum helpers read up to 3 bytes past a window: 16 bytes of slack)
        const int rsm = (TILE_Y + 2 * (wh / 2)) * ((15 + (TILE_X + 2 * (wh / 2)) * eb + 15) / 16) * 16 + 16;
#define HD_LAUNCH_SQ(TY, AP, WN)                                                                               \
    hipLaunchKernelGGL((wiener_column_kernel<TY, AP, WN>), grid, dim3(64), rsm, s, set, total_tiles, nu2, noise_var, \
                       partials, al, ranges, wcb)
#define HD_LAUNCH_SQ_W(TY, AP)            \
    do {                                  \
        if (wh == 3) HD_LAUNCH_SQ(TY, AP, 3); \
        else if (wh == 5) HD_LAUNCH_SQ(TY, AP, 5); \
        else HD_LAUNCH_SQ(TY, AP, 7);     \
    } while (0)
        if (eb == 1) {
            if (apply) HD_LAUNCH_SQ_W(uint8_t, true);
            else HD_LAUNCH_SQ_W(uint8_t, false);
        } else {
            if (apply) HD_LAUNCH_SQ_W(uint16_t, true);
            else HD_LAUNCH_SQ_W(uint16_t, false);
        }
#undef HD_LAUNCH_SQ_W
#undef HD_LAUNCH_SQ
        return hipGetLastError();
    }
    if (eb == 1) {
        if (apply)
            hipLaunchKernelGGL((wiener_stage_kernel<uint8_t, true>), grid, block, smem, s, set,
                               total_tiles, wh, ww, mf, nu2, noise_var, partials, al, ranges, wcb);
        else
            hipLaunchKernelGGL((wiener_stage_kernel<uint8_t, false>), grid, block, smem, s, set,
                               total_tiles, wh, ww, mf, nu2, noise_var, partials, al, ranges, wcb);
    } else {
        if (apply)
            hipLaunchKernelGGL((wiener_stage_kernel<uint16_t, true>), grid, block, smem, s, set,
                               total_tiles, wh, ww, mf, nu2, noise_var, partials, al, ranges, wcb);
        else
            hipLaunchKernelGGL((wiener_stage_kernel<uint16_t, false>), grid, block, smem, s, set,
                               total_tiles, wh, ww, mf, nu2, noise_var, partials, al, ranges, wcb);
    }
    return hipGetLastError();
}

}  // namespace hd

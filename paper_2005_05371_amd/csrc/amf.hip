// Stage 1 of the hybrid de-noiser on gfx950: adaptive median filter (AMF), optionally
// fused with the exact Wiener noise-power partial sums of each tile.
//
// Method (arXiv 2005.05371, Alg. 1, procedure parallelAdapMedian): for every pixel try
// windows k = 3, 5, ..., Smax in order; at level k take zmin, zmax, zmed of the k x k
// window; stage A passes when zmin < zmed < zmax and resolves the pixel: it keeps g when
// zmin < g < zmax (stage B), else takes zmed. A pixel never passing stage A takes zmed of
// the Smax window (or keeps g in keep mode).
//
// Design (one workgroup of 256 threads per 64 x 32 output tile):
//  * the input region (tile + Wiener ring + Smax/2 halo, symmetric padding) is staged in
//    LDS in the image's own element type with 16-byte loads;
//  * level 3 runs for every pixel with a register network: a thread owns a strip of 8
//    pixels in one column, sorts each row triple once (min3 / med3 / max3, shared by the
//    three pixels whose windows contain that row) and takes zmin, zmax and zmed of the
//    3 x 3 window from the row triples (median of 9 = med3 of: the largest row minimum,
//    the median of the row medians, the smallest row maximum);
//  * pixels failing stage A are compacted into an LDS list (wave ballot + one LDS atomic
//    per wave). Each deeper level runs only over that list, with every lane busy, and
//    splits it into: resolved (centre kept), still unresolved (next list) and pixels that
//    need zmed (a second list, so the expensive selection also runs with full lanes);
//  * at levels >= 5 stage A is decided from counts, without sorting: zmed > zmin iff at
//    most (k^2 - 1) / 2 samples equal zmin, and zmed < zmax iff at most (k^2 - 1) / 2
//    samples equal zmax. zmed is exact: a pruned Batcher odd-even merge network in
//    registers for 5 x 5 and 7 x 7, and bisection over the value range above (the
//    smallest t with #(v <= t) > (k^2 - 1) / 2);
//  * with the Wiener fusion, AMF also runs on the window ring around the tile and the
//    tile's exact sum of N * S2 - S1^2 is written to partials[tile] (no atomics).
#include "tile_io.h"

namespace hd {
namespace {

constexpr int NT = STAGE_THREADS;
constexpr int RPT = 8;  // rows per strip in the level-3 pass
// pending lists up to this length go through the deep levels one wave per pixel
constexpr int SPARSE_DEEP = 24;

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) { return min(min(a, b), c); }
__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) { return max(max(a, b), c); }
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}

// Batcher odd-even merge sort of N (power of two) registers; unused outputs are pruned
// by the compiler when only one rank is read.
template <int N>
__device__ __forceinline__ void batcher_sort(uint32_t (&v)[N]) {
#pragma unroll
    for (int p = 1; p < N; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const uint32_t a = v[i + j], b = v[i + j + k];
                        v[i + j] = min(a, b);
                        v[i + j + k] = max(a, b);
                    }
}

// Exact median of the K x K window centred at c (LDS, row pitch lp) through a sorting
// network over NP >= K*K registers padded with 0 below and 0xffff above.
template <typename T, int K, int NP>
__device__ __forceinline__ uint32_t median_network(const T *c, int lp) {
    constexpr int n = K * K, r = K / 2, plo = (NP - n) / 2;
    uint32_t v[NP];
#pragma unroll
    for (int i = 0; i < plo; ++i) v[i] = 0u;
#pragma unroll
    for (int i = plo + n; i < NP; ++i) v[i] = 0xffffu;
#pragma unroll
    for (int dy = 0; dy < K; ++dy)
#pragma unroll
        for (int dx = 0; dx < K; ++dx) v[plo + dy * K + dx] = c[(dy - r) * lp + dx - r];
    batcher_sort<NP>(v);
    return v[plo + (n - 1) / 2];
}

// Exact rank-(k^2-1)/2 element by bisection: smallest t in [lo, hi] with #(v <= t) > half.
template <typename T, int K>
__device__ uint32_t median_bisect(const T *c, int lp, uint32_t lo, uint32_t hi) {
    constexpr int r = K / 2;
    constexpr uint32_t half = (K * K - 1) / 2;
    constexpr int UR = (K <= 5) ? K : 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        uint32_t cnt = 0;
#pragma unroll UR
        for (int dy = -r; dy <= r; ++dy) {
            const T *row = c + dy * lp;
#pragma unroll
            for (int dx = -r; dx <= r; ++dx) cnt += (uint32_t(row[dx]) <= mid);
        }
        if (cnt > half) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Stage-A statistics of the K x K window: min, max and their multiplicities.
template <typename T, int K>
__device__ __forceinline__ void window_stats(const T *c, int lp, uint32_t &mn, uint32_t &mx,
                                             uint32_t &cmin, uint32_t &cmax) {
    constexpr int r = K / 2;
    constexpr int UR = (K <= 5) ? K : 1;
    mn = 0xffffffffu;
    mx = 0u;
#pragma unroll UR
    for (int dy = -r; dy <= r; ++dy) {
        const T *row = c + dy * lp;
#pragma unroll
        for (int dx = -r; dx <= r; ++dx) {
            const uint32_t v = row[dx];
            mn = min(mn, v);
            mx = max(mx, v);
        }
    }
    cmin = 0;
    cmax = 0;
#pragma unroll UR
    for (int dy = -r; dy <= r; ++dy) {
        const T *row = c + dy * lp;
#pragma unroll
        for (int dx = -r; dx <= r; ++dx) {
            const uint32_t v = row[dx];
            cmin += (v == mn);
            cmax += (v == mx);
        }
    }
}

// Level k >= 5, step 1. Returns 0: resolved (value in out), 1: unresolved, go on,
// 2: zmed needed (resolved with the median, or the last level in median mode).
template <typename T, int K>
__device__ int level_test(const T *c, int lp, bool last, bool keep, uint32_t &out) {
    constexpr uint32_t half = (K * K - 1) / 2;
    uint32_t mn, mx, cmin, cmax;
    window_stats<T, K>(c, lp, mn, mx, cmin, cmax);
    const uint32_t g = *c;
    const bool stage_a = (cmin <= half) && (cmax <= half);
    if (stage_a) {
        if (g != mn && g != mx) {  // stage B: centre strictly inside (zmin, zmax)
            out = g;
            return 0;
        }
        out = (mn + 1) | ((mx - 1) << 16);  // bisection bracket for the median
        return 2;
    }
    if (!last) return 1;
    if (keep) {
        out = g;
        return 0;
    }
    out = mn | (mx << 16);
    return 2;
}

// Level k >= 5, step 2: the exact median (networks for 5x5 / 7x7 in the dense variant).
template <typename T, int K, bool DENSE>
__device__ uint32_t level_median(const T *c, int lp, uint32_t bracket) {
    if constexpr (DENSE) {
        if constexpr (K == 5) return median_network<T, 5, 32>(c, lp);
        if constexpr (K == 7) return median_network<T, 7, 64>(c, lp);
    }
    return median_bisect<T, K>(c, lp, bracket & 0xffffu, bracket >> 16);
}

// ---- one wave per pixel (sparse deep levels) ----------------------------------------
// The k*k window of one pixel is spread over the 64 lanes (element e = lane + 64 s).
// zmin / zmax come from one packed 16-bit max reduction of (0xffff - v, v); the counts of
// zmin and zmax from ballots; zmed from a ballot radix select over the bits below the
// common prefix of zmin and zmax. Control flow is uniform across the wave.
__device__ __forceinline__ uint32_t pk_max_u16(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned short, a),
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned short, b)));
}

// Returns 0: resolved (value in out), 1: unresolved, go on.
template <typename T, int K>
__device__ int wave_level(const T *c, int lp, bool last, bool keep, uint32_t &out) {
    constexpr int N = K * K, SL = (N + 63) / 64, r = K / 2;
    constexpr uint32_t half = (N - 1) / 2;
    const int lane = threadIdx.x & 63;
    const uint32_t g = *c;
    uint32_t v[SL];
    unsigned long long valid[SL];
    uint32_t key = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const int e = lane + 64 * s;
        const bool ok = e < N;
        const int dy = e / K, dx = e - (e / K) * K;
        v[s] = ok ? (uint32_t)c[(dy - r) * lp + dx - r] : g;  // g is inside the window
        valid[s] = __ballot(ok);
        key = pk_max_u16(key, ((0xffffu - v[s]) << 16) | v[s]);
    }
    // wave-wide packed max: butterfly inside each 16-lane row (DPP: quad permutes, row
    // rotations), then the four row results through scalar registers
    key = pk_max_u16(key, (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, 0xB1, 0xF, 0xF, false));
    key = pk_max_u16(key, (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x4E, 0xF, 0xF, false));
    key = pk_max_u16(key, (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x124, 0xF, 0xF, false));
    key = pk_max_u16(key, (uint32_t)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x128, 0xF, 0xF, false));
    uint32_t khi = 0, klo = 0;
#pragma unroll
    for (int row = 0; row < 4; ++row) {
        const uint32_t kr = (uint32_t)__builtin_amdgcn_readlane((int)key, 16 * row);
        khi = max(khi, kr >> 16);
        klo = max(klo, kr & 0xffffu);
    }
    const uint32_t mn = 0xffffu - khi, mx = klo;
    uint32_t cmin = 0, cmax = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        cmin += __popcll(__ballot(v[s] == mn) & valid[s]);
        cmax += __popcll(__ballot(v[s] == mx) & valid[s]);
    }
    const bool stage_a = (cmin <= half) && (cmax <= half);
    if (stage_a && g != mn && g != mx) {
        out = g;
        return 0;
    }
    if (!stage_a && !last) return 1;
    if (!stage_a && keep) {
        out = g;
        return 0;
    }
    // exact element of rank `half`: bits above the highest bit where mn and mx differ are
    // shared by every sample; walk the remaining bits from the top, keeping the side
    // that holds the rank
    const int hb = (mn == mx) ? -1 : 31 - __clz(mn ^ mx);
    uint32_t prefix = (hb >= 0) ? (mn & ~((2u << hb) - 1u)) : mn;
    unsigned long long cand[SL];
#pragma unroll
    for (int s = 0; s < SL; ++s) cand[s] = valid[s];
    uint32_t rank = half;
    for (int b = hb; b >= 0; --b) {
        uint32_t zeros = 0;
        unsigned long long zm[SL];
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            zm[s] = __ballot(((v[s] >> b) & 1u) == 0u);
            zeros += __popcll(cand[s] & zm[s]);
        }
        if (rank < zeros) {
#pragma unroll
            for (int s = 0; s < SL; ++s) cand[s] &= zm[s];
        } else {
            rank -= zeros;
            prefix |= 1u << b;
#pragma unroll
            for (int s = 0; s < SL; ++s) cand[s] &= ~zm[s];
        }
    }
    out = prefix;
    return 0;
}

// Wave mode covers windows up to 15 x 15 (at most 4 samples per lane); larger windows
// always take the per-lane path.
template <typename T>
__device__ int wave_level_k(int k, const T *c, int lp, bool last, bool keep, uint32_t &out) {
    switch (k) {
        case 5: return wave_level<T, 5>(c, lp, last, keep, out);
        case 7: return wave_level<T, 7>(c, lp, last, keep, out);
        case 9: return wave_level<T, 9>(c, lp, last, keep, out);
        case 11: return wave_level<T, 11>(c, lp, last, keep, out);
        case 13: return wave_level<T, 13>(c, lp, last, keep, out);
        default: return wave_level<T, 15>(c, lp, last, keep, out);
    }
}

template <typename T>
__device__ int level_test_k(int k, const T *c, int lp, bool last, bool keep, uint32_t &out) {
    switch (k) {
        case 5: return level_test<T, 5>(c, lp, last, keep, out);
        case 7: return level_test<T, 7>(c, lp, last, keep, out);
        case 9: return level_test<T, 9>(c, lp, last, keep, out);
        case 11: return level_test<T, 11>(c, lp, last, keep, out);
        case 13: return level_test<T, 13>(c, lp, last, keep, out);
        case 15: return level_test<T, 15>(c, lp, last, keep, out);
        case 17: return level_test<T, 17>(c, lp, last, keep, out);
        case 19: return level_test<T, 19>(c, lp, last, keep, out);
        case 21: return level_test<T, 21>(c, lp, last, keep, out);
        case 23: return level_test<T, 23>(c, lp, last, keep, out);
        case 25: return level_test<T, 25>(c, lp, last, keep, out);
        case 27: return level_test<T, 27>(c, lp, last, keep, out);
        case 29: return level_test<T, 29>(c, lp, last, keep, out);
        default: return level_test<T, 31>(c, lp, last, keep, out);
    }
}

template <typename T, bool DENSE>
__device__ uint32_t level_median_k(int k, const T *c, int lp, uint32_t bracket) {
    switch (k) {
        case 5: return level_median<T, 5, DENSE>(c, lp, bracket);
        case 7: return level_median<T, 7, DENSE>(c, lp, bracket);
        case 9: return level_median<T, 9, DENSE>(c, lp, bracket);
        case 11: return level_median<T, 11, DENSE>(c, lp, bracket);
        case 13: return level_median<T, 13, DENSE>(c, lp, bracket);
        case 15: return level_median<T, 15, DENSE>(c, lp, bracket);
        case 17: return level_median<T, 17, DENSE>(c, lp, bracket);
        case 19: return level_median<T, 19, DENSE>(c, lp, bracket);
        case 21: return level_median<T, 21, DENSE>(c, lp, bracket);
        case 23: return level_median<T, 23, DENSE>(c, lp, bracket);
        case 25: return level_median<T, 25, DENSE>(c, lp, bracket);
        case 27: return level_median<T, 27, DENSE>(c, lp, bracket);
        case 29: return level_median<T, 29, DENSE>(c, lp, bracket);
        default: return level_median<T, 31, DENSE>(c, lp, bracket);
    }
}

template <typename T>
struct Sq;
template <>
struct Sq<uint8_t> { using type = uint32_t; };
template <>
struct Sq<uint16_t> { using type = unsigned long long; };

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <typename T, bool DENSE>
__global__ __launch_bounds__(NT) void amf_stage_kernel(SliceSet set, int total_tiles, int smax,
                                                       int keep, int wh, int ww,
                                                       unsigned long long *__restrict__ partials,
                                                       int select_mode, int aligned) {
    using S2T = typename Sq<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_cnt[3];
    __shared__ unsigned long long s_wsum[NT / 64];

    int tile;
    if (set.list) {  // listed tiles only (uniform early exit for the spare blocks)
        if ((int)blockIdx.x >= *set.list_count) return;
        tile = set.list[blockIdx.x];
    } else {
        tile = xcd_remap(blockIdx.x, total_tiles);
    }
    const SliceDesc sd = slice_desc(set, slice_index(set, tile));
    const int H = sd.h, W = sd.w;
    const int lt = tile - sd.tile_begin;
    const int ty = lt / sd.tiles_x;
    const int x0 = (lt - ty * sd.tiles_x) * TILE_X;
    const int y0 = ty * TILE_Y;
    const bool moments = wh > 0;
    const AmfSmem L = amf_smem_layout((int)sizeof(T), smax, moments ? wh : 0, moments ? ww : 0);
    const int R = L.R, rh = L.rh, rw = L.rw, AH = L.AH, AW = L.AW;
    const int ry0 = y0 - rh, rx0 = x0 - rw;  // image position of AMF-region element (0, 0)

    T *s_amf = (T *)smem;
    unsigned char *u = smem + L.amf_bytes;
    T *s_in = (T *)u;
    uint16_t *s_list = (uint16_t *)(u + L.in_bytes);  // two lists of AH * AW entries
    const int cap = AH * AW;

    const int tid = threadIdx.x, lane = tid & 63;

    // 1. input region -> LDS
    const Staged st = stage_region<T>(s_in, (const T *)sd.in, H, W, sd.in_pitch, ry0 - R, rx0 - R,
                                      L.IH, AW + 2 * R, aligned != 0);
    const int lp = st.lpt;
    const T *in0 = s_in + R * lp + st.off + R;  // centre of AMF-region element (0, 0)
    if (tid < 3) s_cnt[tid] = 0;
    __syncthreads();

    // 2. level 3 for every pixel of the AMF region: strips of RPT rows, one column each
    const bool last3 = (smax == 3);
    const int nstrip = (AH + RPT - 1) / RPT;
    const int nitems = nstrip * AW;
    const int mAW = div_region_magic(AW);
    for (int item = tid; item < nitems; item += NT) {
        const int s = div_region(item, mAW);
        const int cx = item - s * AW;
        const int rb = s * RPT;
        uint32_t lo[RPT + 2], md[RPT + 2], hi[RPT + 2], ctr[RPT + 2];
        const T *p0 = in0 + (rb - 1) * lp + cx;
#pragma unroll
        for (int j = 0; j < RPT + 2; ++j) {
            // every row of the strip (and one above / below) lies in the staged region
            const T *p = p0 + j * lp;
            const uint32_t a = p[-1], b = p[0], c = p[1];
            lo[j] = min3u(a, b, c);
            md[j] = med3u(a, b, c);
            hi[j] = max3u(a, b, c);
            ctr[j] = b;
        }
        const int gx = rx0 + cx;
        // rows of this strip that are real image pixels inside the AMF region
        const int gy0 = ry0 + rb;
        const int rlo = max(0, -gy0), rhi = min(min(RPT, AH - rb), H - gy0);
        const bool col_ok = gx >= 0 && gx < W && !last3;
        uint32_t defer = 0;
        T *dst = s_amf + rb * AW + cx;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const uint32_t zmin = min3u(lo[j], lo[j + 1], lo[j + 2]);
            const uint32_t zmax = max3u(hi[j], hi[j + 1], hi[j + 2]);
            const uint32_t zmed = med3u(max3u(lo[j], lo[j + 1], lo[j + 2]),
                                        med3u(md[j], md[j + 1], md[j + 2]),
                                        min3u(hi[j], hi[j + 1], hi[j + 2]));
            const uint32_t g = ctr[j + 1];
            const bool stage_a = (zmin < zmed) && (zmed < zmax);
            const bool centre_ok = (zmin < g) && (g < zmax);
            // stage A: g when stage B passes, else zmed; no stage A: final only when
            // Smax == 3 (zmed, or g in keep mode)
            const uint32_t res = (stage_a ? centre_ok : (keep != 0)) ? g : zmed;
            dst[j * AW] = (T)res;
            defer |= (uint32_t)(!stage_a) << j;
        }
        // keep rows [rlo, rhi) only (0 <= rlo <= 7, rhi <= RPT; empty when rhi <= rlo)
        defer = (col_ok && rhi > rlo) ? (defer & ((1u << rhi) - 1u) & ~((1u << rlo) - 1u)) : 0u;
        if (defer) {  // rare outside dense impulse noise: one LDS atomic per lane
            int pos = atomicAdd(&s_cnt[0], __popc(defer));
            while (defer) {
                const int j = __ffs(defer) - 1;
                defer &= defer - 1;
                s_list[pos++] = (uint16_t)((rb + j) * AW + cx);
            }
        }
    }
    __syncthreads();

    // 3. deeper levels. A short pending list (a few pixels, typical of moderate impulse
    //    densities) is run pixel by pixel, one wave per pixel through all its levels, with
    //    no barrier between levels. Otherwise level by level over compacted lists: list A
    //    = s_list[cur*cap ...]; list B holds the next level's pixels from the front and
    //    the zmed pixels from the back.
    int cur = 0;
    const int n0 = s_cnt[0];
    const bool sparse = smax <= 15 && n0 <= SPARSE_DEEP &&
                        (select_mode == SELECT_AUTO || select_mode == SELECT_DENSE);
    if (n0 > 0 && sparse) {
        for (int i = tid >> 6; i < n0; i += NT / 64) {
            const int idx = s_list[i];
            const int r = div_region(idx, mAW), cx = idx - r * AW;
            const T *c = in0 + r * lp + cx;
            uint32_t v = 0;
            for (int k = 5; k <= smax; k += 2)
                if (wave_level_k<T>(k, c, lp, k == smax, keep != 0, v) == 0) break;
            if (lane == 0) s_amf[idx] = (T)v;
        }
        __syncthreads();
    }
    for (int k = 5; k <= smax && !sparse; k += 2) {
        const int n = s_cnt[cur];
        if (n == 0) break;  // uniform: read after a barrier
        const int nxt = cur ^ 1;
        const bool last = (k == smax);
        uint16_t *la = s_list + cur * cap;
        uint16_t *lb = s_list + nxt * cap;
        // per-lane when the list fills the lanes (or bisection is forced), else one wave
        // per pixel; the choice is uniform across the workgroup
        const bool wave_mode = k <= 15 && (select_mode == SELECT_WAVE ||
                                           ((select_mode == SELECT_AUTO || select_mode == SELECT_DENSE) &&
                                            n < (DENSE && k <= 7 ? 64 : NT)));
        if (wave_mode) {
            for (int i = tid >> 6; i < n; i += NT / 64) {
                const int idx = la[i];
                const int r = div_region(idx, mAW), cx = idx - r * AW;
                uint32_t v = 0;
                const int outcome = wave_level_k<T>(k, in0 + r * lp + cx, lp, last, keep != 0, v);
                if (lane == 0) {
                    if (outcome == 0) s_amf[idx] = (T)v;
                    else lb[atomicAdd(&s_cnt[nxt], 1)] = (uint16_t)idx;
                }
            }
            __syncthreads();
            if (tid == 0) s_cnt[cur] = 0;
            __syncthreads();
            cur = nxt;
            continue;
        }
        for (int i = tid; i < n; i += NT) {
            const int idx = la[i];
            const int r = div_region(idx, mAW), cx = idx - r * AW;
            const T *c = in0 + r * lp + cx;
            uint32_t v = 0;
            const int outcome = level_test_k<T>(k, c, lp, last, keep != 0, v);
            if (outcome == 0) {
                s_amf[idx] = (T)v;
            } else if (outcome == 1) {
                lb[atomicAdd(&s_cnt[nxt], 1)] = (uint16_t)idx;
            } else {
                const int pos = cap - 1 - atomicAdd(&s_cnt[2], 1);
                lb[pos] = (uint16_t)idx;
                // the bisection bracket is recomputed from the window in step 2
                (void)v;
            }
        }
        __syncthreads();
        const int m = s_cnt[2];
        for (int i = tid; i < m; i += NT) {
            const int idx = lb[cap - 1 - i];
            const int r = div_region(idx, mAW), cx = idx - r * AW;
            const T *c = in0 + r * lp + cx;
            uint32_t bracket = 0;
            if (!DENSE || k > 7) {
                uint32_t mn, mx, cmin, cmax;
                (void)cmin; (void)cmax;
                // bracket [mn, mx]: always contains the median
                mn = 0xffffffffu; mx = 0u;
                const int rk = k / 2;
                for (int dy = -rk; dy <= rk; ++dy)
                    for (int dx = -rk; dx <= rk; ++dx) {
                        const uint32_t e = c[dy * lp + dx];
                        mn = min(mn, e);
                        mx = max(mx, e);
                    }
                bracket = mn | (mx << 16);
            }
            s_amf[idx] = (T)level_median_k<T, DENSE>(k, c, lp, bracket);
        }
        __syncthreads();
        if (tid == 0) {
            s_cnt[cur] = 0;
            s_cnt[2] = 0;
        }
        __syncthreads();
        cur = nxt;
    }

    // 4. the tile's AMF output -> global. A listed tile also stores the AMF of its ring:
    //    the Wiener stage of that tile reads it whether or not the neighbour is listed
    //    (a listed neighbour writes the same values).
    if (set.list) {
        for (int r = tid >> 6; r < AH; r += NT / 64) {
            const int gy = ry0 + r;
            if (gy < 0 || gy >= H) continue;
            T *dst = (T *)sd.amf + (long long)gy * sd.amf_pitch;
            for (int c = lane; c < AW; c += 64) {
                const int gx = rx0 + c;
                if (gx >= 0 && gx < W) dst[gx] = s_amf[r * AW + c];
            }
        }
    } else {
        store_region<T>((T *)sd.amf, H, W, sd.amf_pitch, y0, x0, s_amf + rh * AW + rw, AW,
                        TILE_Y, min(TILE_X, W - x0), aligned != 0);
    }
    if (!moments) return;

    // 5. exact Wiener variance numerators of the tile's pixels from the AMF region.
    //    Window positions outside the image are mirrored back inside; their AMF values sit
    //    in the region because the ring is at least the window radius wide.
    __syncthreads();  // lists / input region are dead: reuse them for the row sums
    uint32_t *h1 = (uint32_t *)u;
    S2T *h2 = (S2T *)(u + AH * TILE_X * 4);
    const bool in_x = rx0 >= 0 && x0 + TILE_X + rw <= W;
    for (int r = tid >> 6; r < AH; r += NT / 64) {
        const int gy = ry0 + r;
        if (gy < 0 || gy >= H) continue;  // rows outside the image are read through mirror()
        const T *row = s_amf + r * AW;
        uint32_t t1 = 0;
        S2T t2 = 0;
        const int gxc = x0 + lane;
        if (gxc >= W) continue;  // no output column here
        if (in_x) {
            for (int dx = 0; dx < ww; ++dx) {
                const uint32_t v = row[lane + dx];
                t1 += v;
                t2 += (S2T)v * v;
            }
        } else {
            for (int dx = -rw; dx <= rw; ++dx) {
                const uint32_t v = row[mirror(gxc + dx, W) - rx0];
                t1 += v;
                t2 += (S2T)v * v;
            }
        }
        h1[r * TILE_X + lane] = t1;
        h2[r * TILE_X + lane] = t2;
    }
    __syncthreads();
    // N * S2 - S1^2 fits 32 bits for 8-bit data, 64 bits for 16-bit data
    const S2T nwin = (S2T)(wh * ww);
    unsigned long long tsum = 0;
    const int wv = tid >> 6;
    const bool in_y = ry0 >= 0 && y0 + TILE_Y + rh <= H;
    if (x0 + lane < W) {
        const int rows = min(RPT, H - (y0 + wv * RPT));
        for (int j = 0; j < rows; ++j) {
            const int rr = wv * RPT + j;  // tile row
            const int gy = y0 + rr;
            uint32_t s1 = 0;
            S2T s2 = 0;
            if (in_y) {
                for (int dy = 0; dy < wh; ++dy) {
                    s1 += h1[(rr + dy) * TILE_X + lane];
                    s2 += h2[(rr + dy) * TILE_X + lane];
                }
            } else {
                for (int dy = -rh; dy <= rh; ++dy) {
                    const int ri = mirror(gy + dy, H) - ry0;
                    s1 += h1[ri * TILE_X + lane];
                    s2 += h2[ri * TILE_X + lane];
                }
            }
            tsum += (unsigned long long)(nwin * s2 - (S2T)s1 * s1);
        }
    }
    tsum = wave_sum_u64(tsum);
    if (lane == 0) s_wsum[wv] = tsum;
    __syncthreads();
    if (tid == 0) {
        unsigned long long b = 0;
        for (int i = 0; i < NT / 64; ++i) b += s_wsum[i];
        partials[tile] = b;
    }
}

}  // namespace

hipError_t launch_amf_stage(const SliceSet &set, int total_tiles, int eb, int smax, int keep,
                            int wh, int ww, unsigned long long *partials, int select_mode,
                            bool aligned, hipStream_t s) {
    const AmfSmem L = amf_smem_layout(eb, smax, wh, ww);
    const dim3 grid(total_tiles), block(NT);
    const bool dense = select_mode == SELECT_DENSE;
    const int al = aligned ? 1 : 0;
    if (eb == 1) {
        if (dense)
            hipLaunchKernelGGL((amf_stage_kernel<uint8_t, true>), grid, block, L.total, s, set, total_tiles, smax,
                               keep, wh, ww, partials, select_mode, al);
        else
            hipLaunchKernelGGL((amf_stage_kernel<uint8_t, false>), grid, block, L.total, s, set, total_tiles, smax,
                               keep, wh, ww, partials, select_mode, al);
    } else {
        if (dense)
            hipLaunchKernelGGL((amf_stage_kernel<uint16_t, true>), grid, block, L.total, s, set, total_tiles,
                               smax, keep, wh, ww, partials, select_mode, al);
        else
            hipLaunchKernelGGL((amf_stage_kernel<uint16_t, false>), grid, block, L.total, s, set, total_tiles,
                               smax, keep, wh, ww, partials, select_mode, al);
    }
    return hipGetLastError();
}

}  // namespace hd

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
//  * level 3 runs for every pixel with a register network: a thread owns a strip of 8 (12
//    in the resident kernel) pixels in one column, sorts each row triple once (min3 / med3
//    / max3, shared by the three pixels whose windows contain that row) and takes zmin,
//    zmax and zmed of the 3 x 3 window from the row triples (median of 9 = med3 of: the
//    largest row minimum, the median of the row medians, the smallest row maximum);
//  * pixels failing stage A are compacted into an LDS list. A very short list goes through
//    all deeper levels four pixels per wave (one 16-lane DPP row each) up to level 11 and
//    one wave per pixel above. Otherwise the list runs level by level: one lane per pixel
//    when it fills the workgroup's lanes, else several pixels per wave (4-, 8-, 16- or 32-lane
//    groups, wider for larger windows); either way each level first sorts its pixels into
//    resolved, still unresolved (the next level's list) and needing zmed (the back of
//    that list), and then selects zmed for the last group only, packed densely;
//  * at levels >= 5 stage A is decided from counts, without sorting: zmed > zmin iff at
//    most (k^2 - 1) / 2 samples equal zmin, and zmed < zmax iff at most (k^2 - 1) / 2
//    samples equal zmax. zmed is exact: a radix select over ballots or row sums (one wave
//    or one row per pixel), bit bisection with group-wide counts (lane groups), a pruned
//    Batcher odd-even merge network in registers for 5 x 5 (dense variant), or bisection
//    over the value range (the smallest t with #(v <= t) > (k^2 - 1) / 2), per lane;
//  * with the Wiener fusion, AMF also runs on the window ring around the tile and the
//    tile's exact sum of N * S2 - S1^2 is written to partials[tile] (no atomics);
//  * the resident variant (every tile's workgroup on the device at once) keeps going after
//    that: a grid-wide exchange of the noise power (step 6 below), then the Wiener output
//    from the sums held in registers and the AMF still in LDS, in the same launch.
#include <algorithm>
#include <atomic>

#include "tile_io.h"

namespace hd {
namespace {

constexpr int NT = STAGE_THREADS;
constexpr int RPT = 8;  // rows per strip in the level-3 pass
// pending lists up to this length go through the deep levels one wave per pixel
constexpr int SPARSE_DEEP = 24;

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) { return min(min(a, b), c); }
__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) { return max(max(a, b), c); }
// min / median / max of three in one instruction each (the compiler does not always find
// them when the operands are shared with other min / max expressions)
__device__ __forceinline__ uint32_t med3_vop(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t min3_vop(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t max3_vop(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}

// ---- list appends with one LDS atomic per wave -------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wave, every lane active: row shifts by 1, 2,
// 4 and 8 within each 16-lane row, then the row totals through two row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}
// Slots for `cnt` entries per lane (every lane of the wave active) in a list whose length
// is *counter: returns this lane's first slot. One atomic add per wave.
__device__ __forceinline__ int wave_reserve(int *counter, uint32_t cnt) {
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    int base = 0;
    if (total != 0 && (threadIdx.x & 63) == 63) base = atomicAdd(counter, (int)total);
    base = __builtin_amdgcn_readlane(base, 63);
    return base + (int)(incl - cnt);
}
// One slot for each active lane with `take` (any lanes may be active): returns the lane's
// slot (unspecified where take is false). One atomic add per wave.
__device__ __forceinline__ int wave_take(int *counter, bool take) {
    const unsigned long long m = __ballot(take);
    const int before = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    int base = 0;
    if (m != 0) {
        const int leader = __ffsll((long long)m) - 1;
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(counter, __popcll(m));
        base = __builtin_amdgcn_readlane(base, leader);
    }
    return base + before;
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
        for (int dx = 0; dx < K; ++dx) v[plo + dy * K + dx] = (c - r * lp - r)[dy * lp + dx];
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
        for (int dy = 0; dy < K; ++dy) {
            const T *row = c + (dy - r) * lp - r;  // non-negative offsets within a row
#pragma unroll
            for (int dx = 0; dx < K; ++dx) cnt += (uint32_t(row[dx]) <= mid);
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
    for (int dy = 0; dy < K; ++dy) {
        const T *row = c + (dy - r) * lp - r;  // non-negative offsets within a row
#pragma unroll
        for (int dx = 0; dx < K; ++dx) {
            const uint32_t v = row[dx];
            mn = min(mn, v);
            mx = max(mx, v);
        }
    }
    cmin = 0;
    cmax = 0;
#pragma unroll UR
    for (int dy = 0; dy < K; ++dy) {
        const T *row = c + (dy - r) * lp - r;
#pragma unroll
        for (int dx = 0; dx < K; ++dx) {
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

// Level k >= 5, step 2: the exact median (a network for 5x5 in the dense variant).
template <typename T, int K, bool DENSE>
__device__ uint32_t level_median(const T *c, int lp, uint32_t bracket) {
    if constexpr (DENSE) {
        if constexpr (K == 5) return median_network<T, 5, 32>(c, lp);
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

// ---- several pixels per wave (levels 5 to 15 of the deep path) -----------------------
// A pixel owns a group of G lanes: 8 (half a DPP row, eight pixels per wave), 16 (a DPP
// row) or 32 (two rows); its k*k window is spread over the group (element e = j + G s for
// lane j of the group). Every quantity of a pixel is reduced inside its group (quad
// permutes, a half-row mirror, row rotations, folded into the reducing instruction where the
// operation allows, and a swizzle across the two rows of a 32-lane group), leaving the
// result in all of its lanes, so the pixels need no scalar work: zmin / zmax from one
// packed max, their counts from one packed sum, zmed by bisection on the bits of the value
// (the count below a threshold is a group sum). Small groups keep the per-bit reduction
// short relative to the per-sample work; larger ones keep the samples per lane (registers)
// few for the large windows.
// Group size of the level-by-level passes (at most 13 samples per lane: the passes are
// functions of their own, and the kernel reserves the registers of the largest of them):
// 4 lanes at level 7 in the staged kernel (13 samples each: the 49-sample median's bit
// bisection costs fewer instructions per pixel than with 8 lanes), 8 up to level 9, then
// 16 and 32. The single-launch kernel, whose register count sets how many tiles fit the
// device at once, takes 16 lanes up to level 11, as does the short-list path.
template <int K, bool RESIDENT>
constexpr int pass_group() {
    return (!RESIDENT && K == 7) ? 4 : (K <= (RESIDENT ? 0 : 9) ? 8 : (K <= 11 ? 16 : 32));
}

template <int K, int G>
struct DeepGroup {
    static constexpr int LANES = G;
    static constexpr int PER_WAVE = 64 / LANES;
    static constexpr int N = K * K;
    static constexpr int SL = (N + LANES - 1) / LANES;
    static_assert(SL <= 13, "at most 13 samples per lane");
};

// Pointer into LDS (address space 3): the deep-level passes are separate functions, and
// this keeps their window reads 32-bit LDS reads rather than generic 64-bit ones.
#define HD_LDS __attribute__((address_space(3)))

// x combined with the value of the lane the DPP control selects (bound_ctrl set; every
// pattern used here selects a lane of the same row)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, true);
}
constexpr int DPP_QUAD_SWAP1 = 0xB1;     // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_SWAP2 = 0x4E;     // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;   // row_half_mirror: lane i <-> 7 - i in each 8 lanes
constexpr int DPP_ROW_ROR4 = 0x124;      // row_ror:4
constexpr int DPP_ROW_ROR8 = 0x128;      // row_ror:8
__device__ __forceinline__ uint32_t swap_rows(uint32_t x) {
    // lane i <-> lane i ^ 16 within each 32 lanes (bit-mask swizzle: and 0x1f, xor 0x10)
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401f);
}
template <int G>
__device__ __forceinline__ uint32_t group_max_pk(uint32_t x) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 32, "group size");
    x = pk_max_u16(x, dpp<DPP_QUAD_SWAP1>(x));
    x = pk_max_u16(x, dpp<DPP_QUAD_SWAP2>(x));
    if constexpr (G == 4) return x;
    if constexpr (G == 8) return pk_max_u16(x, dpp<DPP_HALF_MIRROR>(x));
    x = pk_max_u16(x, dpp<DPP_ROW_ROR4>(x));
    x = pk_max_u16(x, dpp<DPP_ROW_ROR8>(x));
    if constexpr (G == 32) x = pk_max_u16(x, swap_rows(x));
    return x;
}
template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t x) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 32, "group size");
    x += dpp<DPP_QUAD_SWAP1>(x);
    x += dpp<DPP_QUAD_SWAP2>(x);
    if constexpr (G == 4) return x;
    if constexpr (G == 8) return x + dpp<DPP_HALF_MIRROR>(x);
    x += dpp<DPP_ROW_ROR4>(x);
    x += dpp<DPP_ROW_ROR8>(x);
    if constexpr (G == 32) x += swap_rows(x);
    return x;
}

// LDS offsets (relative to a pixel's centre, row pitch lp) of the window samples that lane
// j of a group holds at level K: sample s is window element e = j + 8 s in row-major
// order. Slots past the window's k^2 elements point at the centre (they are masked out).
template <int K, int G>
struct GroupOffsets {
    using D = DeepGroup<K, G>;
    int off[D::SL];
    __device__ __forceinline__ explicit GroupOffsets(int lp) {
        const int j = threadIdx.x & (D::LANES - 1);
        constexpr int r = K / 2;
#pragma unroll
        for (int s = 0; s < D::SL; ++s) {
            const int e = j + D::LANES * s;
            const int dy = e / K, dx = e - dy * K;
            off[s] = (s < D::SL - 1 || e < D::N) ? (dy - r) * lp + dx - r : 0;
        }
    }
};

// Number of the samples below t, two 16-bit samples per register (t <= 0xffff; a half
// holding 0xffff never counts): per register a saturating t - v, capped at 1, summed per
// half, three packed instructions per two samples. `one` is 0x00010001 made opaque to the
// compiler, which would otherwise turn the capped difference back into compares.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
template <int NP>
__device__ __forceinline__ uint32_t count_below_pk(const uint32_t (&vp)[NP], uint32_t t, u16x2 one) {
    const u16x2 tt = {(unsigned short)t, (unsigned short)t};
    u16x2 d[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
        d[i] = __builtin_elementwise_min(__builtin_elementwise_sub_sat(tt, __builtin_bit_cast(u16x2, vp[i])), one);
    // pairwise sums: independent instructions back to back instead of one dependent chain
#pragma unroll
    for (int w = 1; w < NP; w *= 2)
#pragma unroll
        for (int i = 0; i + w < NP; i += 2 * w) d[i] += d[i + w];
    return (uint32_t)d[0].x + (uint32_t)d[0].y;
}
__device__ __forceinline__ u16x2 opaque_ones() {
    uint32_t w = 0x00010001u;
    asm("" : "+v"(w));
    return __builtin_bit_cast(u16x2, w);
}
// samples (32-bit, 0xffffffff where the slot holds none) -> pairs of 16-bit samples
template <int SL>
__device__ __forceinline__ void pack_samples(const uint32_t (&v)[SL], uint32_t (&vp)[(SL + 1) / 2]) {
#pragma unroll
    for (int i = 0; i < (SL + 1) / 2; ++i) {
        const uint32_t hi = 2 * i + 1 < SL ? v[2 * i + 1] : 0xffffu;
        vp[i] = (v[2 * i] & 0xffffu) | (hi << 16);
    }
}

// One level for the pixel of this lane's group (c: its centre; pend: still undecided).
// Returns true when the pixel goes on to the next level; a pixel decided here gets its
// value in `out` (the same in all lanes of the group).
template <typename T, int K, int G>
__device__ __forceinline__ bool group_level(const HD_LDS T *c, const GroupOffsets<K, G> &go, bool last, bool keep,
                                            bool pend, uint32_t &out) {
    using D = DeepGroup<K, G>;
    constexpr int SL = D::SL;
    constexpr uint32_t half = (D::N - 1) / 2;
    const int j = threadIdx.x & (G - 1);
    const uint32_t g = *c;
    // the last slot is a real sample only on the lanes that still have one; elsewhere it
    // holds a value above every sample, so that it never counts as equal to zmin / zmax
    // or below a threshold, and it adds nothing to the packed max
    const bool tail_ok = j + G * (SL - 1) < D::N;
    uint32_t v[SL], key = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const uint32_t x = c[go.off[s]];
        const bool ok = s < SL - 1 || tail_ok;
        v[s] = ok ? x : 0xffffffffu;
        key = pk_max_u16(key, ok ? (((0xffffu - x) << 16) | x) : 0u);
    }
    key = group_max_pk<G>(key);
    const uint32_t mn = 0xffffu - (key >> 16), mx = key & 0xffffu;
    uint32_t cnt = 0;  // (samples equal to zmin) << 16 | samples equal to zmax
#pragma unroll
    for (int s = 0; s < SL; ++s) cnt += ((uint32_t)(v[s] == mn) << 16) | (uint32_t)(v[s] == mx);
    cnt = group_sum<G>(cnt);
    const bool stage_a = (cnt >> 16) <= half && (cnt & 0xffffu) <= half;
    const bool take_g = (stage_a && g != mn && g != mx) || (!stage_a && last && keep);
    const bool go_on = !stage_a && !last;
    const bool need_z = pend && !take_g && !go_on;
    if (pend && take_g) out = g;
    if (__ballot(need_z) != 0) {
        // zmed = the largest p with #(samples < p) <= (k^2 - 1) / 2, built bit by bit from
        // the top. Bits above the highest one where any group's zmin and zmax differ are
        // shared by every sample of that group; starting a group's search at a higher bit
        // than it needs leaves its prefix unchanged, so one bit range serves every group.
        uint32_t d = mn ^ mx;                       // the same in every lane of a group
        if constexpr (G == 4) d |= dpp<DPP_ROW_ROR4>(d);  // the groups of a DPP row
        if constexpr (G <= 8) d |= dpp<DPP_ROW_ROR8>(d);
        const uint32_t dall = (uint32_t)__builtin_amdgcn_readlane((int)d, 0) |
                              (uint32_t)__builtin_amdgcn_readlane((int)d, 16) |
                              (uint32_t)__builtin_amdgcn_readlane((int)d, 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)d, 48);
        const int hb = dall ? 31 - __clz(dall) : -1;
        uint32_t p = hb >= 0 ? (mn & ~((2u << hb) - 1u)) : mn;
        uint32_t vp[(SL + 1) / 2];
        pack_samples<SL>(v, vp);
        const u16x2 one = opaque_ones();
        for (int b = hb; b >= 0; --b) {
            const uint32_t t = p | (1u << b);
            const uint32_t below = group_sum<G>(count_below_pk(vp, t, one));
            p = below <= half ? t : p;
        }
        if (need_z) out = p;
    }
    return pend && go_on;
}

// Level k, step 1 for the pixel of this lane's group: the samples and the stage-A test
// from the counts of zmin and zmax. 0: decided (value in out: the centre kept by stage B,
// or by keep mode at the last level), 1: goes on to the next level, 2: zmed needed.
template <typename T, int K, int G>
__device__ __forceinline__ int group_stage_a(const HD_LDS T *c, const GroupOffsets<K, G> &go, bool last, bool keep,
                                             uint32_t &out) {
    using D = DeepGroup<K, G>;
    constexpr int SL = D::SL;
    constexpr uint32_t half = (D::N - 1) / 2;
    const int j = threadIdx.x & (G - 1);
    const uint32_t g = *c;
    const bool tail_ok = j + G * (SL - 1) < D::N;
    uint32_t v[SL], key = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const uint32_t x = c[go.off[s]];
        const bool ok = s < SL - 1 || tail_ok;
        v[s] = ok ? x : 0xffffffffu;
        key = pk_max_u16(key, ok ? (((0xffffu - x) << 16) | x) : 0u);
    }
    key = group_max_pk<G>(key);
    const uint32_t mn = 0xffffu - (key >> 16), mx = key & 0xffffu;
    uint32_t cnt = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) cnt += ((uint32_t)(v[s] == mn) << 16) | (uint32_t)(v[s] == mx);
    cnt = group_sum<G>(cnt);
    const bool stage_a = (cnt >> 16) <= half && (cnt & 0xffffu) <= half;
    if ((stage_a && g != mn && g != mx) || (!stage_a && last && keep)) {
        out = g;
        return 0;
    }
    return (!stage_a && !last) ? 1 : 2;
}

// Level k, step 2: zmed of the pixel of this lane's group (every group active; spare
// groups repeat a real pixel), by bisection on the bits of the value as in group_level.
template <typename T, int K, int G>
__device__ __forceinline__ uint32_t group_zmed(const HD_LDS T *c, const GroupOffsets<K, G> &go) {
    using D = DeepGroup<K, G>;
    constexpr int SL = D::SL;
    constexpr uint32_t half = (D::N - 1) / 2;
    const int j = threadIdx.x & (G - 1);
    const bool tail_ok = j + G * (SL - 1) < D::N;
    uint32_t v[SL], key = 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        const uint32_t x = c[go.off[s]];
        const bool ok = s < SL - 1 || tail_ok;
        v[s] = ok ? x : 0xffffffffu;
        key = pk_max_u16(key, ok ? (((0xffffu - x) << 16) | x) : 0u);
    }
    key = group_max_pk<G>(key);
    const uint32_t mn = 0xffffu - (key >> 16), mx = key & 0xffffu;
    uint32_t d = mn ^ mx;
    if constexpr (G == 4) d |= dpp<DPP_ROW_ROR4>(d);  // the groups of a DPP row
    if constexpr (G <= 8) d |= dpp<DPP_ROW_ROR8>(d);
    const uint32_t dall = (uint32_t)__builtin_amdgcn_readlane((int)d, 0) |
                          (uint32_t)__builtin_amdgcn_readlane((int)d, 16) |
                          (uint32_t)__builtin_amdgcn_readlane((int)d, 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)d, 48);
    const int hb = dall ? 31 - __clz(dall) : -1;
    uint32_t p = hb >= 0 ? (mn & ~((2u << hb) - 1u)) : mn;
    uint32_t vp[(SL + 1) / 2];
    pack_samples<SL>(v, vp);
    const u16x2 one = opaque_ones();
    for (int b = hb; b >= 0; --b) {
        const uint32_t t = p | (1u << b);
        const uint32_t below = group_sum<G>(count_below_pk(vp, t, one));
        p = below <= half ? t : p;
    }
    return p;
}

// Slot in a list for each group leader with `take`: one atomic add per wave.
__device__ __forceinline__ int group_take(HD_LDS int *counter, bool take) {
    const int lane = threadIdx.x & 63;
    const unsigned long long m = __ballot(take);
    int base = 0;
    if (m != 0) {
        const int first = __ffsll((long long)m) - 1;
        if (lane == first)
            base = __hip_atomic_fetch_add(counter, __popcll(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        base = __builtin_amdgcn_readlane(base, first);
    }
    return base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One level k over a list of pending pixels (LDS indices into the AMF region), several
// pixels per wave, in two steps so that the costly median runs only for the pixels that
// need it, packed densely: (1) stage A for every pixel: decided pixels get their output,
// those that go on are appended to the front of list lb (count *cnt_next), those that need
// zmed to its back (count *cnt_z); then every workgroup thread meets at a barrier; (2) zmed
// of the pixels at the back of lb. All threads of the workgroup call it. A function of its
// own: inlined, every level's pass would add to the kernel's register count.
template <typename T, int K, bool RESIDENT>
__device__ __attribute__((noinline)) void group_pass(const HD_LDS uint16_t *la, int n, HD_LDS uint16_t *lb, int cap,
                                                     HD_LDS int *cnt_next, HD_LDS int *cnt_z, HD_LDS T *s_amf,
                                                     const HD_LDS T *in0, int lp, int mAW, int AW, bool last,
                                                     bool keep) {
    constexpr int G = pass_group<K, RESIDENT>();
    using D = DeepGroup<K, G>;
    const GroupOffsets<K, G> go(lp);
    const int lane = threadIdx.x & 63;
    constexpr int sh = D::LANES == 4 ? 2 : (D::LANES == 8 ? 3 : (D::LANES == 16 ? 4 : 5));  // log2(D::LANES)
    const int nq = (n + D::PER_WAVE - 1) / D::PER_WAVE;
    for (int q = (int)threadIdx.x >> 6; q < nq; q += NT / 64) {
        const int i = D::PER_WAVE * q + (lane >> sh);
        const bool act = i < n;
        const int idx = la[act ? i : D::PER_WAVE * q];  // spare groups repeat the first pixel
        const int r = div_region(idx, mAW), cx = idx - r * AW;
        uint32_t out = 0;
        const int outcome = group_stage_a<T, K, G>(in0 + r * lp + cx, go, last, keep, out);
        const bool leader = act && (lane & (D::LANES - 1)) == 0;
        const int pn = group_take(cnt_next, leader && outcome == 1);
        const int pz = group_take(cnt_z, leader && outcome == 2);
        if (leader) {
            if (outcome == 0) s_amf[idx] = (T)out;
            else if (outcome == 1) lb[pn] = (uint16_t)idx;
            else lb[cap - 1 - pz] = (uint16_t)idx;
        }
    }
    __syncthreads();
    const int nz = *cnt_z;  // uniform: read after the barrier
    const int nzq = (nz + D::PER_WAVE - 1) / D::PER_WAVE;
    for (int q = (int)threadIdx.x >> 6; q < nzq; q += NT / 64) {
        const int i = D::PER_WAVE * q + (lane >> sh);
        const bool act = i < nz;
        const int idx = lb[cap - 1 - (act ? i : D::PER_WAVE * q)];
        const int r = div_region(idx, mAW), cx = idx - r * AW;
        const uint32_t z = group_zmed<T, K, G>(in0 + r * lp + cx, go);
        if (act && (lane & (D::LANES - 1)) == 0) s_amf[idx] = (T)z;
    }
}

template <typename T, bool RESIDENT>
__device__ __forceinline__ void group_pass_k(int k, const uint16_t *la_g, int n, uint16_t *lb_g, int cap, int *cnt_g,
                                             int *cntz_g, T *s_amf_g, const T *in0_g, int lp, int mAW, int AW,
                                             bool last, bool keep) {
    const HD_LDS uint16_t *la = (const HD_LDS uint16_t *)la_g;
    HD_LDS uint16_t *lb = (HD_LDS uint16_t *)lb_g;
    HD_LDS int *cnt_next = (HD_LDS int *)cnt_g;
    HD_LDS int *cnt_z = (HD_LDS int *)cntz_g;
    HD_LDS T *s_amf = (HD_LDS T *)s_amf_g;
    const HD_LDS T *in0 = (const HD_LDS T *)in0_g;
    switch (k) {
        case 5: group_pass<T, 5, RESIDENT>(la, n, lb, cap, cnt_next, cnt_z, s_amf, in0, lp, mAW, AW, last, keep); break;
        case 7: group_pass<T, 7, RESIDENT>(la, n, lb, cap, cnt_next, cnt_z, s_amf, in0, lp, mAW, AW, last, keep); break;
        case 9: group_pass<T, 9, RESIDENT>(la, n, lb, cap, cnt_next, cnt_z, s_amf, in0, lp, mAW, AW, last, keep); break;
        case 11: group_pass<T, 11, RESIDENT>(la, n, lb, cap, cnt_next, cnt_z, s_amf, in0, lp, mAW, AW, last, keep); break;
        case 13: group_pass<T, 13, RESIDENT>(la, n, lb, cap, cnt_next, cnt_z, s_amf, in0, lp, mAW, AW, last, keep); break;
        default: group_pass<T, 15, RESIDENT>(la, n, lb, cap, cnt_next, cnt_z, s_amf, in0, lp, mAW, AW, last, keep); break;
    }
}

// group_level for a runtime level k of 9 or 11 (offsets computed per call). A function of
// its own, for the same reason as group_pass.
// (The result comes back by value, (still pending) << 32 | output: a reference argument
// would put the output in scratch memory.)
template <typename T>
__device__ __attribute__((noinline)) unsigned long long row_level_lds(int k, const HD_LDS T *c, int lp, bool last,
                                                                      bool keep, bool pend, uint32_t out) {
    const bool p = k == 9 ? group_level<T, 9, 16>(c, GroupOffsets<9, 16>(lp), last, keep, pend, out)
                          : group_level<T, 11, 16>(c, GroupOffsets<11, 16>(lp), last, keep, pend, out);
    return ((unsigned long long)p << 32) | out;
}
template <typename T>
__device__ __forceinline__ bool row_level_k(int k, const T *c, int lp, bool last, bool keep, bool pend,
                                            uint32_t &out) {
    const unsigned long long r = row_level_lds<T>(k, (const HD_LDS T *)c, lp, last, keep, pend, out);
    out = (uint32_t)r;
    return (r >> 32) != 0;
}

// Wave mode covers windows up to 15 x 15 (at most 4 samples per lane); larger windows
// always take the per-lane path.
template <typename T>
__device__ __forceinline__ int wave_level_k(int k, const T *c, int lp, bool last, bool keep, uint32_t &out) {
    switch (k) {
        case 5: return wave_level<T, 5>(c, lp, last, keep, out);
        case 7: return wave_level<T, 7>(c, lp, last, keep, out);
        case 9: return wave_level<T, 9>(c, lp, last, keep, out);
        case 11: return wave_level<T, 11>(c, lp, last, keep, out);
        case 13: return wave_level<T, 13>(c, lp, last, keep, out);
        default: return wave_level<T, 15>(c, lp, last, keep, out);
    }
}
// wave_level_k as a function of its own, for the rarely taken one-wave-per-pixel paths of
// the staged kernel: inlined, its window registers were reserved for the whole kernel,
// which then spilled live values at every tile; as a call, the caller saves what it needs
// only around the call. Returns (outcome << 32) | out.
template <typename T>
__device__ __attribute__((noinline)) unsigned long long wave_level_call(int k, const HD_LDS T *c, int lp, bool last,
                                                                        bool keep) {
    uint32_t out = 0;
    const int outcome = wave_level_k<T>(k, (const T *)c, lp, last, keep, out);
    return ((unsigned long long)(uint32_t)outcome << 32) | out;
}

template <typename T>
__device__ __forceinline__ int level_test_k(int k, const T *c, int lp, bool last, bool keep, uint32_t &out) {
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
__device__ __forceinline__ uint32_t level_median_k(int k, const T *c, int lp, uint32_t bracket) {
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

// Exact Wiener window sums of the tile's pixels from the AMF region in LDS (region element
// (r, c) is image pixel (ry0 + r, rx0 + c); window positions outside the image are mirrored
// back inside, where the ring at least as wide as the window radius holds them). Thread
// (wave wv, lane) owns tile column lane and tile rows wv * RPT + j: s1[j] = S1 and
// num[j] = N * S2 - S1^2 (unspecified for pixels outside the image). `work` holds the row
// sums. WH, WW > 0 fix the window size at compile time (unrolled, loads issued together);
// 0 takes the runtime size.
template <typename T, int WH, int WW>
__device__ __forceinline__ void tile_moments(const T *s_amf, int AW, int AH, unsigned char *work,
                                             int wh_rt, int ww_rt, int H, int W, int x0, int y0,
                                             int rx0, int ry0, uint32_t (&s1o)[RPT],
                                             typename SqT<T>::type (&numo)[RPT]) {
    using S2T = typename SqT<T>::type;
    const int wh = WH > 0 ? WH : wh_rt, ww = WW > 0 ? WW : ww_rt;
    const int rh = wh / 2, rw = ww / 2;
    uint32_t *h1 = (uint32_t *)work;
    S2T *h2 = (S2T *)(work + AH * TILE_X * 4);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int gxc = x0 + lane;
    bool in_x = rx0 >= 0 && x0 + TILE_X + rw <= W;
    bool in_y = ry0 >= 0 && y0 + TILE_Y + rh <= H;
    if ((!in_x || !in_y) && W >= rw && H >= rh) {
        // Window positions outside the image take the value at their mirror position, which
        // one reflection puts inside both the image and the region: copy it there in LDS
        // (columns, then whole rows), so that the sums below need no index mirroring.
        T *a = (T *)s_amf;
        const int lo_c = max(0, -rx0), hi_c = max(0, min(W + rw, rx0 + AW) - W);
        const int nc = lo_c + hi_c;
        for (int i = tid; i < AH * nc; i += NT) {
            const int r = i / nc, k = i - r * nc;
            const int gx = k < lo_c ? rx0 + k : W + (k - lo_c);
            const int sx = gx < 0 ? -1 - gx : 2 * W - 1 - gx;
            a[r * AW + (gx - rx0)] = a[r * AW + (sx - rx0)];
        }
        __syncthreads();
        const int lo_r = max(0, -ry0), hi_r = max(0, min(H + rh, ry0 + AH) - H);
        const int nr = lo_r + hi_r;
        for (int i = tid; i < nr * AW; i += NT) {
            const int k = i / AW, c = i - k * AW;
            const int gy = k < lo_r ? ry0 + k : H + (k - lo_r);
            const int sy = gy < 0 ? -1 - gy : 2 * H - 1 - gy;
            a[(gy - ry0) * AW + c] = a[(sy - ry0) * AW + c];
        }
        __syncthreads();
        in_x = in_y = true;
    }

    // 1. sums over the window width of every region row inside the image
    auto hrow = [&](int r) {
        const int gy = ry0 + r;
        // outside the image: rows are read through mirror() unless the ring was filled;
        // columns past the image edge give no output
        if ((!in_y && (gy < 0 || gy >= H)) || (!in_x && gxc >= W)) return;
        const T *row = s_amf + r * AW;
        uint32_t t1 = 0;
        S2T t2 = 0;
        if constexpr (sizeof(T) == 1 && (WW == 3 || WW == 5 || WW == 7)) {
            if (in_x) {
                byte_window_sums<WW>((const unsigned char *)s_amf, r * AW + lane, t1, t2);
                h1[r * TILE_X + lane] = t1;
                h2[r * TILE_X + lane] = t2;
                return;
            }
        }
        if (in_x) {
#pragma unroll
            for (int dx = 0; dx < ww; ++dx) {
                const uint32_t v = row[lane + dx];
                t1 += v;
                t2 += square_u16<S2T>(v);
            }
        } else {
            for (int dx = -rw; dx <= rw; ++dx) {
                const uint32_t v = row[mirror(gxc + dx, W) - rx0];
                t1 += v;
                t2 += square_u16<S2T>(v);
            }
        }
        h1[r * TILE_X + lane] = t1;
        h2[r * TILE_X + lane] = t2;
    };
    if constexpr (WH > 0) {
        constexpr int RPW = (TILE_Y + 2 * (WH / 2) + NT / 64 - 1) / (NT / 64);
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + (NT / 64) * i;
            if (r < AH) hrow(r);
        }
    } else {
        for (int r = wv; r < AH; r += NT / 64) hrow(r);
    }
    __syncthreads();

    // 2. sums over the window height, sliding down the thread's rows
    const S2T nwin = (S2T)(wh * ww);
    const int j0 = wv * RPT;
    if (in_y) {
        if constexpr (WH > 0) {
            constexpr int NR = RPT + WH - 1;
            uint32_t c1[NR];
            S2T c2[NR];
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                c1[i] = h1[(j0 + i) * TILE_X + lane];
                c2[i] = h2[(j0 + i) * TILE_X + lane];
            }
            uint32_t s1 = 0;
            S2T s2 = 0;
#pragma unroll
            for (int i = 0; i < WH; ++i) {
                s1 += c1[i];
                s2 += c2[i];
            }
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (j > 0) {
                    s1 += c1[j + WH - 1] - c1[j - 1];
                    s2 += c2[j + WH - 1] - c2[j - 1];
                }
                s1o[j] = s1;
                numo[j] = window_num<S2T>(nwin, s1, s2);
            }
        } else {
            uint32_t s1 = 0;
            S2T s2 = 0;
            for (int dy = 0; dy < wh; ++dy) {
                s1 += h1[(j0 + dy) * TILE_X + lane];
                s2 += h2[(j0 + dy) * TILE_X + lane];
            }
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (j > 0) {
                    s1 += h1[(j0 + j + wh - 1) * TILE_X + lane] - h1[(j0 + j - 1) * TILE_X + lane];
                    s2 += h2[(j0 + j + wh - 1) * TILE_X + lane] - h2[(j0 + j - 1) * TILE_X + lane];
                }
                s1o[j] = s1;
                numo[j] = window_num<S2T>(nwin, s1, s2);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int gy = y0 + j0 + j;
            uint32_t s1 = 0;
            S2T s2 = 0;
            if (gy < H) {
                for (int dy = -rh; dy <= rh; ++dy) {
                    const int ri = mirror(gy + dy, H) - ry0;
                    s1 += h1[ri * TILE_X + lane];
                    s2 += h2[ri * TILE_X + lane];
                }
            }
            s1o[j] = s1;
            numo[j] = window_num<S2T>(nwin, s1, s2);
        }
    }
}

template <typename T>
__device__ __forceinline__ void tile_moments_any(const T *s_amf, int AW, int AH, unsigned char *work,
                                                 int wh, int ww, int H, int W, int x0, int y0, int rx0,
                                                 int ry0, uint32_t (&s1o)[RPT],
                                                 typename SqT<T>::type (&numo)[RPT]) {
    if (wh == 3 && ww == 3)
        tile_moments<T, 3, 3>(s_amf, AW, AH, work, wh, ww, H, W, x0, y0, rx0, ry0, s1o, numo);
    else if (wh == 5 && ww == 5)
        tile_moments<T, 5, 5>(s_amf, AW, AH, work, wh, ww, H, W, x0, y0, rx0, ry0, s1o, numo);
    else if (wh == 7 && ww == 7)
        tile_moments<T, 7, 7>(s_amf, AW, AH, work, wh, ww, H, W, x0, y0, rx0, ry0, s1o, numo);
    else
        tile_moments<T, 0, 0>(s_amf, AW, AH, work, wh, ww, H, W, x0, y0, rx0, ry0, s1o, numo);
}

// Barrier words of the resident kernel are only ever touched by atomic read-modify-write
// operations at device scope: those resolve at the coherence point shared by all XCDs, so
// a poll never reads a stale copy from its own L2 and a release is seen at once.
// (A read is a compare-and-swap that stores back what it finds: an add of zero would be
// turned into a plain load by the compiler.)
__device__ __forceinline__ unsigned int sync_read(unsigned int *p) {
    unsigned int v = 0xffffffffu;
    __hip_atomic_compare_exchange_strong(p, &v, 0xffffffffu, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return v;
}
__device__ __forceinline__ void sync_write(unsigned int *p, unsigned int v) {
    (void)__hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long sync_read64(unsigned long long *p) {
    unsigned long long v = ~0ull;
    __hip_atomic_compare_exchange_strong(p, &v, ~0ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return v;
}
__device__ __forceinline__ unsigned long long sync_xchg64(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait for *flag != v: at most `limit` ticks of the 100 MHz real-time counter
// (the library default is 1 s; limit 0 does not wait at all), polling with a growing
// pause (about 0.1 to 0.45 us) so that a thousand waiting workgroups do not saturate the
// atomic units. False on timeout.
__device__ __forceinline__ int resident_wait(unsigned int *flag, unsigned int v, unsigned long long limit) {
    if (limit == 0) return 0;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int pause = 0;
    while (sync_read(flag) == v) {
        if (pause < 2) __builtin_amdgcn_s_sleep(4);
        else if (pause < 6) __builtin_amdgcn_s_sleep(8);
        else __builtin_amdgcn_s_sleep(16);
        ++pause;
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return 0;
    }
    return 1;
}

// resident_wait for a 64-bit word: waits for *p != v and returns the value seen in `seen`.
__device__ __forceinline__ int resident_wait64(unsigned long long *p, unsigned long long v,
                                               unsigned long long &seen, unsigned long long limit) {
    if (limit == 0) return 0;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int pause = 0;
    while ((seen = sync_read64(p)) == v) {
        // every waiter polls its own word: short pauses
        if (pause < 4) __builtin_amdgcn_s_sleep(2);
        else __builtin_amdgcn_s_sleep(8);
        ++pause;
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return 0;
    }
    return 1;
}

// The library's error word on each device: bit 0 is set when a wait of the resident
// kernel's exchange gave up (that workgroup wrote NaN). The host reads and clears it
// (hd_check_errors); kernels only ever set bits.
static __device__ unsigned int g_error_word;

// Packed arrival: a 64-bit word holds an arrival count in its top byte and a sum below it.
// (Arrival stays two-level: a single word taking every workgroup's add queues them at the
// memory-side atomic unit, and the last arrival waits several microseconds.)
constexpr int PACK_SHIFT = 56;
constexpr unsigned long long PACK_ONE = 1ull << PACK_SHIFT;
constexpr unsigned long long PACK_MASK = PACK_ONE - 1;

// The resident kernel's grid-wide barrier: arrival in two levels, release by the last
// arrival through every group's slot (results, then the group's flag). Layout of the words
// and the protocol: see step 6 of the kernel.
struct ResidentGrid {
    unsigned int *w;
    int nb, grp, g, ng;
    unsigned int *slot;
    unsigned int *err;         // the device's error word
    unsigned long long limit;  // wait bound in real-time counter ticks
    __device__ __forceinline__ ResidentGrid(unsigned int *words, unsigned int *err_word, unsigned long long wait_limit)
        : w(words), err(err_word), limit(wait_limit) {
        nb = (int)gridDim.x;
        grp = resident_group_size(nb);
        const int sh = 31 - __clz(grp);  // grp is a power of two
        g = (int)blockIdx.x >> sh;
        ng = (nb + grp - 1) >> sh;
        slot = w + RESIDENT_SLOT_WORDS * (g + 1);
    }
    // the group's release flag (read before arriving)
    __device__ __forceinline__ unsigned int read_flag() const { return sync_read(slot + 32); }
    // workgroups of this group and the first of them
    __device__ __forceinline__ int group_first() const { return g * grp; }
    __device__ __forceinline__ int group_size() const { return min(grp, nb - g * grp); }
    // store this workgroup's partial, then arrive in the group: true for the group's last
    // arrival (one thread per workgroup)
    __device__ __forceinline__ bool arrive_group(unsigned long long *partial, unsigned long long v) const {
        (void)sync_xchg64(partial, v);
        // release at device scope: the partial is performed before the arrival is
        const unsigned int a = __hip_atomic_fetch_add(slot, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (a != (unsigned int)group_size() - 1u) return false;
        sync_write(slot, 0u);
        return true;
    }
    // (the group's last arrival) arrive at the top level: true for the last overall
    __device__ __forceinline__ bool arrive_top() const {
        // release: the group's summary and the reset of its counter are performed first
        const unsigned int t = __hip_atomic_fetch_add(w + 32, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (t != (unsigned int)ng - 1u) return false;
        sync_write(w + 32, 0u);
        return true;
    }
    __device__ __forceinline__ unsigned long long *summary(int gg) const {
        return (unsigned long long *)(w + RESIDENT_SLOT_WORDS * (gg + 1) + 112);
    }
    // (every thread of the last workgroup) n results into every group's slot at word
    // offset `off`, then that group's flag
    __device__ __forceinline__ void release(const unsigned long long *res, int n, int off) const {
        for (int gg = (int)threadIdx.x; gg < ng; gg += NT) {
            unsigned int *sl = w + RESIDENT_SLOT_WORDS * (gg + 1);
            for (int i = 0; i < n; ++i) (void)sync_xchg64((unsigned long long *)(sl + off) + i, res[i]);
            // release: the results are performed before the flag moves
            (void)__hip_atomic_fetch_add(sl + 32, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // Packed round for one additive value per workgroup (every partial sum < 2^56): one
    // atomic add of (1, v) per workgroup on its group's word; the group's last arrival adds
    // (1, group sum) to the top word; the last overall gets the exact total from the value
    // that add returns. 0: a member, 1: a group's last, 2: the last overall (total set).
    __device__ __forceinline__ unsigned long long *pack_group() const {
        return (unsigned long long *)(slot + 128);
    }
    __device__ __forceinline__ unsigned long long *pack_flag(int b) const {
        return (unsigned long long *)(w + RESIDENT_GROUP_WORDS + RESIDENT_BLOCK_WORDS * b);
    }
    __device__ __forceinline__ int arrive_packed(unsigned long long v, unsigned long long &total) const {
        unsigned long long *top = (unsigned long long *)(w + 128);
        const unsigned long long old =
            __hip_atomic_fetch_add(pack_group(), PACK_ONE + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((old >> PACK_SHIFT) != (unsigned long long)(group_size() - 1)) return 0;
        (void)sync_xchg64(pack_group(), 0ull);  // every member has added: zero for the next launch
        const unsigned long long gsum = (old & PACK_MASK) + v;
        const unsigned long long old2 =
            __hip_atomic_fetch_add(top, PACK_ONE + gsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((old2 >> PACK_SHIFT) != (unsigned long long)(ng - 1)) return 1;
        (void)sync_xchg64(top, 0ull);
        total = (old2 & PACK_MASK) + gsum;
        return 2;
    }
    // (every thread of the last overall) the total into every workgroup's release word: an
    // exclusive or with a value whose top bit is set, so every word changes and a waiter
    // that knows its word's value before the round recovers the total
    __device__ __forceinline__ void release_packed(unsigned long long total) const {
        for (int b = (int)threadIdx.x; b < nb; b += NT)
            (void)__hip_atomic_fetch_xor(pack_flag(b), (1ull << 63) | total, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    }
    // wait for this workgroup's release word to leave `base`; the total in `total`; false on
    // timeout
    __device__ __forceinline__ int wait_packed(unsigned long long base, unsigned long long &total) const {
        unsigned long long seen = base;
        const int ok = resident_wait64(pack_flag((int)blockIdx.x), base, seen, limit);
        if (!ok) __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        total = (seen ^ base) & PACK_MASK;
        return ok;
    }
    // wait for the group's flag to leave `base` (one thread); false on timeout
    __device__ __forceinline__ int wait(unsigned int base) const {
        const int ok = resident_wait(slot + 32, base, limit);
        if (!ok) __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return ok;
    }
    __device__ __forceinline__ unsigned long long result(int off, int i) const {
        return sync_read64((unsigned long long *)(slot + off) + i);
    }
};

// The staged kernel is held to 64 registers (eight waves per SIMD, a few values spilled
// around the level passes): its level loop leaves waves idle at barriers while lists are
// short, and more resident workgroups fill those gaps (measured faster than 80 registers
// with six waves or 86 with five). The single-launch variant keeps what it needs.
template <typename T, bool DENSE, bool RESIDENT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(RESIDENT ? 1 : 8))) void amf_stage_kernel(SliceSet set, int total_tiles, int smax,
                                                       int keep, int wh, int ww,
                                                       unsigned long long *__restrict__ partials,
                                                       int select_mode, int aligned, float mf,
                                                       unsigned int *sync_words, double *nu2,
                                                       int store_amf, int stretch, int packed,
                                                       WienerConst wcb, int maw, unsigned int *err_word,
                                                       unsigned long long wait_limit, int tile_rows) {
    using S2T = typename SqT<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_cnt[3];
    __shared__ unsigned long long s_wsum[NT / 64];

    // The AMF tile: TR rows of 64 columns (TR = TILE_Y except in the staged stage without
    // the Wiener ring and without a tile list, where the host may pick 16 or 64). TR = 16:
    // two workgroups per 64 x 32 tile (the upper and lower half); TR = 64: the workgroup of
    // an even tile row covers it and the next, and odd rows' workgroups exit.
    const int TR = RESIDENT ? TILE_Y : tile_rows;
    int tile, half = 0;
    if (set.list) {  // listed tiles only (uniform early exit for the spare blocks)
        if ((int)blockIdx.x >= *set.list_count) return;
        tile = set.list[blockIdx.x];
    } else if (TR < TILE_Y) {
        const int u = xcd_remap(blockIdx.x, 2 * total_tiles);
        tile = u >> 1;
        half = u & 1;
    } else {
        tile = xcd_remap(blockIdx.x, total_tiles);
    }
    const int si = slice_index(set, tile);
    const SliceDesc sd = slice_desc(set, si);
    const int H = sd.h, W = sd.w;
    const int lt = tile - sd.tile_begin;
    const int ty = div_tiles(lt, sd.tiles_x);
    const int x0 = (lt - ty * sd.tiles_x) * TILE_X;
    const int y0 = ty * TILE_Y + half * TR;
    if ((TR > TILE_Y && (ty & 1)) || y0 >= H) return;  // uniform: covered elsewhere / below the image
    const bool moments = RESIDENT || wh > 0;
    constexpr int K3R = RESIDENT ? RESIDENT_STRIP : STAGED_STRIP;  // rows per level-3 strip
    const AmfSmem L = amf_smem_layout((int)sizeof(T), smax, moments ? wh : 0, moments ? ww : 0, K3R, TR);
    const int R = L.R, rh = L.rh, rw = L.rw, AH = L.AH, AW = L.AW;
    const int ry0 = y0 - rh, rx0 = x0 - rw;  // image position of AMF-region element (0, 0)

    T *s_amf = (T *)smem;
    unsigned char *u = smem + L.amf_bytes;
    T *s_in = (T *)u;
    uint16_t *s_list = (uint16_t *)(u + L.in_bytes);  // two lists of AH * AW entries
    const int cap = AH * AW;

    const int tid = threadIdx.x, lane = tid & 63;

    // The barrier words' values before this launch's rounds, read first so that the reads'
    // latency hides behind the staging (no round of this launch starts before every
    // workgroup has arrived, which is after these reads).
    __shared__ unsigned int s_flag0;
    __shared__ unsigned long long s_pack0;
    unsigned int flag_base = 0;
    unsigned long long pack_base = 0;
    if (RESIDENT && tid == 0) {
        const ResidentGrid rg0(sync_words, err_word, wait_limit);
        if (packed) pack_base = sync_read64(rg0.pack_flag((int)blockIdx.x));
        if (!packed || stretch) flag_base = rg0.read_flag();
    }

    // 1. input region -> LDS
    const Staged st = stage_region<T, true>(s_in, (const T *)sd.in, H, W, sd.in_pitch, ry0 - R, rx0 - R,
                                      L.IH, AW + 2 * R, aligned != 0);
    const int lp = st.lpt;
    const T *in0 = s_in + R * lp + st.off + R;  // centre of AMF-region element (0, 0)
    if (tid < 3) s_cnt[tid] = 0;
    if (RESIDENT && tid == 0) {
        s_flag0 = flag_base;
        s_pack0 = pack_base;
    }
    __syncthreads();

    // 2. level 3 for every pixel of the AMF region: strips of K3R rows, one column each
    const bool last3 = (smax == 3);
    const uint32_t keep1 = keep != 0 ? 1u : 0u;
    const int nstrip = (AH + K3R - 1) / K3R;
    const int nitems = nstrip * AW;
    const int mAW = maw;  // div_region_magic(AW), from the host
    // (whole waves run every iteration, so that the list append is one atomic per wave)
    for (int item0 = 0; item0 < nitems; item0 += NT) {
        const int item = item0 + tid;
        uint32_t defer = 0;
        int cx = 0, rb = 0;
        if (item < nitems) {
        const int s = div_region(item, mAW);
        cx = item - s * AW;
        rb = s * K3R;
        uint32_t lo[K3R + 2], md[K3R + 2], hi[K3R + 2], ctr[K3R + 2];
        // left neighbour of the strip's top row: the three reads of a row then take the LDS
        // offsets 0, 1, 2 (an offset cannot be negative)
        const T *p0 = in0 + (rb - 1) * lp + cx - 1;
#pragma unroll
        for (int j = 0; j < K3R + 2; ++j) {
            // every row of the strip (and one above / below) lies in the staged region
            const T *p = p0 + j * lp;
            const uint32_t a = p[0], b = p[1], c = p[2];
            lo[j] = min3_vop(a, b, c);
            md[j] = med3_vop(a, b, c);
            hi[j] = max3_vop(a, b, c);
            ctr[j] = b;
        }
        const int gx = rx0 + cx;
        // rows of this strip that are real image pixels inside the AMF region
        const int gy0 = ry0 + rb;
        const int rlo = max(0, -gy0), rhi = min(min(K3R, AH - rb), H - gy0);
        const bool col_ok = gx >= 0 && gx < W && !last3;
        T *dst = s_amf + rb * AW + cx;
#pragma unroll
        for (int j = 0; j < K3R; ++j) {
            const uint32_t zmin = min3_vop(lo[j], lo[j + 1], lo[j + 2]);
            const uint32_t zmax = max3_vop(hi[j], hi[j + 1], hi[j + 2]);
            const uint32_t zmed = med3_vop(max3_vop(lo[j], lo[j + 1], lo[j + 2]),
                                           med3_vop(md[j], md[j + 1], md[j + 2]),
                                           min3_vop(hi[j], hi[j + 1], hi[j + 2]));
            const uint32_t g = ctr[j + 1];
            // 0 / 1 flags combined with bitwise operators: no branches per pixel
            const uint32_t stage_a = (uint32_t)(zmin < zmed) & (uint32_t)(zmed < zmax);
            const uint32_t centre_ok = (uint32_t)(zmin < g) & (uint32_t)(g < zmax);
            // stage A: g when stage B passes, else zmed; no stage A: final only when
            // Smax == 3 (zmed, or g in keep mode)
            const uint32_t use_g = (stage_a & centre_ok) | ((stage_a ^ 1u) & keep1);
            dst[j * AW] = (T)(use_g ? g : zmed);
            defer |= (stage_a ^ 1u) << j;
        }
        // keep rows [rlo, rhi) only (0 <= rlo < K3R, rhi <= K3R; empty when rhi <= rlo)
        defer = (col_ok && rhi > rlo) ? (defer & ((1u << rhi) - 1u) & ~((1u << rlo) - 1u)) : 0u;
        }
        if (__ballot(defer != 0) != 0) {  // uniform; rare outside dense impulse noise
            int pos = wave_reserve(&s_cnt[0], (uint32_t)__popc(defer));
            while (defer) {
                const int j = __ffs(defer) - 1;
                defer &= defer - 1;
                s_list[pos++] = (uint16_t)((rb + j) * AW + cx);
            }
        }
    }
    __syncthreads();

    // one level of one pixel over the whole wave (rare paths; a call in the staged kernel)
    auto wave_step = [&](int k, const T *cc, bool lastk, uint32_t &v) -> int {
        if constexpr (RESIDENT) {
            return wave_level_k<T>(k, cc, lp, lastk, keep != 0, v);
        } else {
            const unsigned long long res = wave_level_call<T>(k, (const HD_LDS T *)cc, lp, lastk, keep != 0);
            v = (uint32_t)res;
            return (int)(res >> 32);
        }
    };

    // 3. deeper levels. A short pending list (a few pixels, typical of moderate impulse
    //    densities) is run four pixels per wave through all their levels up to 11, with no
    //    barrier between levels. Otherwise level by level over compacted lists: list A =
    //    s_list[cur*cap ...]; list B holds the next level's pixels from the front and the
    //    zmed pixels from the back (one lane per pixel), or only the next level's pixels
    //    (four pixels per wave).
    int cur = 0;
    const int n0 = s_cnt[0];
    const bool sparse = smax <= 15 && n0 <= SPARSE_DEEP &&
                        (select_mode == SELECT_AUTO || select_mode == SELECT_DENSE);
    if (n0 > 0 && sparse) {
        // four pixels per wave (one per 16-lane DPP row) through levels 5 to 11, then the
        // few left (Smax >= 13 only) one wave per pixel
        const int nq = (n0 + 3) >> 2;
        for (int q = tid >> 6; q < nq; q += NT / 64) {
            const int i = 4 * q + (lane >> 4);
            const bool act = i < n0;
            const int idx = s_list[act ? i : 4 * q];  // spare rows repeat the first pixel
            const int r = div_region(idx, mAW), cx = idx - r * AW;
            const T *c = in0 + r * lp + cx;
            uint32_t out = 0;
            // levels 5 and 7 inline (the common case), 9 and 11 through a call
            const HD_LDS T *cl = (const HD_LDS T *)c;
            bool pend = group_level<T, 5, 16>(cl, GroupOffsets<5, 16>(lp), smax == 5, keep != 0, act, out);
            if (smax >= 7 && __ballot(pend) != 0)
                pend = group_level<T, 7, 16>(cl, GroupOffsets<7, 16>(lp), smax == 7, keep != 0, pend, out);
            for (int k = 9; k <= smax && k <= 11 && __ballot(pend) != 0; k += 2)
                pend = row_level_k<T>(k, c, lp, k == smax, keep != 0, pend, out);
            if (act && !pend && (lane & 15) == 0) s_amf[idx] = (T)out;
            unsigned long long rest = __ballot(pend && (lane & 15) == 0);
            while (rest) {
                const int l = __ffsll((long long)rest) - 1;
                rest &= rest - 1;
                const int idp = __builtin_amdgcn_readlane(idx, l);
                const int rp = div_region(idp, mAW), cp = idp - rp * AW;
                const T *cc = in0 + rp * lp + cp;
                uint32_t v = 0;
                for (int k = 13; k <= smax; k += 2)
                    if (wave_step(k, cc, k == smax, v) == 0) break;
                if (lane == 0) s_amf[idp] = (T)v;
            }
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
        // per-lane when the list fills the lanes (or bisection is forced), else several
        // pixels per wave (one wave per pixel in the SELECT_WAVE strategy); the choice is
        // uniform across the workgroup
        const bool quad_mode = k <= 15 && (select_mode == SELECT_AUTO || select_mode == SELECT_DENSE) &&
                               n < (DENSE && k <= 5 ? 64 : NT);
        if (quad_mode) {
            group_pass_k<T, RESIDENT>(k, la, n, lb, cap, &s_cnt[nxt], &s_cnt[2], s_amf, in0, lp, mAW, AW, last,
                                      keep != 0);
            __syncthreads();
            if (tid == 0) {
                s_cnt[cur] = 0;
                s_cnt[2] = 0;
            }
            __syncthreads();
            cur = nxt;
            continue;
        }
        const bool wave_mode = k <= 15 && select_mode == SELECT_WAVE;
        if (wave_mode) {
            for (int i = tid >> 6; i < n; i += NT / 64) {
                const int idx = la[i];
                const int r = div_region(idx, mAW), cx = idx - r * AW;
                uint32_t v = 0;
                const int outcome = wave_step(k, in0 + r * lp + cx, last, v);
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
            if (outcome == 0) s_amf[idx] = (T)v;
            // the next level's pixels from the front of list B, the zmed pixels from its back
            // (the bisection bracket is recomputed from the window in step 2)
            const int pn = wave_take(&s_cnt[nxt], outcome == 1);
            const int pz = wave_take(&s_cnt[2], outcome == 2);
            if (outcome == 1) lb[pn] = (uint16_t)idx;
            if (outcome == 2) lb[cap - 1 - pz] = (uint16_t)idx;
        }
        __syncthreads();
        const int m = s_cnt[2];
        for (int i = tid; i < m; i += NT) {
            const int idx = lb[cap - 1 - i];
            const int r = div_region(idx, mAW), cx = idx - r * AW;
            const T *c = in0 + r * lp + cx;
            uint32_t bracket = 0;
            if (!DENSE || k > 5) {  // the dense variant has a network (no bracket) for 5 x 5 only
                uint32_t mn, mx, cmin, cmax;
                (void)cmin; (void)cmax;
                // bracket [mn, mx]: always contains the median
                mn = 0xffffffffu; mx = 0u;
                const int rk = k / 2;
                for (int dy = -rk; dy <= rk; ++dy)
                    for (int dx = 0; dx < k; ++dx) {
                        const uint32_t e = (c + dy * lp - rk)[dx];
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
    } else if (!RESIDENT || store_amf) {
        store_region<T>((T *)sd.amf, H, W, sd.amf_pitch, y0, x0, s_amf + rh * AW + rw, AW,
                        TR, min(TILE_X, W - x0), aligned != 0);
    }
    if (!moments) return;

    // 5. exact Wiener window sums of the tile's pixels and the tile's sum of N * S2 - S1^2
    __syncthreads();  // lists / input region are dead: reuse them for the row sums
    uint32_t s1v[RPT];
    S2T numv[RPT];
    tile_moments_any<T>(s_amf, AW, AH, u, wh, ww, H, W, x0, y0, rx0, ry0, s1v, numv);
    const int wv = tid >> 6, j0 = wv * RPT;
    const bool col_ok = x0 + lane < W;
    const int rows_ok = min(RPT, H - (y0 + j0));
    unsigned long long tsum = 0;
#pragma unroll
    for (int j = 0; j < RPT; ++j)
        if (col_ok && j < rows_ok) tsum += (unsigned long long)numv[j];
    tsum = wave_sum_u64(tsum);
    if (lane == 0) s_wsum[wv] = tsum;
    // the resident kernel prepares every output term that does not need the noise power
    // before the exchange, so that little is left to do after it
    WienerPrep wp[RESIDENT ? RPT : 1];
    if constexpr (RESIDENT) {
        const T *arow = s_amf + (j0 + rh) * AW + lane + rw;
#pragma unroll
        for (int j = 0; j < RPT; ++j) wp[j] = wiener_prep<S2T>(s1v[j], numv[j], (float)arow[j * AW], wcb);
    }
    __syncthreads();
    if constexpr (!RESIDENT) {
        if (tid == 0) {
            unsigned long long b = 0;
            for (int i = 0; i < NT / 64; ++i) b += s_wsum[i];
            partials[tile] = b;
        }
    } else {
        // 6. grid-wide exchange of the slice noise powers (first exchange), and with the contrast
        //    stretch a second exchange for the slices' output range. Everything that crosses
        //    workgroups (sums, counters, flags, results) moves by device-scope atomic
        //    read-modify-write operations, which resolve at the coherence point all XCDs
        //    share, so a read never returns a stale cached copy. Two such operations of one
        //    thread on different words may still complete out of order: every arrival and
        //    every flag raise that publishes earlier stores (partials, summaries, results,
        //    a counter's reset) is a release at device scope, which waits for those stores
        //    to complete before it is issued. A reader issues its reads only after the
        //    arrival or flag value it depends on has come back. Arrival is two-level (groups of consecutive workgroups, each
        //    counter on its own line, so no address sees more than a few dozen operations).
        //    Round 1 is packed for one slice whose sum fits 56 bits (the launcher decides):
        //    count and sum in one 64-bit add per workgroup and per group, the total released
        //    by exclusive-or into one word per workgroup (ResidentGrid::arrive_packed).
        //    Otherwise partials are stored and read back: the last workgroup to arrive
        //    combines the partials of every slice, copies the results into every group's
        //    slot and raises the group flags.
        //    Every wait is bounded: a workgroup that gives up sets bit 0 of the device's
        //    error word and writes NaN, and still arrives in a later round.
        //    Words (u32): [32] top-level arrivals, [128..129] packed top sum. Group g's
        //    slot starts at word RESIDENT_SLOT_WORDS * (g + 1) (4 KB apart, so the groups'
        //    traffic spreads over memory channels): [0] arrivals, [32] release flag,
        //    [64..79] the slices' noise powers (8 doubles), [96..111] the slices' output
        //    ranges (8 x (min, max)), [112..115] the group summary, [128..129] packed group
        //    sum. After the slots, one 64-bit release word per workgroup, 128 bytes apart.
        //    Counters and packed sums return to zero in every round; flags only advance and
        //    release words only change, and a workgroup waits for its flag or word to move
        //    from the value it read at the start of the launch.
        __shared__ int s_ok, s_role;
        __shared__ unsigned long long s_res[RESIDENT_MAX_SLICES];
        __shared__ unsigned long long s_lo[NT / 64], s_hi[NT / 64];
        ResidentGrid rg(sync_words, err_word, wait_limit);
        // A single slice's partials are indexed by workgroup, so that each group's last
        // arrival can sum its group's partials (one parallel round of reads) into the
        // group's summary, and the last overall reads only the group summaries; several
        // slices index them by tile and the last overall sums each slice's tiles.
        const bool one = set.n == 1;
        unsigned long long *mine = &partials[one ? (int)blockIdx.x : tile];
        // first exchange: noise powers
        if (packed) {
            // one slice whose sum fits the packed word: the packed round (no partials array,
            // no fences; the total travels in the release itself)
            if (tid == 0) {
                unsigned long long b = 0;
                for (int i = 0; i < NT / 64; ++i) b += s_wsum[i];
                unsigned long long total = 0;
                s_role = rg.arrive_packed(b, total);
                s_res[0] = total;
            }
            __syncthreads();
            if (s_role == 2) rg.release_packed(s_res[0]);
            if (tid == 0) {
                unsigned long long total = s_res[0];
                const int ok = s_role == 2 || rg.wait_packed(s_pack0, total);
                const SliceExtent e = slice_extent(set, 0);
                const double n = (double)(wh * ww), npx = (double)e.h * (double)e.w;
                const double v = npx > 0 ? (double)total / (n * n * npx) : 0.0;
                if (s_role == 2 && nu2) nu2[0] = v;  // the caller's copy, read after the launch
                s_res[0] = (unsigned long long)__double_as_longlong(v);
                s_ok = ok;
            }
            __syncthreads();
        } else {
        if (tid == 0) {
            unsigned long long b = 0;
            for (int i = 0; i < NT / 64; ++i) b += s_wsum[i];
            s_ok = 1;
            s_role = rg.arrive_group(mine, b) ? 1 : 0;
        }
        __syncthreads();
        if (s_role == 1) {
            if (one) {
                unsigned long long lo = 0, hi = 0;
                if (tid < rg.group_size()) lo = sync_read64(&partials[rg.group_first() + tid]);
                block_sum_u128(lo, hi, s_lo, s_hi);
                if (tid == 0) {
                    (void)sync_xchg64(rg.summary(rg.g), lo);
                    (void)sync_xchg64(rg.summary(rg.g) + 1, hi);
                }
            }
            if (tid == 0) s_role = rg.arrive_top() ? 2 : 1;
            __syncthreads();
        }
        if (s_role == 2) {
            const double n = (double)(wh * ww);
            for (int i = 0; i < set.n; ++i) {
                const SliceExtent e = slice_extent(set, i);
                unsigned long long lo = 0, hi = 0;
                if (one) {
                    if (tid < rg.ng) {
                        lo = sync_read64(rg.summary(tid));
                        hi = sync_read64(rg.summary(tid) + 1);
                    }
                } else {
                    for (int k = tid; k < e.ntiles; k += NT) {
                        const unsigned long long pv = sync_read64(&partials[e.tile_begin + k]);
                        lo += pv;
                        hi += (lo < pv);
                    }
                }
                block_sum_u128(lo, hi, s_lo, s_hi);
                if (tid == 0) {
                    // nu2 = exact sum / (N^2 h w), as in the stand-alone reduction
                    const double total = (double)hi * 18446744073709551616.0 + (double)lo;
                    const double npx = (double)e.h * (double)e.w;
                    const double v = npx > 0 ? total / (n * n * npx) : 0.0;
                    s_res[i] = (unsigned long long)__double_as_longlong(v);
                    if (nu2) nu2[i] = v;  // the caller's copy, read after the launch
                }
                __syncthreads();
            }
            rg.release(s_res, set.n, 64);
        }
        if (tid == 0) {
            const int ok = s_role == 2 || rg.wait(s_flag0);
            if (s_role != 2) s_res[si] = rg.result(64, si);
            s_ok = ok;
        }
        __syncthreads();
        }
        const double nu2d = s_ok ? __longlong_as_double((long long)s_res[si])
                                 : __longlong_as_double(0x7ff8000000000000ll);

        // 7. Wiener output of the tile's pixels
        const WienerConst wc = with_noise(wcb, nu2d);
        float y[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) y[j] = wiener_finish(wp[j], wc);
        float *orow = sd.out + (long long)(y0 + j0) * sd.out_pitch + x0 + lane;
        if (stretch) {
            // second exchange: the slice's output range, then the stretch of the tile's outputs
            float mn = __builtin_inff(), mx = -__builtin_inff();
#pragma unroll
            for (int j = 0; j < RPT; ++j)
                if (col_ok && j < rows_ok) {
                    mn = fminf(mn, y[j]);
                    mx = fmaxf(mx, y[j]);
                }
            block_minmax(mn, mx, s_lo, s_hi);
            __syncthreads();
            if (tid == 0) s_role = rg.arrive_group(mine, pack_range(mn, mx)) ? 1 : 0;
            __syncthreads();
            if (s_role == 1) {
                if (one) {
                    float a = __builtin_inff(), b = -__builtin_inff();
                    if (tid < rg.group_size()) {
                        const unsigned long long pv = sync_read64(&partials[rg.group_first() + tid]);
                        a = range_lo(pv);
                        b = range_hi(pv);
                    }
                    block_minmax(a, b, s_lo, s_hi);
                    if (tid == 0) (void)sync_xchg64(rg.summary(rg.g), pack_range(a, b));
                }
                if (tid == 0) s_role = rg.arrive_top() ? 2 : 1;
                __syncthreads();
            }
            if (s_role == 2) {
                for (int i = 0; i < set.n; ++i) {
                    const SliceExtent e = slice_extent(set, i);
                    float a = __builtin_inff(), b = -__builtin_inff();
                    if (one) {
                        if (tid < rg.ng) {
                            const unsigned long long pv = sync_read64(rg.summary(tid));
                            a = range_lo(pv);
                            b = range_hi(pv);
                        }
                    } else {
                        for (int k = tid; k < e.ntiles; k += NT) {
                            const unsigned long long pv = sync_read64(&partials[e.tile_begin + k]);
                            a = fminf(a, range_lo(pv));
                            b = fmaxf(b, range_hi(pv));
                        }
                    }
                    block_minmax(a, b, s_lo, s_hi);
                    if (tid == 0) s_res[i] = pack_range(a, b);
                    __syncthreads();
                }
                rg.release(s_res, set.n, 96);
            }
            if (tid == 0) {
                // the flag moved once in the first exchange unless that exchange was packed
                const int ok = s_role == 2 || rg.wait(s_flag0 + (packed ? 0u : 1u));
                if (s_role != 2) s_res[si] = rg.result(96, si);
                s_ok = s_ok && ok;
            }
            __syncthreads();
            const unsigned long long rr = s_ok ? s_res[si] : pack_range(__builtin_nanf(""), __builtin_nanf(""));
            const float lo = range_lo(rr), hi = range_hi(rr);
#pragma unroll
            for (int j = 0; j < RPT; ++j) y[j] = stretch_pixel(y[j], lo, hi);
        }
        // a workgroup whose wait gave up has no valid noise power or range: NaN, explicitly
        // (the Wiener gain's max() would otherwise turn a NaN noise power into gain 0)
        const float fail_nan = __builtin_nanf("");
#pragma unroll
        for (int j = 0; j < RPT; ++j)
            if (col_ok && j < rows_ok) orow[(long long)j * sd.out_pitch] = s_ok ? y[j] : fail_nan;
    }
}

template <bool RESIDENT>
hipError_t launch_amf(const SliceSet &set, int total_tiles, int eb, int smax, int keep, int wh,
                      int ww, unsigned long long *partials, int select_mode, bool aligned,
                      float mf, unsigned int *words, double *nu2, int store_amf, int stretch,
                      int packed, int lds_bytes, unsigned int *err, unsigned long long wait_limit,
                      hipStream_t s, int tile_rows = TILE_Y) {
    if (tile_rows != TILE_Y &&
        (RESIDENT || wh > 0 || set.list || (tile_rows != TILE_Y / 2 && tile_rows != 2 * TILE_Y)))
        return hipErrorInvalidValue;
    const AmfSmem L = amf_smem_layout(eb, smax, wh, ww, RESIDENT ? RESIDENT_STRIP : STAGED_STRIP, tile_rows);
    const int lds = lds_bytes > L.total ? lds_bytes : L.total;
    const WienerConst wcb = wiener_const(RESIDENT ? wh : 0, RESIDENT ? ww : 0, mf);
    const int maw = div_region_magic(L.AW);
    const dim3 grid(tile_rows < TILE_Y ? 2 * total_tiles : total_tiles), block(NT);
    const bool dense = select_mode == SELECT_DENSE;
    const int al = aligned ? 1 : 0;
#define HD_LAUNCH_AMF(TY, DN)                                                                         \
    hipLaunchKernelGGL((amf_stage_kernel<TY, DN, RESIDENT>), grid, block, lds, s, set, total_tiles,     \
                       smax, keep, wh, ww, partials, select_mode, al, mf, words, nu2, store_amf, stretch, \
                       packed, wcb, maw, err, wait_limit, tile_rows)
    if (eb == 1) {
        if (dense) HD_LAUNCH_AMF(uint8_t, true);
        else HD_LAUNCH_AMF(uint8_t, false);
    } else {
        if (dense) HD_LAUNCH_AMF(uint16_t, true);
        else HD_LAUNCH_AMF(uint16_t, false);
    }
#undef HD_LAUNCH_AMF
    return hipGetLastError();
}

}  // namespace

hipError_t launch_amf_stage(const SliceSet &set, int total_tiles, int eb, int smax, int keep,
                            int wh, int ww, unsigned long long *partials, int select_mode,
                            bool aligned, hipStream_t s, int tile_rows) {
    return launch_amf<false>(set, total_tiles, eb, smax, keep, wh, ww, partials, select_mode, aligned,
                             1.0f, nullptr, nullptr, 0, 0, 0, 0, nullptr, 0, s, tile_rows);
}

hipError_t launch_hybrid_resident(const SliceSet &set, int total_tiles, int eb, int smax, int keep,
                                  int wh, int ww, int max_value, unsigned long long *partials,
                                  unsigned int *sync_words, double *nu2, int select_mode,
                                  bool aligned, bool store_amf, bool stretch, int lds_bytes,
                                  unsigned long long wait_limit, hipStream_t s) {
    unsigned int *err = device_error_word();
    if (!err) return hipErrorInvalidSymbol;
    // every group's partials are summed by one workgroup: at most NT of them per group
    if (total_tiles > RESIDENT_MAX_GROUPS * resident_group_size(total_tiles) || total_tiles > RESIDENT_MAX_BLOCKS ||
        set.n > RESIDENT_MAX_SLICES ||
        resident_group_size(total_tiles) > NT)
        return hipErrorInvalidValue;
    // the packed round needs one slice and a total below 2^56: N * S2 - S1^2 = N^2 var <=
    // N^2 (V / 2)^2 per pixel (N = window size, V = the dtype's largest value: pixels above
    // the declared max value are allowed), summed over every tile's pixels; one bit of
    // margin. Always true for 8-bit data.
    const double n = (double)wh * ww, v = eb == 1 ? 255.0 : 65535.0;
    const double bound = n * n * (v * v / 4.0) * (double)(TILE_X * TILE_Y) * total_tiles;
    const int packed = set.n == 1 && bound < 36028797018963968.0 /* 2^55 */ ? 1 : 0;
    return launch_amf<true>(set, total_tiles, eb, smax, keep, wh, ww, partials, select_mode, aligned,
                            (float)max_value, sync_words, nu2, store_amf ? 1 : 0, stretch ? 1 : 0, packed,
                            lds_bytes, err, wait_limit, s);
}

unsigned int *device_error_word() {
    // the symbol's address on each device, looked up once with that device current
    constexpr int kMaxDevices = 64;
    static std::atomic<unsigned int *> addr[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    unsigned int *p = addr[dev].load();
    if (!p) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(g_error_word)) != hipSuccess || !q) {
            (void)hipGetLastError();
            return nullptr;
        }
        p = (unsigned int *)q;
        addr[dev].store(p);
    }
    return p;
}

static const void *resident_fn(int eb, int select_mode) {
    const bool dense = select_mode == SELECT_DENSE;
    if (eb == 1) return dense ? (const void *)amf_stage_kernel<uint8_t, true, true>
                              : (const void *)amf_stage_kernel<uint8_t, false, true>;
    return dense ? (const void *)amf_stage_kernel<uint16_t, true, true>
                 : (const void *)amf_stage_kernel<uint16_t, false, true>;
}

int resident_capacity(int eb, int smax, int wh, int ww, int select_mode) {
    const AmfSmem L = amf_smem_layout(eb, smax, wh, ww, RESIDENT_STRIP);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, resident_fn(eb, select_mode), NT, L.total) !=
            hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return std::min(per_cu * cus, RESIDENT_MAX_BLOCKS);
}

int resident_lds_bytes(int eb, int smax, int wh, int ww, int select_mode, int total_tiles) {
    const AmfSmem L = amf_smem_layout(eb, smax, wh, ww, RESIDENT_STRIP);
    const void *fn = resident_fn(eb, select_mode);
    int dev = 0, cus = 0, lds_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, L.total) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        return L.total;
    }
    const int want = (total_tiles + cus - 1) / cus;
    if (want < 1 || want >= per_cu) return L.total;
    // the smallest size, in 256-byte steps, at which at most `want` workgroups fit a CU
    int b = lds_cu / (want + 1);
    b = (b > L.total ? b : L.total) & ~255;
    for (; b <= 65536; b += 256) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, NT, b) != hipSuccess) {
            (void)hipGetLastError();
            return L.total;
        }
        if (occ <= want) return occ == want ? b : L.total;
    }
    return L.total;
}

}  // namespace hd

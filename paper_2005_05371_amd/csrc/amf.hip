// Adaptive median filter (AMF) for gfx950.
//
// Method (arXiv 2005.05371, Alg. 1, procedure parallelAdapMedian): for every pixel try
// windows k = 3, 5, ..., Smax in order; at level k take zmin, zmax, zmed of the k x k
// window; stage A passes when zmin < zmed < zmax and resolves the pixel: it keeps g when
// zmin < g < zmax (stage B), else takes zmed. A pixel never passing stage A takes zmed of
// the Smax window (or keeps g in keep mode).
//
// Design:
//  * one workgroup (256 threads = 4 waves) per 64 x 32 output tile; the tile plus an
//    Smax/2 halo (symmetric padding) is staged once in LDS as 16-bit values;
//  * level 3 runs for every pixel with a register network: each thread owns a column
//    strip of 8 pixels, sorts each row triple once (min3 / med3 / max3, shared by the
//    three pixels whose windows contain it) and gets zmin, zmax, zmed of the 3 x 3
//    window from the row triples (median of 9 = med3(max of row minima, med of row
//    medians, min of row maxima));
//  * pixels that fail stage A are compacted into an LDS list (wave ballot + one LDS
//    atomic per wave); each deeper level runs only over that list, with all lanes busy,
//    and re-compacts what is still unresolved, so lanes that resolve early never pay for
//    larger windows;
//  * at level k >= 5 stage A is decided from counts, without sorting: zmed > zmin iff
//    fewer than (k^2 + 1) / 2 samples equal zmin, and zmed < zmax iff fewer than
//    (k^2 + 1) / 2 samples equal zmax. zmed itself is only needed when the centre pixel
//    is an extreme of the window (or at Smax); it is found exactly as the smallest
//    value t with #(v <= t) >= (k^2 + 1) / 2, by bisection over the value range.
#include "hd_internal.h"

namespace hd {
namespace {

constexpr int TX = 64;               // tile width: one wave spans a tile row
constexpr int TY = 32;               // tile height
constexpr int NT = 256;              // threads per workgroup
constexpr int RPT = TY / (NT / TX);  // pixels per thread in the level-3 pass (8)
constexpr int RMAX = 15;             // largest window radius (Smax 31)
constexpr int LDS_IN = (TY + 2 * RMAX) * (TX + 2 * RMAX);

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
    return min(min(a, b), c);
}
__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) {
    return max(max(a, b), c);
}
__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}

// One level k >= 5 for the pixel whose window centre is `c` (LDS, row pitch lp).
// Returns the output value; `resolved` tells whether stage A passed. When stage A fails
// and this is not the last level the return value is unused.
template <int K>
__device__ uint32_t amf_level(const uint16_t *c, int lp, uint32_t g, bool last, bool keep,
                              bool &resolved) {
    constexpr int r = K / 2;
    constexpr uint32_t half = (K * K - 1) / 2;  // 0-based rank of the median
    constexpr int UR = (K <= 9) ? K : 1;
    uint32_t mn = 0xffffu, mx = 0u;
#pragma unroll UR
    for (int dy = -r; dy <= r; ++dy) {
        const uint16_t *row = c + dy * lp;
#pragma unroll
        for (int dx = -r; dx <= r; ++dx) {
            const uint32_t v = row[dx];
            mn = min(mn, v);
            mx = max(mx, v);
        }
    }
    uint32_t cmin = 0, cmax = 0;
#pragma unroll UR
    for (int dy = -r; dy <= r; ++dy) {
        const uint16_t *row = c + dy * lp;
#pragma unroll
        for (int dx = -r; dx <= r; ++dx) {
            const uint32_t v = row[dx];
            cmin += (v == mn);
            cmax += (v == mx);
        }
    }
    const bool stage_a = (cmin <= half) && (cmax <= half);
    resolved = stage_a;
    if (stage_a && g != mn && g != mx) return g;  // stage B: keep the centre value
    if (!stage_a && (!last || keep)) return g;    // requeued, or keep-mode final value
    // zmed: smallest t with #(v <= t) >= half + 1; strictly inside (mn, mx) under stage A
    uint32_t lo = stage_a ? mn + 1 : mn;
    uint32_t hi = stage_a ? mx - 1 : mx;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        uint32_t cnt = 0;
#pragma unroll UR
        for (int dy = -r; dy <= r; ++dy) {
            const uint16_t *row = c + dy * lp;
#pragma unroll
            for (int dx = -r; dx <= r; ++dx) cnt += (uint32_t(row[dx]) <= mid);
        }
        if (cnt > half) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ uint32_t amf_level_dispatch(int k, const uint16_t *c, int lp, uint32_t g, bool last,
                                       bool keep, bool &resolved) {
    switch (k) {
        case 5: return amf_level<5>(c, lp, g, last, keep, resolved);
        case 7: return amf_level<7>(c, lp, g, last, keep, resolved);
        case 9: return amf_level<9>(c, lp, g, last, keep, resolved);
        case 11: return amf_level<11>(c, lp, g, last, keep, resolved);
        case 13: return amf_level<13>(c, lp, g, last, keep, resolved);
        case 15: return amf_level<15>(c, lp, g, last, keep, resolved);
        case 17: return amf_level<17>(c, lp, g, last, keep, resolved);
        case 19: return amf_level<19>(c, lp, g, last, keep, resolved);
        case 21: return amf_level<21>(c, lp, g, last, keep, resolved);
        case 23: return amf_level<23>(c, lp, g, last, keep, resolved);
        case 25: return amf_level<25>(c, lp, g, last, keep, resolved);
        case 27: return amf_level<27>(c, lp, g, last, keep, resolved);
        case 29: return amf_level<29>(c, lp, g, last, keep, resolved);
        default: return amf_level<31>(c, lp, g, last, keep, resolved);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void amf_tile_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                      int H, int W, long long ip, long long op,
                                                      int smax, int keep) {
    __shared__ uint16_t s_in[LDS_IN];
    __shared__ uint16_t s_out[TY * TX];
    __shared__ uint16_t s_list[2][TY * TX];
    __shared__ int s_cnt[2];

    const int R = smax >> 1;
    const int lp = TX + 2 * R;
    const int lh = TY + 2 * R;
    const int x0 = blockIdx.x * TX;
    const int y0 = blockIdx.y * TY;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;

    // 1. tile + halo -> LDS (mirrored indices at the image border)
    for (int ly = wv; ly < lh; ly += NT / 64) {
        const T *src = in + (long long)mirror(y0 + ly - R, H) * ip;
        uint16_t *dst = s_in + ly * lp;
        for (int lx = lane; lx < lp; lx += 64) dst[lx] = (uint16_t)src[mirror(x0 + lx - R, W)];
    }
    if (tid < 2) s_cnt[tid] = 0;
    __syncthreads();

    // 2. level 3 for all pixels: row triples sorted once, shared by 3 output rows
    const int rb = wv * RPT;
    const bool col_ok = (x0 + lane) < W;
    uint32_t lo[RPT + 2], md[RPT + 2], hi[RPT + 2], ctr[RPT + 2];
#pragma unroll
    for (int j = 0; j < RPT + 2; ++j) {
        const uint16_t *p = s_in + (rb + j - 1 + R) * lp + lane + R;
        const uint32_t a = p[-1], b = p[0], c = p[1];
        lo[j] = min3u(a, b, c);
        md[j] = med3u(a, b, c);
        hi[j] = max3u(a, b, c);
        ctr[j] = b;
    }
    const bool last3 = (smax == 3);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const uint32_t zmin = min3u(lo[j], lo[j + 1], lo[j + 2]);
        const uint32_t zmax = max3u(hi[j], hi[j + 1], hi[j + 2]);
        const uint32_t zmed = med3u(max3u(lo[j], lo[j + 1], lo[j + 2]),
                                    med3u(md[j], md[j + 1], md[j + 2]),
                                    min3u(hi[j], hi[j + 1], hi[j + 2]));
        const uint32_t g = ctr[j + 1];
        const bool stage_a = (zmin < zmed) && (zmed < zmax);
        uint32_t res;
        if (stage_a) res = (zmin < g && g < zmax) ? g : zmed;
        else res = keep ? g : zmed;  // final only when Smax == 3
        const int idx = (rb + j) * TX + lane;
        s_out[idx] = (uint16_t)res;
        const bool defer = col_ok && (y0 + rb + j) < H && !stage_a && !last3;
        const unsigned long long bal = __ballot(defer);
        if (bal) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&s_cnt[0], (int)__popcll(bal));
            base = __shfl(base, 0);
            if (defer) s_list[0][base + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)idx;
        }
    }
    __syncthreads();

    // 3. deeper levels over the compacted list of still-unresolved pixels
    int cur = 0;
    for (int k = 5; k <= smax; k += 2) {
        const int n = s_cnt[cur];
        if (n == 0) break;  // uniform: read after a barrier
        const int nxt = cur ^ 1;
        const bool last = (k == smax);
        for (int i = tid; i < n; i += NT) {
            const int idx = s_list[cur][i];
            const int py = idx / TX, px = idx % TX;
            const uint16_t *c = s_in + (py + R) * lp + px + R;
            const uint32_t g = *c;
            bool resolved;
            const uint32_t v = amf_level_dispatch(k, c, lp, g, last, keep != 0, resolved);
            if (resolved || last) {
                s_out[idx] = (uint16_t)v;
            } else {
                const int pos = atomicAdd(&s_cnt[nxt], 1);
                s_list[nxt][pos] = (uint16_t)idx;
            }
        }
        __syncthreads();
        if (tid == 0) s_cnt[cur] = 0;
        __syncthreads();
        cur = nxt;
    }

    // 4. tile -> global
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int y = y0 + rb + j;
        if (col_ok && y < H) out[(long long)y * op + x0 + lane] = (T)s_out[(rb + j) * TX + lane];
    }
}

}  // namespace

hipError_t launch_amf(const void *in, void *out, int h, int w, long long in_pitch,
                      long long out_pitch, int dt_bytes, int smax, int keep, hipStream_t s) {
    const dim3 grid((w + TX - 1) / TX, (h + TY - 1) / TY);
    if (dt_bytes == 1) {
        hipLaunchKernelGGL(amf_tile_kernel<uint8_t>, grid, dim3(NT), 0, s,
                           (const uint8_t *)in, (uint8_t *)out, h, w, in_pitch, out_pitch, smax, keep);
    } else {
        hipLaunchKernelGGL(amf_tile_kernel<uint16_t>, grid, dim3(NT), 0, s,
                           (const uint16_t *)in, (uint16_t *)out, h, w, in_pitch, out_pitch, smax, keep);
    }
    return hipGetLastError();
}

}  // namespace hd

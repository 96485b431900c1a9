// Internal declarations shared by the HIP translation units of libhybrid_denoise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

// Output tile of every stage kernel: 64 columns (one wave) x 32 rows, 256 threads.
constexpr int TILE_X = 64;
constexpr int TILE_Y = 32;
constexpr int STAGE_THREADS = 256;
constexpr int RMAX_AMF = 15;   // Smax <= 31
constexpr int RMAX_WIN = 7;    // Wiener window side <= 15

// Symmetric (half-sample) mirror of i into [0, n), period 2n: ... c b a | a b c | c b a ...
// Reflects at the nearer edge until inside: one step for any index less than n past an
// edge, more only for images narrower than a window radius (compact code, no division).
__host__ __device__ __forceinline__ int mirror(int i, int n) {
    while ((unsigned)i >= (unsigned)n) i = (i < 0) ? -1 - i : 2 * n - 1 - i;
    return i;
}

// One image of a (possibly batched) call. Pitches are in elements.
struct SliceDesc {
    const void *in;    // stage-1 input g (AMF), or the integer image of a Wiener-only call
    void *amf;         // AMF output a (stage-1 output, stage-2 input)
    float *out;        // Wiener output
    long long in_pitch, amf_pitch, out_pitch;
    int h, w;
    int tiles_x;       // ceil(w / TILE_X)
    int tile_begin;    // index of this slice's first tile in the launch
};

// Either one slice passed by value, or a device table of n slices. With `list` set, the
// stage kernels work on the listed tiles only (global tile ids, *list_count of them; the
// grid may be larger), and the noise reduction sums only tiles whose flag is set.
struct SliceSet {
    SliceDesc one;
    const SliceDesc *many;  // device memory, n entries, tile_begin ascending
    int n;
    const int *list = nullptr;
    const int *list_count = nullptr;
    const int *flags = nullptr;
};

// Per-call options of the selection strategy for the median at window levels >= 5.
enum SelectMode : int {
    SELECT_AUTO = 0,    // short pending lists: one wave per pixel through all its levels;
                        // long lists, level by level: one lane per pixel (bisection) when
                        // the list fills the workgroup, else one wave per pixel
    SELECT_BISECT = 1,  // one lane per pixel, bisection over the value range at every level
    SELECT_WAVE = 2,    // one wave per pixel at every level >= 5, level by level
    SELECT_DENSE = 3,   // as AUTO, with a register sorting network for the 5x5 median and
                        // lane groups from level 7 on (the variant for dense impulse noise)
};

// Host option HD_OPT_SURROGATE_FUSED (the surrogate's inference kernels).
bool surrogate_fused_inference();

// Dynamic LDS bytes of the AMF stage kernel (host and device agree on the layout).
struct AmfSmem {
    int R, rh, rw, AH, AW, IH, IW, nch_max, in_bytes, amf_bytes, list_bytes, mom_bytes, total;
};
// Rows per strip of the level-3 pass: 8 in the staged kernel (a 32-row region is exactly
// 256 strips of one column), 12 in the resident one (its 34- or 36-row region with the
// Wiener ring then takes one strip per thread instead of two for a third of them).
constexpr int STAGED_STRIP = 8;
constexpr int RESIDENT_STRIP = 12;
// `rows`: the AMF tile's height (the staged stage without the Wiener ring may run 16-, 32-
// or 64-row tiles; everything else uses TILE_Y).
__host__ __device__ inline AmfSmem amf_smem_layout(int eb, int smax, int wh, int ww, int strip, int rows_t = TILE_Y) {
    AmfSmem s;
    s.R = smax / 2;
    s.rh = wh / 2;
    s.rw = ww / 2;
    s.AH = rows_t + 2 * s.rh;
    s.AW = TILE_X + 2 * s.rw;
    // the level-3 pass works in strips of `strip` rows; rows past AH are computed and ignored
    const int rows = (s.AH + strip - 1) / strip * strip;
    s.IH = rows + 2 * s.R;
    s.IW = s.AW + 2 * s.R;
    s.nch_max = (15 + s.IW * eb + 15) / 16;
    s.in_bytes = s.IH * (s.nch_max | 1) * 16;  // the row pitch is an odd number of chunks
    s.amf_bytes = ((rows * s.AW * eb) + 15) & ~15;
    s.list_bytes = 2 * s.AH * s.AW * 2;
    const int s2b = eb == 1 ? 4 : 8;
    s.mom_bytes = (wh > 0) ? s.AH * TILE_X * (4 + s2b) : 0;
    const int u1 = s.in_bytes + s.list_bytes;
    s.total = s.amf_bytes + (u1 > s.mom_bytes ? u1 : s.mom_bytes);
    return s;
}

// Dynamic LDS bytes of the Wiener stage kernel.
__host__ __device__ inline int wiener_smem_bytes(int eb, int wh, int ww) {
    const int rh = wh / 2, rw = ww / 2;
    const int rows = TILE_Y + 2 * rh, cols = TILE_X + 2 * rw;
    const int nch_max = (15 + cols * eb + 15) / 16;
    const int in_bytes = rows * nch_max * 16;
    const int s2b = eb == 1 ? 4 : 8;
    return in_bytes + rows * TILE_X * (4 + s2b);
}

// ---- launchers (all asynchronous on `s`) -------------------------------------------
// Stage 1: AMF of every tile of `set`; with wh, ww > 0 also the exact sum of the Wiener
// variance numerators N*S2 - S1^2 of the tile's pixels into partials[tile] (AMF is also
// computed on the window ring around the tile so that the tile needs no neighbour).
// tile_rows (16, 32 or 64; only 32 with the Wiener ring or a tile list): the AMF tile's
// height. 16: two workgroups per 64 x 32 tile; 64: the workgroups of odd tile rows exit and
// the even row's workgroup covers both.
hipError_t launch_amf_stage(const SliceSet &set, int total_tiles, int eb, int smax, int keep,
                            int wh, int ww, unsigned long long *partials, int select_mode,
                            bool aligned, hipStream_t s, int tile_rows = TILE_Y);

// The whole hybrid in one launch (estimated noise power, no tile list): AMF with the
// window ring, window sums, per-tile partials, a grid-wide barrier whose last arrival
// turns the partials of every slice into nu2[i] (as launch_noise_reduce), Wiener output;
// with `stretch`, a second barrier for every slice's output range and the contrast stretch
// before the store. For at most RESIDENT_MAX_SLICES slices (the last arrival reduces them
// one after another). Requires every tile's workgroup to be resident at once:
// total_tiles <= resident_capacity(...). sync_words (RESIDENT_SYNC_WORDS words) must be zero before the
// first launch; later launches reuse them as left. AMF output is written only with
// store_amf. lds_bytes: dynamic LDS per workgroup, at least the layout's (0: the layout's).
// Launches sharing sync_words must not overlap.
constexpr int RESIDENT_MAX_GROUPS = 128;
constexpr int RESIDENT_MAX_SLICES = 8;
constexpr int RESIDENT_SLOT_WORDS = 1024;  // 4 KB per group slot; slot 0 holds the header
constexpr int RESIDENT_GROUP_WORDS = RESIDENT_SLOT_WORDS * (RESIDENT_MAX_GROUPS + 1);
// then one release word per workgroup, 128 bytes apart (each waiter polls its own line)
constexpr int RESIDENT_MAX_BLOCKS = 4096;
constexpr int RESIDENT_BLOCK_WORDS = 32;
constexpr int RESIDENT_SYNC_WORDS = RESIDENT_GROUP_WORDS + RESIDENT_BLOCK_WORDS * RESIDENT_MAX_BLOCKS;
// a power of two (the group index is a shift), at least 32, at most RESIDENT_MAX_GROUPS groups
__host__ __device__ inline int resident_group_size(int blocks) {
    const int g = (blocks + RESIDENT_MAX_GROUPS - 1) / RESIDENT_MAX_GROUPS;
    int p = 32;
    while (p < g) p <<= 1;
    return p;
}
// wait_limit: bound of every exchange wait in ticks of the 100 MHz real-time counter (0: a
// workgroup that would wait gives up at once); a workgroup that gives up sets bit 0 of
// the device's error word and writes NaN.
hipError_t launch_hybrid_resident(const SliceSet &set, int total_tiles, int eb, int smax, int keep,
                                  int wh, int ww, int max_value, unsigned long long *partials,
                                  unsigned int *sync_words, double *nu2, int select_mode,
                                  bool aligned, bool store_amf, bool stretch, int lds_bytes,
                                  unsigned long long wait_limit, hipStream_t s);

// Address of the current device's error word (a file-scope device variable), looked up
// once per device; null when the lookup fails.
unsigned int *device_error_word();

// Workgroups of the resident kernel that the current device holds at once (0 on error).
int resident_capacity(int eb, int smax, int wh, int ww, int select_mode);

// Dynamic LDS per workgroup of the resident kernel for total_tiles tiles: enough to cap the
// occupancy at ceil(total_tiles / CUs) workgroups per CU, so that no CU holds more than one
// tile above the average (the slowest CU sets the barrier's time); the layout's own size
// when that cap would not lower the occupancy or cannot be reached within 64 KB.
int resident_lds_bytes(int eb, int smax, int wh, int ww, int select_mode, int total_tiles);

// Per-slice noise power: nu2[i] = sum(partials of slice i) / (N^2 h w), exact integer sum.
hipError_t launch_noise_reduce(const SliceSet &set, const unsigned long long *partials,
                               int wh, int ww, double *nu2, hipStream_t s);

// Stage 2 on the integer image `amf` of every slice: with apply, out = Wiener output using
// nu2[slice] (nu2 != null) or noise_var; without apply, only partials[tile].
hipError_t launch_wiener_stage(const SliceSet &set, int total_tiles, int eb, int max_value,
                               int wh, int ww, bool apply, const double *nu2, double noise_var,
                               unsigned long long *partials, bool aligned, hipStream_t s,
                               unsigned long long *ranges = nullptr);

// Per-tile (min, max) of the float outputs `out` of every slice.
hipError_t launch_tile_ranges(const SliceSet &set, int total_tiles, unsigned long long *tile_ranges,
                              hipStream_t s);

// Contrast stretch of every slice's Wiener output in place: the slice's range from the
// per-tile ranges that the apply wrote (tile_ranges), then out = (out - min) / (max - min).
// slice_ranges: one word per slice of scratch.
hipError_t launch_stretch(const SliceSet &set, int total_tiles, const unsigned long long *tile_ranges,
                          unsigned long long *slice_ranges, hipStream_t s);

// Sets the calling thread's message returned by hd_last_error().
void set_error_message(const char *msg);

// *p = v (one device double), as a kernel so that it can sit in a captured graph.
hipError_t launch_fill_f64(double *p, double v, hipStream_t s);

// Degraded copy of a clean integer image (Gaussian, then salt and pepper; Philox4x32-10
// stream `stream_id` under `seed`). noisy may equal clean (in place).
hipError_t launch_degrade(const void *clean, void *noisy, int h, int w, long long cpitch, long long npitch,
                          int eb, int max_value, double sigma, double density, unsigned long long seed,
                          uint32_t stream_id, hipStream_t s);

// Frequency-domain Wiener step (see fft.hip): lengths up to FFT_MAX_LEN whose prime
// factors are 2, 3 and 5.
constexpr int FFT_MAX_LEN = 4096;
bool fft_size_ok(int n);
size_t wiener_fft_scratch_bytes(int h, int w);
hipError_t launch_wiener_fft(const void *a, long long ap, const void *f, long long fp, float *out, long long op,
                             int h, int w, int eb, int max_value, void *scratch, hipStream_t s);

// Device table of the `parts` strips of an image (see strip_table_kernel); parts <= 256.
hipError_t launch_strip_table(SliceDesc *table, const void *in, void *out, int h, int w,
                              long long in_pitch, long long out_pitch, int eb, int parts, hipStream_t s);

// p[0 .. n) = 0 with a kernel (safe inside a captured graph, unlike a memset node).
hipError_t launch_zero_u32(unsigned int *p, int n, hipStream_t s);

}  // namespace hd

// C ABI of libhybrid_denoise: argument checks, scratch management, launch sequencing,
// batched plans (device slice table + captured hipGraph) and the strategy autotuner.
// The declarations and their contract are in include/hybrid_denoise.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hybrid_denoise.h"
#include "hd_internal.h"

namespace {

thread_local char g_last_error[512] = "";

hd_status fail(hd_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

hd_status ok() {
    g_last_error[0] = '\0';
    return HD_OK;
}

hd_status hip_fail(hipError_t e, const char *what) {
    return fail(HD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int dtype_bytes(int32_t dt) { return dt == HD_U8 ? 1 : (dt == HD_U16 ? 2 : 0); }

// Tile counts and LDS indices stay far inside int range below this side length; with
// pitches up to 2^32 elements every byte span (h - 1) * pitch * 4 + w * 4 < 2^55 fits in
// int64 and size_t arithmetic.
constexpr int32_t kMaxSide = 1 << 20;
constexpr int64_t kMaxPitch = 1LL << 32;
constexpr long long kMaxTiles = 1LL << 30;

hd_status check_image(const void *p, int32_t h, int32_t w, int64_t pitch, const char *name) {
    if (!p) return fail(HD_ERR_NULL, "%s is NULL", name);
    if (h < 1 || w < 1 || h > kMaxSide || w > kMaxSide)
        return fail(HD_ERR_DIMS, "bad dimensions %d x %d (each must be in 1..%d)", h, w, kMaxSide);
    if (pitch < w) return fail(HD_ERR_DIMS, "%s pitch %lld < width %d", name, (long long)pitch, w);
    if (pitch > kMaxPitch)
        return fail(HD_ERR_DIMS, "%s pitch %lld above %lld elements", name, (long long)pitch, (long long)kMaxPitch);
    return HD_OK;
}

hd_status check_smax(int32_t smax) {
    if (smax <= 1 || (smax % 2) == 0)
        return fail(HD_ERR_SMAX, "SMAX must be an odd integer > 1 (got %d)", smax);
    if (smax > HD_SMAX_LIMIT)
        return fail(HD_ERR_SMAX, "Smax %d above the library limit %d", smax, HD_SMAX_LIMIT);
    return HD_OK;
}

hd_status check_window(int32_t wh, int32_t ww) {
    if (wh < 1 || ww < 1 || (wh % 2) == 0 || (ww % 2) == 0 || wh > HD_WIN_LIMIT || ww > HD_WIN_LIMIT)
        return fail(HD_ERR_WINDOW, "Wiener window %d x %d must be odd, 1..%d", wh, ww, HD_WIN_LIMIT);
    return HD_OK;
}

hd_status check_maxval(int32_t m, int32_t dt) {
    const int32_t top = dt == HD_U8 ? 255 : 65535;
    if (m < 1 || m > top) return fail(HD_ERR_MAXVAL, "max_value %d outside 1..%d", m, top);
    return HD_OK;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

size_t span_bytes(int32_t h, int32_t w, int64_t pitch, int elem) {
    return ((size_t)(h - 1) * (size_t)pitch + (size_t)w) * (size_t)elem;
}

bool aligned16(const void *p, int64_t pitch, int eb) {
    return ((uintptr_t)p & 15) == 0 && ((pitch * eb) & 15) == 0;
}

int tiles_x_of(int w) { return (w + hd::TILE_X - 1) / hd::TILE_X; }
int tiles_of(int h, int w) { return tiles_x_of(w) * ((h + hd::TILE_Y - 1) / hd::TILE_Y); }
int64_t amf_pitch_of(int w, int eb) { return (((int64_t)w * eb + 15) / 16 * 16) / eb; }
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---- options and autotuned strategies ----------------------------------------------
std::atomic<int> g_select_mode{-1};  // -1: autotuned / default
std::atomic<int> g_fuse{-1};         // -1: autotuned / default
std::atomic<int> g_use_graph{1};
std::atomic<int> g_resident{-1};     // -1: default (on)
std::atomic<int> g_sg_fused{0};      // surrogate inference in one row-streaming launch
std::atomic<int> g_tile_rows{-1};    // -1: autotuned / default (32)
// bound of every wait in the resident kernel's exchange, in microseconds (default 1 s)
constexpr long long kDefaultWaitUs = 1000000;
std::atomic<long long> g_wait_us{kDefaultWaitUs};

// Allocation fault injector: when n > 0, the n-th scratch allocation from now fails with
// HD_ERR_NOMEM (then the injector disarms). Armed by hd_set_option(HD_OPT_FAIL_ALLOC, n) or,
// at the first allocation, by the environment variable HD_FAIL_ALLOC=n.
std::atomic<int> g_fail_alloc{-1};  // -1: not yet read from the environment
bool alloc_fault() {
    int n = g_fail_alloc.load();
    if (n < 0) {
        const char *v = getenv("HD_FAIL_ALLOC");
        const int env = v ? atoi(v) : 0;
        int expect = -1;
        g_fail_alloc.compare_exchange_strong(expect, env > 0 ? env : 0);
        n = g_fail_alloc.load();
    }
    while (n > 0) {
        if (g_fail_alloc.compare_exchange_weak(n, n - 1)) return n == 1;
    }
    return false;
}

// Library scratch allocations (device memory), all through the fault injector.
hipError_t scratch_malloc_async(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (alloc_fault()) return hipErrorOutOfMemory;
    return hipMallocAsync(p, bytes, s);
}
hipError_t scratch_malloc(void **p, size_t bytes) {
    *p = nullptr;
    if (alloc_fault()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

struct Strategy {
    int select_mode;   // hd::SelectMode
    int fuse;          // 1: Wiener partials fused into the AMF stage (ring recompute)
    int resident = 1;  // 1: one resident launch for the whole hybrid when it fits
    int tile_rows = hd::TILE_Y;  // AMF tile height of the staged stage without the ring: 16, 32, 64
};

struct TuneEntry {
    int eb, smax, wh, ww;
    Strategy best;
    double us;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
bool g_tune_loaded = false;

const char *tune_path() { return getenv("HD_AUTOTUNE_CACHE"); }

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *p = tune_path();
    if (!p) return;
    FILE *f = fopen(p, "r");
    if (!f) return;
    // one entry per line: {"eb":1,"smax":9,"wh":5,"ww":5,"select":0,"fuse":1,"rows":32,"us":12.5}
    // (lines without "rows" are read as 32-row tiles)
    char line[256];
    while (fgets(line, sizeof line, f)) {
        TuneEntry e{};
        if (sscanf(line, " {\"eb\":%d,\"smax\":%d,\"wh\":%d,\"ww\":%d,\"select\":%d,\"fuse\":%d,\"rows\":%d,\"us\":%lf}",
                   &e.eb, &e.smax, &e.wh, &e.ww, &e.best.select_mode, &e.best.fuse, &e.best.tile_rows,
                   &e.us) == 8 ||
            sscanf(line, " {\"eb\":%d,\"smax\":%d,\"wh\":%d,\"ww\":%d,\"select\":%d,\"fuse\":%d,\"us\":%lf}",
                   &e.eb, &e.smax, &e.wh, &e.ww, &e.best.select_mode, &e.best.fuse, &e.us) == 7) {
            if (e.best.tile_rows != hd::TILE_Y / 2 && e.best.tile_rows != 2 * hd::TILE_Y) e.best.tile_rows = hd::TILE_Y;
            g_tune.push_back(e);
        }
    }
    fclose(f);
}

void tune_save_locked() {
    const char *p = tune_path();
    if (!p) return;
    FILE *f = fopen(p, "w");
    if (!f) return;
    for (const auto &e : g_tune)
        fprintf(f, "{\"eb\":%d,\"smax\":%d,\"wh\":%d,\"ww\":%d,\"select\":%d,\"fuse\":%d,\"rows\":%d,\"us\":%.3f}\n",
                e.eb, e.smax, e.wh, e.ww, e.best.select_mode, e.best.fuse, e.best.tile_rows, e.us);
    fclose(f);
}

void tune_store(int eb, int smax, int wh, int ww, const Strategy &best, double us) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    bool found = false;
    for (auto &t : g_tune)
        if (t.eb == eb && t.smax == smax && t.wh == wh && t.ww == ww) {
            t.best = best;
            t.us = us;
            found = true;
        }
    if (!found) g_tune.push_back(TuneEntry{eb, smax, wh, ww, best, us});
    tune_save_locked();
}

// Tuned strategy for the key (eb, smax, window); the AMF-only call (window 0 x 0) takes the
// selection mode tuned for any window with the same element size and Smax.
Strategy strategy_for(int eb, int smax, int wh, int ww) {
    Strategy s{hd::SELECT_AUTO, 1};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        for (const auto &e : g_tune)
            if (e.eb == eb && e.smax == smax && ((e.wh == wh && e.ww == ww) || wh == 0)) s = e.best;
    }
    const int sm = g_select_mode.load(), fu = g_fuse.load(), rs = g_resident.load(), tr = g_tile_rows.load();
    if (sm >= 0) s.select_mode = sm;
    if (fu >= 0) s.fuse = fu;
    if (tr > 0) s.tile_rows = tr;
    s.resident = rs != 0;
    return s;
}

// Workgroups of the resident kernel the current device holds at once, cached per key.
int resident_capacity_cached(int eb, int smax, int wh, int ww, int select_mode) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const bool dense = select_mode == hd::SELECT_DENSE;
    const auto key = std::make_tuple(dev, eb, smax, wh, ww, dense ? 1 : 0);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int c = hd::resident_capacity(eb, smax, wh, ww, select_mode);
    cache[key] = c;
    return c;
}

// Dynamic LDS of the resident kernel for a tile count (even spread over the CUs), cached.
int resident_lds_cached(int eb, int smax, int wh, int ww, int select_mode, int tiles) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const auto key = std::make_tuple(dev, eb, smax, wh, ww, select_mode == hd::SELECT_DENSE ? 1 : 0, tiles);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int b = hd::resident_lds_bytes(eb, smax, wh, ww, select_mode, tiles);
    cache[key] = b;
    return b;
}

// Barrier words of the resident kernel: zero before the first launch, then reused as each
// launch leaves them.
struct ResidentSync {
    unsigned int *words = nullptr;
    bool fresh = false;  // zero them (on the stream) before the launch
};
size_t resident_sync_bytes() { return round256((size_t)hd::RESIDENT_SYNC_WORDS * 4); }
ResidentSync resident_sync_at(unsigned char *p, bool fresh) {
    ResidentSync r;
    r.words = (unsigned int *)p;
    r.fresh = fresh;
    return r;
}

// Events around each stage launch of one enqueue (hybrid_denoise_batched_timed).
struct StageTimer {
    hipEvent_t ev[2 * HD_STAGES] = {};
    bool used[HD_STAGES] = {};
    hipStream_t s = nullptr;
    hd_status begin(int i) {
        used[i] = true;
        const hipError_t e = hipEventRecord(ev[2 * i], s);
        return e == hipSuccess ? HD_OK : hip_fail(e, "stage event");
    }
    hd_status end(int i) {
        const hipError_t e = hipEventRecord(ev[2 * i + 1], s);
        return e == hipSuccess ? HD_OK : hip_fail(e, "stage event");
    }
};
#define HD_TIMED(timer, i, stmt)                                   \
    do {                                                           \
        if (timer) {                                               \
            const hd_status ts_ = (timer)->begin(i);               \
            if (ts_ != HD_OK) return ts_;                          \
        }                                                          \
        stmt;                                                      \
        if (timer) {                                               \
            const hd_status te_ = (timer)->end(i);                 \
            if (te_ != HD_OK) return te_;                          \
        }                                                          \
    } while (0)

// Enqueue the hybrid pipeline for `set` on stream s. Scratch: partials (one u64 per tile)
// and nu2 (one double per slice) must be provided when nu2 is estimated. With `timer`,
// events are recorded around every stage launch.
hd_status enqueue_hybrid(const hd::SliceSet &set, int total_tiles, int eb, int max_value, int smax,
                         int wh, int ww, double noise_var, int keep, bool aligned_in, bool aligned_a,
                         unsigned long long *partials, double *nu2, const Strategy &strat, hipStream_t s,
                         const ResidentSync *rsync = nullptr, bool store_amf = true, bool stretch = false,
                         unsigned long long *slice_ranges = nullptr, StageTimer *timer = nullptr) {
    hipError_t e;
    const bool estimate = noise_var < 0.0;
    if (estimate && strat.resident && rsync && rsync->words && !set.list && !set.flags &&
        set.n <= hd::RESIDENT_MAX_SLICES &&
        total_tiles <= resident_capacity_cached(eb, smax, wh, ww, strat.select_mode)) {
        if (rsync->fresh) {
            e = hd::launch_zero_u32(rsync->words, hd::RESIDENT_SYNC_WORDS, s);
            if (e != hipSuccess) return hip_fail(e, "sync clear launch");
        }
        HD_TIMED(timer, 0,
                 e = hd::launch_hybrid_resident(set, total_tiles, eb, smax, keep, wh, ww, max_value, partials,
                                                rsync->words, nu2, strat.select_mode, aligned_in && aligned_a,
                                                store_amf, stretch,
                                                resident_lds_cached(eb, smax, wh, ww, strat.select_mode,
                                                                    total_tiles),
                                                (unsigned long long)g_wait_us.load() * 100ull, s));
        if (e != hipSuccess) return hip_fail(e, "resident hybrid launch");
        return HD_OK;
    }
    const bool fused = estimate && strat.fuse;
    // other tile heights only for the plain AMF stage over whole slices
    const int rows = (fused || set.list) ? hd::TILE_Y : strat.tile_rows;
    HD_TIMED(timer, 0,
             e = hd::launch_amf_stage(set, total_tiles, eb, smax, keep, fused ? wh : 0, fused ? ww : 0,
                                      partials, strat.select_mode, aligned_in && aligned_a, s, rows));
    if (e != hipSuccess) return hip_fail(e, "amf stage launch");
    if (estimate) {
        if (!fused) {
            HD_TIMED(timer, 1,
                     e = hd::launch_wiener_stage(set, total_tiles, eb, max_value, wh, ww, false, nullptr, 0.0,
                                                 partials, aligned_a, s));
            if (e != hipSuccess) return hip_fail(e, "wiener partials launch");
        }
        HD_TIMED(timer, 2, e = hd::launch_noise_reduce(set, partials, wh, ww, nu2, s));
        if (e != hipSuccess) return hip_fail(e, "noise reduce launch");
    }
    HD_TIMED(timer, 3,
             e = hd::launch_wiener_stage(set, total_tiles, eb, max_value, wh, ww, true, estimate ? nu2 : nullptr,
                                         noise_var, nullptr, aligned_a, s, stretch ? partials : nullptr));
    if (e != hipSuccess) return hip_fail(e, "wiener apply launch");
    if (stretch) {
        HD_TIMED(timer, 4, e = hd::launch_stretch(set, total_tiles, partials, slice_ranges, s));
        if (e != hipSuccess) return hip_fail(e, "contrast stretch launch");
    }
    return HD_OK;
}

// ---- batched plans -------------------------------------------------------------------
struct Plan {
    std::vector<hd_slice> slices;
    int eb = 0, max_value = 0, smax = 0, wh = 0, ww = 0, keep = 0, stretch = 0, device = -1;
    double noise_var = 0;
    Strategy strat{};
    hd::SliceDesc *d_table = nullptr;
    unsigned char *d_scratch = nullptr;
    hd::SliceSet set{};
    int total_tiles = 0;
    bool aligned_in = true;
    unsigned long long *partials = nullptr;
    double *nu2 = nullptr;
    unsigned long long *ranges = nullptr;
    ResidentSync rsync{};
    bool single_kernel = false;  // plan_single_kernel(), decided once at build
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hd::SliceDesc> table_host;  // source of the table upload, kept with the plan
    hipEvent_t done = nullptr;              // recorded after every run outside a capture
    bool ran = false;
    ~Plan() {
        if (done) (void)hipEventDestroy(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (d_table) (void)hipFree(d_table);
        if (d_scratch) (void)hipFree(d_scratch);
    }
    bool same(const hd_slice *s, int n, int eb_, int mv, int sm, int h_, int w_, double nv, int kp,
              int str, int dev, const Strategy &st) const {
        if ((int)slices.size() != n || eb != eb_ || max_value != mv || smax != sm || wh != h_ ||
            ww != w_ || noise_var != nv || keep != kp || stretch != str || device != dev ||
            strat.select_mode != st.select_mode || strat.fuse != st.fuse || strat.resident != st.resident)
            return false;
        return memcmp(slices.data(), s, sizeof(hd_slice) * (size_t)n) == 0;
    }
};

std::mutex g_plan_mu;
std::vector<std::unique_ptr<Plan>> g_plans;
constexpr size_t kMaxPlans = 8;
// Evicted plans whose last run may still be on the device: freed once their event has
// completed (checked at every batched call), never by waiting for the device.
std::vector<std::unique_ptr<Plan>> g_retired;

bool plan_idle(const Plan &p) {
    if (!p.ran || !p.done) return true;
    const hipError_t e = hipEventQuery(p.done);
    if (e == hipErrorNotReady) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

void reap_retired_locked() {
    g_retired.erase(std::remove_if(g_retired.begin(), g_retired.end(),
                                   [](const std::unique_ptr<Plan> &p) { return plan_idle(*p); }),
                    g_retired.end());
}

hd_status build_plan(Plan &p, const hd_slice *sl, int n, hipStream_t stream) {
    std::vector<hd::SliceDesc> tab((size_t)n);
    long long tiles = 0;
    size_t a_bytes = 0;
    std::vector<size_t> a_off((size_t)n);
    for (int i = 0; i < n; ++i) {
        const int64_t ap = amf_pitch_of(sl[i].w, p.eb);
        a_off[(size_t)i] = a_bytes;
        a_bytes += round256((size_t)sl[i].h * (size_t)ap * (size_t)p.eb);
        tiles += tiles_of(sl[i].h, sl[i].w);
    }
    if (tiles > kMaxTiles) return fail(HD_ERR_DIMS, "batch too large (%lld tiles)", tiles);
    const size_t part_off = a_bytes;
    const size_t nu2_off = part_off + round256((size_t)tiles * 8);
    const size_t range_off = nu2_off + round256((size_t)n * 8);
    const size_t sync_off = range_off + round256((size_t)n * 8);
    const size_t total = sync_off + resident_sync_bytes();
    hipError_t e = scratch_malloc((void **)&p.d_scratch, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p.d_scratch = nullptr;
        return fail(HD_ERR_NOMEM, "batched scratch (%zu bytes): %s", total, hipGetErrorString(e));
    }
    int tb = 0;
    p.aligned_in = true;
    for (int i = 0; i < n; ++i) {
        hd::SliceDesc &d = tab[(size_t)i];
        d.in = sl[i].in;
        d.amf = p.d_scratch + a_off[(size_t)i];
        d.out = sl[i].out;
        d.in_pitch = sl[i].in_pitch;
        d.amf_pitch = amf_pitch_of(sl[i].w, p.eb);
        d.out_pitch = sl[i].out_pitch;
        d.h = sl[i].h;
        d.w = sl[i].w;
        d.tiles_x = tiles_x_of(sl[i].w);
        d.tile_begin = tb;
        tb += tiles_of(sl[i].h, sl[i].w);
        p.aligned_in = p.aligned_in && aligned16(sl[i].in, sl[i].in_pitch, p.eb);
    }
    p.total_tiles = tb;
    p.partials = (unsigned long long *)(p.d_scratch + part_off);
    p.nu2 = (double *)(p.d_scratch + nu2_off);
    p.ranges = (unsigned long long *)(p.d_scratch + range_off);
    // zeroed once here, ahead of the first run on the caller's stream (every resident
    // launch leaves them zero); when the caller's stream is being captured, each run
    // clears them with a kernel instead (no memset node in a captured graph)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (stream) (void)hipStreamIsCapturing(stream, &cs);
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing) {
        // stream-ordered before the plan's first run on this stream (a run on another
        // stream must be ordered after this call by the caller, as for any shared plan)
        e = hipMemsetAsync(p.d_scratch + sync_off, 0, resident_sync_bytes(), stream);
        if (e != hipSuccess) return hip_fail(e, "sync words clear");
    }
    p.rsync = resident_sync_at(p.d_scratch + sync_off, capturing);
    e = scratch_malloc((void **)&p.d_table, sizeof(hd::SliceDesc) * (size_t)n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p.d_table = nullptr;
        return fail(HD_ERR_NOMEM, "slice table: %s", hipGetErrorString(e));
    }
    p.table_host = tab;
    // in stream order, unless the caller is capturing the stream (the upload must not
    // become a node of the caller's graph)
    e = capturing ? hipMemcpy(p.d_table, p.table_host.data(), sizeof(hd::SliceDesc) * (size_t)n,
                              hipMemcpyHostToDevice)
                  : hipMemcpyAsync(p.d_table, p.table_host.data(), sizeof(hd::SliceDesc) * (size_t)n,
                                   hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "slice table upload");
    if (!capturing) {
        e = hipEventCreateWithFlags(&p.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            p.done = nullptr;
            return hip_fail(e, "plan event");
        }
    }
    p.set.one = tab[0];
    p.set.many = p.d_table;
    p.set.n = n;
    if (n == 1) p.set.many = nullptr;
    p.slices.assign(sl, sl + n);
    return HD_OK;
}

hd_status plan_enqueue(Plan &p, hipStream_t s) {
    // the batched call returns only the Wiener output: the resident path skips the AMF store
    return enqueue_hybrid(p.set, p.total_tiles, p.eb, p.max_value, p.smax, p.wh, p.ww, p.noise_var,
                          p.keep, p.aligned_in, true, p.partials, p.nu2, p.strat, s, &p.rsync, false,
                          p.stretch != 0, p.ranges);
}

// True when the plan's whole enqueue is the one resident kernel: a graph of one kernel
// only adds launch latency, so such plans launch it directly.
bool plan_single_kernel(const Plan &p) {
    return p.noise_var < 0.0 && p.strat.resident && p.set.n <= hd::RESIDENT_MAX_SLICES && !p.rsync.fresh &&
           p.total_tiles <= resident_capacity_cached(p.eb, p.smax, p.wh, p.ww, p.strat.select_mode);
}

hd_status plan_run_inner(Plan &p, hipStream_t s, bool capturing) {
    if (!g_use_graph.load() || capturing || p.single_kernel) return plan_enqueue(p, s);
    hipError_t e;
    if (!p.exec) {
        if (!p.cap) {
            e = hipStreamCreateWithFlags(&p.cap, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "capture stream");
        }
        e = hipStreamBeginCapture(p.cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        hd_status st = plan_enqueue(p, p.cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p.cap, &g);
        if (st != HD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        p.graph = g;
        e = hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            p.exec = nullptr;
            return hip_fail(e, "graph instantiate");
        }
    }
    e = hipGraphLaunch(p.exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return HD_OK;
}

hd_status plan_run(Plan &p, hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s) (void)hipStreamIsCapturing(s, &cs);
    const bool capturing = cs != hipStreamCaptureStatusNone;
    const hd_status st = plan_run_inner(p, s, capturing);
    if (st == HD_OK && !capturing && p.done) {
        const hipError_t e = hipEventRecord(p.done, s);
        if (e != hipSuccess) return hip_fail(e, "plan event record");
        p.ran = true;
    }
    return st;
}

}  // namespace

namespace {
hd_status find_plan(const hd_slice *slices, int n, int eb, int max_value, int smax, int win_h, int win_w,
                    double noise_var, int keep, int stretch, int dev, const Strategy &strat, hipStream_t stream,
                    Plan **out);
}  // namespace

namespace hd {
void set_error_message(const char *msg) { snprintf(g_last_error, sizeof g_last_error, "%s", msg); }
}  // namespace hd

extern "C" {

int32_t hd_version(void) { return 200; }

const char *hd_last_error(void) { return g_last_error; }

hd_status hd_check_errors(void *stream) {
    hipStream_t s = (hipStream_t)stream;
    unsigned int *dw = hd::device_error_word();
    if (!dw) return fail(HD_ERR_HIP, "error word lookup failed");
    unsigned int v = 0;
    hipError_t e = hipMemcpyAsync(&v, dw, sizeof v, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "error word read");
    if (v == 0) return ok();
    if ((e = hd::launch_zero_u32(dw, 1, s)) != hipSuccess) return hip_fail(e, "error word clear");
    return fail(HD_ERR_TIMEOUT,
                "a wait of the single-launch exchange gave up (flags 0x%x): its workgroups wrote NaN; the "
                "grid was probably not co-resident (other work on the device)", v);
}

hd_status hd_set_option(int32_t key, int32_t value) {
    switch (key) {
        case HD_OPT_SELECT:
            if (value < -1 || value > 3) return fail(HD_ERR_ARG, "select mode %d", value);
            g_select_mode.store(value);
            return ok();
        case HD_OPT_FUSE_MOMENTS:
            if (value < -1 || value > 1) return fail(HD_ERR_ARG, "fuse value %d", value);
            g_fuse.store(value);
            return ok();
        case HD_OPT_GRAPHS:
            if (value < 0 || value > 1) return fail(HD_ERR_ARG, "graph value %d", value);
            g_use_graph.store(value);
            return ok();
        case HD_OPT_RESIDENT:
            if (value < -1 || value > 1) return fail(HD_ERR_ARG, "resident value %d", value);
            g_resident.store(value);
            return ok();
        case HD_OPT_WAIT_LIMIT_US:
            if (value < -1) return fail(HD_ERR_ARG, "wait limit %d us", value);
            g_wait_us.store(value < 0 ? kDefaultWaitUs : (long long)value);
            return ok();
        case HD_OPT_TILE_ROWS:
            if (value != -1 && value != hd::TILE_Y / 2 && value != hd::TILE_Y && value != 2 * hd::TILE_Y)
                return fail(HD_ERR_ARG, "tile rows %d (16, 32, 64 or -1)", value);
            g_tile_rows.store(value);
            return ok();
        case HD_OPT_SURROGATE_FUSED:
            if (value < 0 || value > 1) return fail(HD_ERR_ARG, "surrogate fusion value %d", value);
            g_sg_fused.store(value);
            return ok();
        case HD_OPT_FAIL_ALLOC:
            if (value < 0) return fail(HD_ERR_ARG, "allocation fault count %d", value);
            g_fail_alloc.store(value);
            return ok();
        default:
            return fail(HD_ERR_ARG, "unknown option %d", key);
    }
}

int32_t hd_resident_capacity(int32_t dt, int32_t smax, int32_t win_h, int32_t win_w,
                             int32_t select_mode) {
    const int eb = dtype_bytes(dt);
    if (!eb || smax < 3 || smax > HD_SMAX_LIMIT || (smax & 1) == 0 || win_h < 1 || win_w < 1 ||
        win_h > HD_WIN_LIMIT || win_w > HD_WIN_LIMIT || (win_h & 1) == 0 || (win_w & 1) == 0 ||
        select_mode < -1 || select_mode > 3)
        return 0;
    const int sel = select_mode >= 0 ? select_mode : strategy_for(eb, smax, win_h, win_w).select_mode;
    const int cap = resident_capacity_cached(eb, smax, win_h, win_w, sel);
    // group sizes up to a workgroup; one release word per workgroup
    const int lim = std::min(hd::RESIDENT_MAX_GROUPS * hd::STAGE_THREADS, hd::RESIDENT_MAX_BLOCKS);
    return cap < lim ? cap : lim;
}

hd_status amf_filter(const void *in, void *out, int32_t h, int32_t w, int64_t in_pitch,
                     int64_t out_pitch, int32_t dt, int32_t smax, uint32_t flags,
                     void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_smax(smax)) != HD_OK) return st;
    if (flags & ~HD_AMF_UNRESOLVED_KEEP) return fail(HD_ERR_ARG, "unknown flags 0x%x", flags);
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, eb)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    hd::SliceSet set{};
    set.one = hd::SliceDesc{in, out, nullptr, in_pitch, out_pitch, 0, h, w, tiles_x_of(w), 0};
    set.n = 1;
    const Strategy strat = strategy_for(eb, smax, 0, 0);
    hipError_t e = hd::launch_amf_stage(set, tiles_of(h, w), eb, smax,
                                        (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0, 0, 0, nullptr,
                                        strat.select_mode,
                                        aligned16(in, in_pitch, eb) && aligned16(out, out_pitch, eb),
                                        (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "amf launch");
    return ok();
}

hd_status degrade_image(const void *clean, void *noisy, int32_t h, int32_t w, int64_t clean_pitch,
                        int64_t noisy_pitch, int32_t dt, int32_t max_value, double sigma,
                        double density, uint64_t seed, uint32_t stream_id, void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(clean, h, w, clean_pitch, "clean")) != HD_OK) return st;
    if ((st = check_image(noisy, h, w, noisy_pitch, "noisy")) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (!(sigma >= 0.0) || !(sigma < 1e9)) return fail(HD_ERR_ARG, "sigma %g", sigma);
    if (!(density >= 0.0) || !(density <= 1.0)) return fail(HD_ERR_ARG, "density %g", density);
    if (clean != noisy && overlaps(clean, span_bytes(h, w, clean_pitch, eb), noisy,
                                   span_bytes(h, w, noisy_pitch, eb)))
        return fail(HD_ERR_ALIAS, "clean and noisy overlap (only exact in-place is allowed)");
    if (clean == noisy && clean_pitch != noisy_pitch)
        return fail(HD_ERR_ALIAS, "in-place degradation needs equal pitches");
    const hipError_t e = hd::launch_degrade(clean, noisy, h, w, clean_pitch, noisy_pitch, eb, max_value,
                                            sigma, density, (unsigned long long)seed, stream_id,
                                            (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "degrade launch");
    return ok();
}

hd_status wiener_fft(const void *in, const void *original, float *out, int32_t h, int32_t w, int64_t in_pitch,
                     int64_t orig_pitch, int64_t out_pitch, int32_t dt, int32_t max_value, void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(original, h, w, orig_pitch, "original")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (!hd::fft_size_ok(h) || !hd::fft_size_ok(w))
        return fail(HD_ERR_DIMS, "%d x %d: each side must be <= %d with prime factors 2, 3, 5 only", h, w,
                    hd::FFT_MAX_LEN);
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, 4)) ||
        overlaps(original, span_bytes(h, w, orig_pitch, eb), out, span_bytes(h, w, out_pitch, 4)))
        return fail(HD_ERR_ALIAS, "the output overlaps an input");
    hipStream_t s = (hipStream_t)stream;
    void *scr = nullptr;
    hipError_t e = scratch_malloc_async(&scr, hd::wiener_fft_scratch_bytes(h, w), s);
    if (e != hipSuccess || !scr) {
        (void)hipGetLastError();
        return fail(HD_ERR_NOMEM, "scratch allocation failed: %s", hipGetErrorString(e));
    }
    st = HD_OK;
    if ((e = hd::launch_wiener_fft(in, in_pitch, original, orig_pitch, out, out_pitch, h, w, eb, max_value, scr,
                                   s)) != hipSuccess)
        st = hip_fail(e, "frequency-domain wiener launch");
    hipError_t ef = hipFreeAsync(scr, s);
    if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "scratch free");
    return st == HD_OK ? ok() : st;
}

hd_status contrast_stretch(float *img, int32_t h, int32_t w, int64_t pitch, void *stream) {
    hd_status st;
    if ((st = check_image(img, h, w, pitch, "img")) != HD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int nt = tiles_of(h, w);
    unsigned char *scr = nullptr;
    hipError_t e = scratch_malloc_async((void **)&scr, round256((size_t)nt * 8) + 256, s);
    if (e != hipSuccess || !scr) {
        (void)hipGetLastError();
        return fail(HD_ERR_NOMEM, "scratch allocation failed: %s", hipGetErrorString(e));
    }
    hd::SliceSet set{};
    set.one = hd::SliceDesc{nullptr, nullptr, img, 0, 0, pitch, h, w, tiles_x_of(w), 0};
    set.n = 1;
    unsigned long long *tr = (unsigned long long *)scr;
    unsigned long long *sr = (unsigned long long *)(scr + round256((size_t)nt * 8));
    st = HD_OK;
    if ((e = hd::launch_tile_ranges(set, nt, tr, s)) != hipSuccess) st = hip_fail(e, "range launch");
    if (st == HD_OK && (e = hd::launch_stretch(set, nt, tr, sr, s)) != hipSuccess)
        st = hip_fail(e, "contrast stretch launch");
    hipError_t ef = hipFreeAsync(scr, s);
    if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "scratch free");
    return st == HD_OK ? ok() : st;
}

hd_status amf_filter_parts(const void *in, void *out, int32_t h, int32_t w, int64_t in_pitch,
                           int64_t out_pitch, int32_t dt, int32_t smax, int32_t parts, uint32_t flags,
                           void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_smax(smax)) != HD_OK) return st;
    if (parts < 1 || parts > HD_PARTS_LIMIT || parts > h)
        return fail(HD_ERR_ARG, "parts %d: need 1 <= parts <= min(h, %d)", parts, HD_PARTS_LIMIT);
    if (flags & ~HD_AMF_UNRESOLVED_KEEP) return fail(HD_ERR_ARG, "unknown flags 0x%x", flags);
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, eb)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    if (parts == 1) return amf_filter(in, out, h, w, in_pitch, out_pitch, dt, smax, flags, stream);
    hipStream_t s = (hipStream_t)stream;
    long long tiles = 0;
    for (int i = 0; i < parts; ++i) {
        const int r0 = (int)((long long)i * h / parts), r1 = (int)((long long)(i + 1) * h / parts);
        tiles += tiles_of(r1 - r0, w);
    }
    hd::SliceDesc *table = nullptr;
    hipError_t e = scratch_malloc_async((void **)&table, sizeof(hd::SliceDesc) * (size_t)parts, s);
    if (e != hipSuccess || !table) {
        (void)hipGetLastError();
        return fail(HD_ERR_NOMEM, "strip table: %s", hipGetErrorString(e));
    }
    st = HD_OK;
    if ((e = hd::launch_strip_table(table, in, out, h, w, in_pitch, out_pitch, eb, parts, s)) != hipSuccess)
        st = hip_fail(e, "strip table launch");
    if (st == HD_OK) {
        hd::SliceSet set{};
        set.many = table;
        set.n = parts;
        const Strategy strat = strategy_for(eb, smax, 0, 0);
        e = hd::launch_amf_stage(set, (int)tiles, eb, smax, (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0, 0, 0,
                                 nullptr, strat.select_mode,
                                 aligned16(in, in_pitch, eb) && aligned16(out, out_pitch, eb), s);
        if (e != hipSuccess) st = hip_fail(e, "amf launch");
    }
    hipError_t ef = hipFreeAsync(table, s);
    if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "strip table free");
    return st == HD_OK ? ok() : st;
}

hd_status wiener_filter(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                        int64_t out_pitch, int32_t dt, int32_t max_value, int32_t win_h,
                        int32_t win_w, double noise_var, double *nu2_out, void *stream) {
    hd_status st;
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_window(win_h, win_w)) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, 4)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    hipStream_t s = (hipStream_t)stream;
    hd::SliceSet set{};
    set.one = hd::SliceDesc{in, const_cast<void *>(in), out, in_pitch, in_pitch, out_pitch, h, w,
                            tiles_x_of(w), 0};
    set.n = 1;
    const int nt = tiles_of(h, w);
    const bool al = aligned16(in, in_pitch, eb);
    hipError_t e;
    if (noise_var >= 0.0) {
        e = hd::launch_wiener_stage(set, nt, eb, max_value, win_h, win_w, true, nullptr, noise_var,
                                    nullptr, al, s);
        if (e != hipSuccess) return hip_fail(e, "wiener apply launch");
        if (nu2_out && (e = hd::launch_fill_f64(nu2_out, noise_var, s)) != hipSuccess)
            return hip_fail(e, "nu2 fill launch");
        return ok();
    }
    unsigned char *scr = nullptr;
    const size_t nu2_off = round256((size_t)nt * 8);
    e = scratch_malloc_async((void **)&scr, nu2_off + 256, s);
    if (e != hipSuccess || !scr) {
        (void)hipGetLastError();
        return fail(HD_ERR_NOMEM, "scratch allocation failed: %s", hipGetErrorString(e));
    }
    unsigned long long *partials = (unsigned long long *)scr;
    double *nu2 = nu2_out ? nu2_out : (double *)(scr + nu2_off);
    st = HD_OK;
    if ((e = hd::launch_wiener_stage(set, nt, eb, max_value, win_h, win_w, false, nullptr, 0.0,
                                     partials, al, s)) != hipSuccess)
        st = hip_fail(e, "wiener partials launch");
    if (st == HD_OK && (e = hd::launch_noise_reduce(set, partials, win_h, win_w, nu2, s)) != hipSuccess)
        st = hip_fail(e, "noise reduce launch");
    if (st == HD_OK && (e = hd::launch_wiener_stage(set, nt, eb, max_value, win_h, win_w, true, nu2,
                                                    -1.0, nullptr, al, s)) != hipSuccess)
        st = hip_fail(e, "wiener apply launch");
    hipError_t ef = hipFreeAsync(scr, s);
    if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "scratch free");
    return st == HD_OK ? ok() : st;
}

static hd_status hybrid_checks(const void *in, const float *out, int32_t h, int32_t w,
                               int64_t in_pitch, int64_t out_pitch, int32_t dt, int32_t max_value,
                               int32_t smax, int32_t win_h, int32_t win_w, uint32_t flags) {
    hd_status st;
    if (!dtype_bytes(dt)) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    const int eb = dtype_bytes(dt);
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_image(out, h, w, out_pitch, "out")) != HD_OK) return st;
    if ((st = check_smax(smax)) != HD_OK) return st;
    if ((st = check_window(win_h, win_w)) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (flags & ~(HD_AMF_UNRESOLVED_KEEP | HD_CONTRAST_STRETCH))
        return fail(HD_ERR_ARG, "unknown flags 0x%x", flags);
    if (overlaps(in, span_bytes(h, w, in_pitch, eb), out, span_bytes(h, w, out_pitch, 4)))
        return fail(HD_ERR_ALIAS, "input and output overlap");
    return HD_OK;
}

}  // extern "C"

namespace {

// Scratch of hybrid_denoise_noalloc: a file-scope device array, one per device, held until
// the process ends. Host code never uses the array's name as an address: each device's
// address comes from hipGetSymbolAddress, looked up once with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)HD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

unsigned char *noalloc_scratch() {
    constexpr int kMaxDevices = 64;
    static std::atomic<unsigned char *> addr[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    unsigned char *p = addr[dev].load();
    if (!p) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) {
            (void)hipGetLastError();
            return nullptr;
        }
        p = (unsigned char *)q;
        addr[dev].store(p);
    }
    return p;
}

// hybrid_denoise, with its scratch either allocated in stream order (noalloc false) or
// taken from the device's static scratch array (noalloc true: no allocation at all).
hd_status hybrid_impl(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch, int64_t out_pitch,
                      int32_t dt, int32_t max_value, int32_t smax, int32_t win_h, int32_t win_w,
                      double noise_var, uint32_t flags, void *amf_out, int64_t amf_pitch, double *nu2_out,
                      void *stream, bool noalloc) {
    hd_status st = hybrid_checks(in, out, h, w, in_pitch, out_pitch, dt, max_value, smax, win_h,
                                 win_w, flags);
    if (st != HD_OK) return st;
    const int eb = dtype_bytes(dt);
    const size_t in_span = span_bytes(h, w, in_pitch, eb);
    if (amf_out) {
        if ((st = check_image(amf_out, h, w, amf_pitch, "amf_out")) != HD_OK) return st;
        const size_t a_span = span_bytes(h, w, amf_pitch, eb);
        if (overlaps(in, in_span, amf_out, a_span) ||
            overlaps(out, span_bytes(h, w, out_pitch, 4), amf_out, a_span))
            return fail(HD_ERR_ALIAS, "amf_out overlaps the input or the output");
    }
    hipStream_t s = (hipStream_t)stream;
    const int nt = tiles_of(h, w);
    const bool estimate = noise_var < 0.0;
    // scratch: [a (when amf_out is NULL)][partials][nu2]
    const int64_t ap = amf_out ? amf_pitch : amf_pitch_of(w, eb);
    const size_t a_bytes = amf_out ? 0 : round256((size_t)h * (size_t)ap * (size_t)eb);
    const bool stretch = (flags & HD_CONTRAST_STRETCH) != 0;
    // scratch: [a (when amf_out is NULL)][partials / tile ranges][nu2][slice range][sync]
    const size_t p_bytes = (estimate || stretch) ? round256((size_t)nt * 8) : 0;
    const size_t n_bytes = (estimate && !nu2_out) ? 256 : 0;
    const size_t r_bytes = stretch ? 256 : 0;
    const size_t y_bytes = estimate ? resident_sync_bytes() : 0;
    unsigned char *scr = nullptr;
    hipError_t e;
    const size_t need = a_bytes + p_bytes + n_bytes + r_bytes + y_bytes;
    if (noalloc) {
        if (need > kNoAllocScratchBytes)
            return fail(HD_ERR_DIMS,
                        "%d x %d needs %zu bytes of scratch; the no-allocation entry point holds %zu "
                        "(HD_NOALLOC_SCRATCH_BYTES)",
                        h, w, need, kNoAllocScratchBytes);
        if (need && !(scr = noalloc_scratch())) return fail(HD_ERR_HIP, "scratch symbol lookup failed");
    } else if (need) {
        e = scratch_malloc_async((void **)&scr, need, s);
        if (e != hipSuccess || !scr) {
            (void)hipGetLastError();
            return fail(HD_ERR_NOMEM, "scratch allocation failed: %s", hipGetErrorString(e));
        }
    }
    void *a = amf_out ? amf_out : (void *)scr;
    unsigned long long *partials = (estimate || stretch) ? (unsigned long long *)(scr + a_bytes) : nullptr;
    unsigned long long *srange = stretch ? (unsigned long long *)(scr + a_bytes + p_bytes + n_bytes) : nullptr;
    double *nu2 = estimate ? (nu2_out ? nu2_out : (double *)(scr + a_bytes + p_bytes)) : nullptr;
    hd::SliceSet set{};
    set.one = hd::SliceDesc{in, a, out, in_pitch, ap, out_pitch, h, w, tiles_x_of(w), 0};
    set.n = 1;
    const Strategy strat = strategy_for(eb, smax, win_h, win_w);
    const ResidentSync rs =
        estimate ? resident_sync_at(scr + a_bytes + p_bytes + n_bytes + r_bytes, true) : ResidentSync{};
    st = enqueue_hybrid(set, nt, eb, max_value, smax, win_h, win_w, noise_var,
                        (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0, aligned16(in, in_pitch, eb),
                        aligned16(a, ap, eb), partials, nu2, strat, s, &rs, amf_out != nullptr, stretch,
                        srange);
    if (st == HD_OK && !estimate && nu2_out && (e = hd::launch_fill_f64(nu2_out, noise_var, s)) != hipSuccess)
        st = hip_fail(e, "nu2 fill launch");
    if (scr && !noalloc) {
        hipError_t ef = hipFreeAsync(scr, s);
        if (st == HD_OK && ef != hipSuccess) st = hip_fail(ef, "scratch free");
    }
    return st == HD_OK ? ok() : st;
}

}  // namespace

extern "C" {

hd_status hybrid_denoise(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                         int64_t out_pitch, int32_t dt, int32_t max_value, int32_t smax,
                         int32_t win_h, int32_t win_w, double noise_var, uint32_t flags,
                         void *amf_out, int64_t amf_pitch, double *nu2_out, void *stream) {
    return hybrid_impl(in, out, h, w, in_pitch, out_pitch, dt, max_value, smax, win_h, win_w, noise_var, flags,
                       amf_out, amf_pitch, nu2_out, stream, false);
}

hd_status hybrid_denoise_noalloc(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                                 int64_t out_pitch, int32_t dt, int32_t max_value, int32_t smax,
                                 int32_t win_h, int32_t win_w, double noise_var, uint32_t flags,
                                 void *amf_out, int64_t amf_pitch, double *nu2_out, void *stream) {
    return hybrid_impl(in, out, h, w, in_pitch, out_pitch, dt, max_value, smax, win_h, win_w, noise_var, flags,
                       amf_out, amf_pitch, nu2_out, stream, true);
}

static hd_status batched_checks(const hd_slice *slices, int32_t n, int32_t dt, int32_t max_value,
                                int32_t smax, int32_t win_h, int32_t win_w, uint32_t flags) {
    if (!slices) return fail(HD_ERR_NULL, "slices is NULL");
    if (n < 1) return fail(HD_ERR_ARG, "slice count %d < 1", n);
    if (!dtype_bytes(dt)) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    for (int i = 0; i < n; ++i) {
        hd_status st = hybrid_checks(slices[i].in, slices[i].out, slices[i].h, slices[i].w,
                                     slices[i].in_pitch, slices[i].out_pitch, dt, max_value, smax,
                                     win_h, win_w, flags);
        if (st != HD_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "slice %d: %s", i, g_last_error);
            return fail(st, "%s", msg);
        }
    }
    return HD_OK;
}

hd_status hybrid_denoise_batched(const hd_slice *slices, int32_t n, int32_t dt, int32_t max_value,
                                 int32_t smax, int32_t win_h, int32_t win_w, double noise_var,
                                 uint32_t flags, void *stream) {
    hd_status st0 = batched_checks(slices, n, dt, max_value, smax, win_h, win_w, flags);
    if (st0 != HD_OK) return st0;
    const int eb = dtype_bytes(dt);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "get device");
    const int keep = (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0;
    const int stretch = (flags & HD_CONTRAST_STRETCH) ? 1 : 0;
    const Strategy strat = strategy_for(eb, smax, win_h, win_w);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    Plan *p = nullptr;
    hd_status st = find_plan(slices, n, eb, max_value, smax, win_h, win_w, noise_var, keep, stretch, dev, strat,
                             (hipStream_t)stream, &p);
    if (st != HD_OK) return st;
    st = plan_run(*p, (hipStream_t)stream);
    return st == HD_OK ? ok() : st;
}

hd_status hybrid_denoise_batched_timed(const hd_slice *slices, int32_t n, int32_t dt, int32_t max_value,
                                       int32_t smax, int32_t win_h, int32_t win_w, double noise_var,
                                       uint32_t flags, float *stage_ms, void *stream) {
    if (!stage_ms) return fail(HD_ERR_NULL, "stage_ms is NULL");
    hd_status st = batched_checks(slices, n, dt, max_value, smax, win_h, win_w, flags);
    if (st != HD_OK) return st;
    const int eb = dtype_bytes(dt);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "get device");
    const int keep = (flags & HD_AMF_UNRESOLVED_KEEP) ? 1 : 0;
    const int stretch = (flags & HD_CONTRAST_STRETCH) ? 1 : 0;
    const Strategy strat = strategy_for(eb, smax, win_h, win_w);
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s) (void)hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone) return fail(HD_ERR_ARG, "the timed call cannot be captured");
    std::lock_guard<std::mutex> lk(g_plan_mu);
    Plan *p = nullptr;
    st = find_plan(slices, n, eb, max_value, smax, win_h, win_w, noise_var, keep, stretch, dev, strat, s, &p);
    if (st != HD_OK) return st;
    StageTimer t;
    t.s = s;
    for (auto &ev : t.ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) {
            st = hip_fail(e, "stage event create");
            break;
        }
    if (st == HD_OK)
        st = enqueue_hybrid(p->set, p->total_tiles, p->eb, p->max_value, p->smax, p->wh, p->ww, p->noise_var,
                            p->keep, p->aligned_in, true, p->partials, p->nu2, p->strat, s, &p->rsync, false,
                            p->stretch != 0, p->ranges, &t);
    if (st == HD_OK && p->done && (e = hipEventRecord(p->done, s)) == hipSuccess) p->ran = true;
    for (int i = 0; i < HD_STAGES; ++i) {
        stage_ms[i] = 0.0f;
        if (st == HD_OK && t.used[i]) {
            if ((e = hipEventSynchronize(t.ev[2 * i + 1])) != hipSuccess ||
                (e = hipEventElapsedTime(&stage_ms[i], t.ev[2 * i], t.ev[2 * i + 1])) != hipSuccess)
                st = hip_fail(e, "stage timing");
        }
    }
    for (auto &ev : t.ev)
        if (ev) (void)hipEventDestroy(ev);
    return st == HD_OK ? ok() : st;
}

}  // extern "C"

namespace {
hd_status find_plan(const hd_slice *slices, int n, int eb, int max_value, int smax, int win_h, int win_w,
                    double noise_var, int keep, int stretch, int dev, const Strategy &strat, hipStream_t stream,
                    Plan **out) {
    Plan *p = nullptr;
    for (auto &q : g_plans)
        if (q->same(slices, n, eb, max_value, smax, win_h, win_w, noise_var, keep, stretch, dev, strat))
            p = q.get();
    reap_retired_locked();
    if (!p) {
        if (g_plans.size() >= kMaxPlans) {
            // the evicted plan's last run may still be in flight: retire it until its
            // event has completed
            g_retired.push_back(std::move(g_plans.front()));
            g_plans.erase(g_plans.begin());
            reap_retired_locked();
        }
        auto np = std::make_unique<Plan>();
        np->eb = eb;
        np->max_value = max_value;
        np->smax = smax;
        np->wh = win_h;
        np->ww = win_w;
        np->noise_var = noise_var;
        np->keep = keep;
        np->stretch = stretch;
        np->device = dev;
        np->strat = strat;
        hd_status st = build_plan(*np, slices, n, stream);
        if (st != HD_OK) return st;
        np->single_kernel = plan_single_kernel(*np);
        g_plans.push_back(std::move(np));
        p = g_plans.back().get();
    }
    *out = p;
    return HD_OK;
}
}  // namespace

extern "C" {

void hd_release_plans(void) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    // waits for each plan's own last run (its event), not for the device
    for (auto *v : {&g_plans, &g_retired})
        for (auto &p : *v)
            if (p->ran && p->done) (void)hipEventSynchronize(p->done);
    g_plans.clear();
    g_retired.clear();
}

hd_status hd_autotune_hybrid(const void *in, int32_t h, int32_t w, int64_t in_pitch, int32_t dt,
                             int32_t max_value, int32_t smax, int32_t win_h, int32_t win_w,
                             int32_t iters, int32_t *best_select, int32_t *best_fuse,
                             int32_t *best_tile_rows, void *stream) {
    const int eb = dtype_bytes(dt);
    if (!eb) return fail(HD_ERR_DTYPE, "unknown dtype %d", (int)dt);
    hd_status st;
    if ((st = check_image(in, h, w, in_pitch, "in")) != HD_OK) return st;
    if ((st = check_smax(smax)) != HD_OK) return st;
    if ((st = check_window(win_h, win_w)) != HD_OK) return st;
    if ((st = check_maxval(max_value, dt)) != HD_OK) return st;
    if (iters < 1) return fail(HD_ERR_ARG, "iters %d < 1", iters);
    hipStream_t s = (hipStream_t)stream;
    const int nt = tiles_of(h, w);
    const int64_t ap = amf_pitch_of(w, eb);
    const size_t a_bytes = round256((size_t)h * (size_t)ap * (size_t)eb);
    const size_t o_bytes = round256((size_t)h * (size_t)w * 4);
    const size_t p_bytes = round256((size_t)nt * 8);
    unsigned char *scr = nullptr;
    hipError_t e = scratch_malloc((void **)&scr, a_bytes + o_bytes + p_bytes + 256 + resident_sync_bytes());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HD_ERR_NOMEM, "autotune scratch: %s", hipGetErrorString(e));
    }
    hd::SliceSet set{};
    set.one = hd::SliceDesc{in, scr, (float *)(scr + a_bytes), in_pitch, ap, w, h, w, tiles_x_of(w), 0};
    set.n = 1;
    unsigned long long *partials = (unsigned long long *)(scr + a_bytes + o_bytes);
    double *nu2 = (double *)(scr + a_bytes + o_bytes + p_bytes);
    const ResidentSync rs = resident_sync_at(scr + a_bytes + o_bytes + p_bytes + 256, false);
    if ((e = hipMemsetAsync(rs.words, 0, resident_sync_bytes(), s)) != hipSuccess) {
        (void)hipFree(scr);
        return hip_fail(e, "autotune sync clear");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    Strategy best{hd::SELECT_AUTO, 1};
    double best_us = 1e30;
    const Strategy cands[] = {{hd::SELECT_AUTO, 1},  {hd::SELECT_AUTO, 0},   {hd::SELECT_DENSE, 1},
                              {hd::SELECT_DENSE, 0}, {hd::SELECT_WAVE, 1},   {hd::SELECT_WAVE, 0},
                              {hd::SELECT_BISECT, 1}, {hd::SELECT_BISECT, 0},
                              {hd::SELECT_AUTO, 0, 1, hd::TILE_Y / 2},  {hd::SELECT_AUTO, 0, 1, 2 * hd::TILE_Y},
                              {hd::SELECT_DENSE, 0, 1, hd::TILE_Y / 2}, {hd::SELECT_DENSE, 0, 1, 2 * hd::TILE_Y}};
    st = HD_OK;
    for (const Strategy &c : cands) {
        // the tile height only matters for the staged AMF stage: not timed for an image
        // that runs as one resident launch
        if (c.tile_rows != hd::TILE_Y && c.resident && nt <= resident_capacity_cached(eb, smax, win_h, win_w, c.select_mode))
            continue;
        // warm-up, then timed repetitions
        st = enqueue_hybrid(set, nt, eb, max_value, smax, win_h, win_w, -1.0, 0,
                            aligned16(in, in_pitch, eb), true, partials, nu2, c, s, &rs, false);
        if (st != HD_OK) break;
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < iters && st == HD_OK; ++i)
            st = enqueue_hybrid(set, nt, eb, max_value, smax, win_h, win_w, -1.0, 0,
                                aligned16(in, in_pitch, eb), true, partials, nu2, c, s, &rs, false);
        (void)hipEventRecord(e1, s);
        if (st != HD_OK) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            st = hip_fail(e, "autotune sync");
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double us = 1000.0 * ms / iters;
        if (us < best_us) {
            best_us = us;
            best = c;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scr);
    if (st != HD_OK) return st;
    tune_store(eb, smax, win_h, win_w, best, best_us);
    if (best_select) *best_select = best.select_mode;
    if (best_fuse) *best_fuse = best.fuse;
    if (best_tile_rows) *best_tile_rows = best.tile_rows;
    return ok();
}

hd_status hd_autotune_batched(const hd_slice *slices, int32_t n, int32_t dt, int32_t max_value, int32_t smax,
                              int32_t win_h, int32_t win_w, int32_t iters, int32_t *best_select,
                              int32_t *best_fuse, int32_t *best_tile_rows, void *stream) {
    hd_status st = batched_checks(slices, n, dt, max_value, smax, win_h, win_w, 0);
    if (st != HD_OK) return st;
    if (iters < 1) return fail(HD_ERR_ARG, "iters %d < 1", iters);
    const int eb = dtype_bytes(dt);
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s) (void)hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone) return fail(HD_ERR_ARG, "the autotuner cannot be captured");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "get device");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "autotune events");
    }
    const Strategy cands[] = {{hd::SELECT_AUTO, 1},  {hd::SELECT_AUTO, 0},   {hd::SELECT_DENSE, 1},
                              {hd::SELECT_DENSE, 0}, {hd::SELECT_WAVE, 1},   {hd::SELECT_WAVE, 0},
                              {hd::SELECT_BISECT, 1}, {hd::SELECT_BISECT, 0},
                              {hd::SELECT_AUTO, 0, 1, hd::TILE_Y / 2},  {hd::SELECT_AUTO, 0, 1, 2 * hd::TILE_Y},
                              {hd::SELECT_DENSE, 0, 1, hd::TILE_Y / 2}, {hd::SELECT_DENSE, 0, 1, 2 * hd::TILE_Y}};
    Strategy best{hd::SELECT_AUTO, 1};
    double best_us = 1e30;
    for (const Strategy &c0 : cands) {
        // one temporary plan per candidate, run as the batched call runs it (graph replay,
        // or the single resident launch), on the caller's slices and outputs
        Strategy c = c0;
        c.resident = g_resident.load() != 0;
        Plan p;
        p.eb = eb;
        p.max_value = max_value;
        p.smax = smax;
        p.wh = win_h;
        p.ww = win_w;
        p.noise_var = -1.0;
        p.device = dev;
        p.strat = c;
        if ((st = build_plan(p, slices, n, s)) != HD_OK) break;
        p.single_kernel = plan_single_kernel(p);
        // the tile height only matters for the staged AMF stage: not timed for a single launch
        if (p.single_kernel && c.tile_rows != hd::TILE_Y) continue;
        if ((st = plan_run(p, s)) != HD_OK) break;  // warm-up (and graph capture)
        if ((e = hipEventRecord(e0, s)) != hipSuccess) {
            st = hip_fail(e, "autotune event");
            break;
        }
        for (int i = 0; i < iters && st == HD_OK; ++i) st = plan_run(p, s);
        if (st != HD_OK) break;
        float ms = 0.0f;
        if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
            st = hip_fail(e, "autotune timing");
            break;
        }
        const double us = 1000.0 * ms / iters;
        if (us < best_us) {
            best_us = us;
            best = c0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HD_OK) return st;
    tune_store(eb, smax, win_h, win_w, best, best_us);
    if (best_select) *best_select = best.select_mode;
    if (best_fuse) *best_fuse = best.fuse;
    if (best_tile_rows) *best_tile_rows = best.tile_rows;
    return ok();
}

}  // extern "C"

namespace hd {
bool surrogate_fused_inference() { return g_sg_fused.load() != 0; }
}  // namespace hd

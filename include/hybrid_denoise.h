/*
 * hybrid_denoise.h -- C ABI of the MI355X (gfx950) hybrid de-noiser.
 *
 * The method (Youssef, Mahmoud, El-Horbaty, "A Parallel Hybrid Technique for
 * Multi-Noise Removal from Grayscale Medical Images", arXiv 2005.05371):
 *   1. adaptive median filter (AMF): for each pixel try windows k = 3, 5, ..., Smax;
 *      at the first k where zmin < zmed < zmax (stage A) the pixel is resolved: it keeps
 *      its value g when zmin < g < zmax (stage B), else takes zmed (Alg. 1, procedure
 *      parallelAdapMedian, level loop and output masks);
 *   2. Wiener filter applied to the AMF output (Sec. IV, Fig. 4; Alg. 1, procedure
 *      parallelHybrid). This library uses the local mean / variance adaptive form:
 *      out = mu + (a - mu) * max(s2 - nu2, 0) / max(s2, nu2), out = mu when both are 0,
 *      mu / s2 = mean / population variance of the AMF output a over a win_h x win_w
 *      window, nu2 = noise power (caller value, or the mean of s2 over the image).
 *
 * Conventions shared by every entry point
 *   - Image pointers are DEVICE memory owned by the caller. Images are row-major with a
 *     row pitch given in ELEMENTS (>= width). The library never frees them.
 *   - Borders use symmetric padding (... c b a | a b c | c b a ...), repeated
 *     periodically, so windows may be larger than the image.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null stream) and
 *     does not synchronise the device. Scratch memory is allocated and freed in stream
 *     order on that stream (hipMallocAsync / hipFreeAsync).
 *   - Arguments are checked on the host before anything is enqueued; on error nothing
 *     is enqueued, the status is returned and hd_last_error() describes it. A HIP
 *     runtime failure returns HD_ERR_HIP. No C++ exception crosses this boundary.
 *   - Floating-point outputs are float32, normalised: intensity / max_value.
 *   - Input and output buffers must not overlap (windows read neighbours):
 *     HD_ERR_ALIAS.
 *   - Calls on the same stream are ordered; calls on different streams that share
 *     output buffers race, as any two kernels would.
 */
#ifndef HYBRID_DENOISE_H
#define HYBRID_DENOISE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pixel types. Every `dt` argument is an int32_t holding one of these values (any other
 * value is rejected with HD_ERR_DTYPE); a plain integer, so that no caller can hand the
 * library an enumeration value outside the enumeration's range. */
typedef enum {
    HD_U8 = 1,  /* uint8 pixels  */
    HD_U16 = 2  /* uint16 pixels (e.g. 12-bit CT data) */
} hd_dtype;

typedef enum {
    HD_OK = 0,
    HD_ERR_NULL = 1,    /* a required pointer is NULL */
    HD_ERR_DIMS = 2,    /* height / width < 1, pitch < width, or too large */
    HD_ERR_DTYPE = 3,   /* unknown dtype */
    HD_ERR_SMAX = 4,    /* Smax not an odd integer > 1 (Alg. 1, step a), or > HD_SMAX_LIMIT */
    HD_ERR_WINDOW = 5,  /* Wiener window not odd, < 1 or > HD_WIN_LIMIT */
    HD_ERR_MAXVAL = 6,  /* max_value < 1 or above the dtype's range */
    HD_ERR_ALIAS = 7,   /* input and output overlap */
    HD_ERR_NOMEM = 8,   /* scratch allocation failed */
    HD_ERR_HIP = 9,     /* HIP runtime error (launch, device) */
    HD_ERR_ARG = 10,    /* any other bad argument (flags, counts, ...) */
    HD_ERR_TIMEOUT = 11 /* hd_check_errors: a bounded wait of the single-launch path gave up */
} hd_status;

/* AMF flag: a pixel that never passes stage A up to Smax keeps its own value (the
 * listing's initial copy f = g). Default (flag clear): it takes zmed of the Smax window. */
#define HD_AMF_UNRESOLVED_KEEP 1u

/* Hybrid flag: apply the post-processing contrast stretch of Alg. 1, step e to the Wiener
 * output of every slice: out = (out - min) / (max - min) over the slice, so it spans
 * [0, 1]; a constant slice is left unchanged. (The paper names the step only; the linear
 * min-max stretch is this library's reading.) */
#define HD_CONTRAST_STRETCH 2u

#define HD_SMAX_LIMIT 31   /* largest accepted Smax */
#define HD_WIN_LIMIT 15    /* largest accepted Wiener window side */

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t hd_version(void);

/* Message for the last error on the calling thread ("" if none). Valid until the next
 * call on this thread. */
const char *hd_last_error(void);

/* Errors that kernels report after their launch returned. The single-launch path of
 * HD_OPT_RESIDENT exchanges the per-slice noise power (and, with HD_CONTRAST_STRETCH, the
 * output range) across all its workgroups, which must all be on the device at once; the
 * library checks that from the device's occupancy, but other work sharing the device can
 * still keep some of them out. Every wait of that exchange is bounded (HD_OPT_WAIT_LIMIT_US,
 * default 1 s): a workgroup that gives up writes NaN for its pixels, sets a flag in a word
 * the library keeps on the device, and the kernel still ends normally. This call
 * synchronises `stream`, reads and clears that word of the current device and returns
 * HD_ERR_TIMEOUT if any wait gave up since the last check (on any stream), else HD_OK. */
hd_status hd_check_errors(void *stream);

/* Adaptive median filter (Alg. 1, procedure parallelAdapMedian).
 *   in, out      : device images of dtype `dt`, h x w, pitches in elements; out has the
 *                  same dtype; they must not overlap.
 *   smax         : largest window side; odd, 3 <= smax <= HD_SMAX_LIMIT
 *                  (the paper's "SMAX must be an odd integer > 1").
 *   flags        : 0 or HD_AMF_UNRESOLVED_KEEP.
 * The result is exact (integer order statistics): no rounding is involved. */
hd_status amf_filter(const void *in, void *out, int32_t h, int32_t w, int64_t in_pitch,
                     int64_t out_pitch, int32_t dt, int32_t smax, uint32_t flags,
                     void *stream);

/* The paper's frequency-domain Wiener step (Alg. 1, step d: wnrFn(adapOnly, original);
 * Sec. III), which takes the clean original as its second argument. With A = DFT2(in) and
 * F = DFT2(original) (H x W, the image's own size, periodic), the noise spectrum is
 * N = A - F and each frequency is weighted by |F|^2 / (|F|^2 + |N|^2) (0 where both
 * vanish): out = real(IDFT2(gain A)) / max_value. (The paper names the step only; this
 * oracle-assisted Wiener gain is the library's reading.) Float32 transforms.
 *   in, original : device integer images of dtype dt (in: usually the AMF output).
 *   out          : device float32 image; must not overlap the inputs.
 *   h, w         : each <= 4096 with prime factors 2, 3 and 5 only (HD_ERR_DIMS otherwise).
 * Uses stream-ordered library scratch (16 h w bytes). */
hd_status wiener_fft(const void *in, const void *original, float *out, int32_t h, int32_t w, int64_t in_pitch,
                     int64_t orig_pitch, int64_t out_pitch, int32_t dt, int32_t max_value, void *stream);

/* Degradation of a clean image on the device (Alg. 1, step 3, degradImage; the paper names
 * it only). Reading: additive Gaussian noise, then salt and pepper:
 *   g = clip(rint(x + sigma z), 0, max_value)     (z standard normal, half-to-even)
 *   with probability density: g = 0 or max_value (one half each).
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011); pixel p (row-major index) of
 * stream stream_id uses counter (p mod 2^32, p div 2^32, stream_id, 0) under key
 * (seed mod 2^32, seed div 2^32); words r0, r1 give z by Box-Muller in double precision
 * (u1 = (r0 + 1) / 2^32, u2 = r1 / 2^32, z = sqrt(-2 ln u1) cos(2 pi u2)), r2 < floor(density
 * 2^32) makes the impulse and r3 odd makes it max_value. The result depends only on the
 * arguments (no state), never on the launch.
 *   clean, noisy : device images of dtype dt, h x w (pitches in elements); noisy may be
 *                  clean itself (in place, equal pitches), other overlaps are rejected.
 *   sigma        : >= 0, grey levels;  density : 0 .. 1. */
hd_status degrade_image(const void *clean, void *noisy, int32_t h, int32_t w, int64_t clean_pitch,
                        int64_t noisy_pitch, int32_t dt, int32_t max_value, double sigma,
                        double density, uint64_t seed, uint32_t stream_id, void *stream);

/* Post-processing contrast stretch of a float32 image in place (Alg. 1, step e; the reading
 * of HD_CONTRAST_STRETCH): img = (img - min) / (max - min), unchanged when constant.
 *   img          : device float32 image, h x w, pitch in elements.
 * Uses stream-ordered library scratch. */
hd_status contrast_stretch(float *img, int32_t h, int32_t w, int64_t pitch, void *stream);

/* The paper's partitioned AMF (Alg. 1, procedure parallelAdapMedian with `parts`; Fig. 5):
 * the image is cut into `parts` horizontal strips, strip i = rows [floor(i h / parts),
 * floor((i + 1) h / parts)), and every strip is filtered as an image of its own: its
 * windows mirror at the strip's own borders (no halo across the cuts), so pixels near a
 * cut can differ from amf_filter. (The paper does not say how its image splitter cuts; the
 * row strips are this library's reading.) All strips run in one launch.
 *   parts        : 1 .. min(h, HD_PARTS_LIMIT); 1 is amf_filter.
 *   other arguments as in amf_filter. */
#define HD_PARTS_LIMIT 256
hd_status amf_filter_parts(const void *in, void *out, int32_t h, int32_t w, int64_t in_pitch,
                           int64_t out_pitch, int32_t dt, int32_t smax, int32_t parts, uint32_t flags,
                           void *stream);

/* Adaptive Wiener filter of an integer image (the hybrid's second stage, Alg. 1,
 * procedure parallelHybrid, step d; local mean / variance form, see top of file).
 *   in           : device image of dtype `dt` (h x w, in_pitch elements).
 *   out          : device float32 image (h x w, out_pitch elements), normalised by max_value.
 *   max_value    : 1 .. 255 (HD_U8) or 1 .. 65535 (HD_U16).
 *   win_h, win_w : odd window sides, 1 .. HD_WIN_LIMIT.
 *   noise_var    : >= 0: the noise power nu2 in squared grey levels; < 0: estimate it as
 *                  the mean local variance over the image (exact integer sums).
 *   nu2_out      : optional DEVICE double* receiving the nu2 used (NULL to skip). */
hd_status wiener_filter(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                        int64_t out_pitch, int32_t dt, int32_t max_value, int32_t win_h,
                        int32_t win_w, double noise_var, double *nu2_out, void *stream);

/* Hybrid de-noiser: Wiener(AMF(in)) (Sec. IV, Fig. 4; Alg. 1, procedure parallelHybrid,
 * steps b and d), and with HD_CONTRAST_STRETCH in flags the contrast stretch of step e.
 *   amf_out      : optional DEVICE buffer (dtype dt, h x w, amf_pitch elements) receiving
 *                  the AMF stage; NULL -> stream-ordered library scratch.
 *   flags        : HD_AMF_UNRESOLVED_KEEP and / or HD_CONTRAST_STRETCH.
 *   other arguments as in amf_filter / wiener_filter. */
hd_status hybrid_denoise(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                         int64_t out_pitch, int32_t dt, int32_t max_value, int32_t smax,
                         int32_t win_h, int32_t win_w, double noise_var, uint32_t flags,
                         void *amf_out, int64_t amf_pitch, double *nu2_out, void *stream);

/* hybrid_denoise for callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same arguments, result and kernels, but
 * every scratch buffer (the AMF image when amf_out is NULL, per-tile partial sums, the
 * noise power, the single-launch exchange's words) lives in a static device array of
 * HD_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on until the
 * process ends; nothing is allocated or freed. An image whose scratch would not fit
 * (about h * w * bytes-per-pixel, plus 1.1 MB) is rejected with HD_ERR_DIMS before
 * anything is enqueued (a 4096 x 4096 16-bit image fits). All calls on one device share
 * that array: calls that overlap in time on one device (different streams, or threads)
 * race and give undefined results. Each call clears what must start at zero. */
#define HD_NOALLOC_SCRATCH_BYTES (40u << 20)
hd_status hybrid_denoise_noalloc(const void *in, float *out, int32_t h, int32_t w, int64_t in_pitch,
                                 int64_t out_pitch, int32_t dt, int32_t max_value, int32_t smax,
                                 int32_t win_h, int32_t win_w, double noise_var, uint32_t flags,
                                 void *amf_out, int64_t amf_pitch, double *nu2_out, void *stream);

/* ---- batched path ------------------------------------------------------------------
 * Many slices of uneven sizes in one call: the tiles of all slices form one work list,
 * each stage is one launch over it, and the noise power nu2 is estimated per slice
 * (exact per-slice sums). The first call with a given slice list builds a plan (device
 * slice table, scratch for the AMF stage and the per-slice sums) and captures the stage
 * launches into a hipGraph; later calls with the same list (same pointers, sizes and
 * parameters) replay the graph with one hipGraphLaunch. When `stream` is itself being
 * captured, the stage kernels are enqueued directly (they land in the caller's graph).
 * A plan's scratch is shared by every call that reuses the plan: two such calls in
 * flight on different streams race. Up to 8 plans are cached per process; an evicted plan
 * is freed once its last run has completed (an event; nothing waits for the device). A plan
 * whose kernels were captured into the caller's own graph must stay cached while that
 * graph is replayed. hd_release_plans() frees them all. */
typedef struct {
    const void *in;     /* device image, dtype of the call, h x w, in_pitch elements */
    float *out;         /* device float32 output, h x w, out_pitch elements */
    int32_t h, w;
    int64_t in_pitch, out_pitch;
} hd_slice;

/* Hybrid de-noiser over n slices (host array `slices`, copied into the plan).
 * Arguments and errors as hybrid_denoise; a failing slice check names the slice. */
hd_status hybrid_denoise_batched(const hd_slice *slices, int32_t n, int32_t dt,
                                 int32_t max_value, int32_t smax, int32_t win_h, int32_t win_w,
                                 double noise_var, uint32_t flags, void *stream);

/* Diagnostics: one step of hybrid_denoise_batched (same slices, parameters, plan and
 * strategy, same kernels) enqueued as plain launches on `stream` with HIP events around
 * every stage kernel; waits for them and writes each stage's duration in milliseconds to
 * stage_ms (host array of HD_STAGES floats; 0 for a stage the step does not run):
 *   [0] the AMF stage (or the whole hybrid when it runs as one launch), [1] the separate
 *   noise-power sums, [2] the per-slice noise-power reduction, [3] the Wiener apply,
 *   [4] the contrast stretch. The outputs are those of hybrid_denoise_batched.
 * Synchronises `stream`; not capturable (HD_ERR_ARG while `stream` is being captured). */
#define HD_STAGES 5
hd_status hybrid_denoise_batched_timed(const hd_slice *slices, int32_t n, int32_t dt,
                                       int32_t max_value, int32_t smax, int32_t win_h, int32_t win_w,
                                       double noise_var, uint32_t flags, float *stage_ms,
                                       void *stream);

/* Frees every cached batched plan, after waiting for each plan's own last run. */
void hd_release_plans(void);

/* ---- strategy options and autotuner --------------------------------------------------
 * Every strategy gives bit-identical results; they differ only in speed.
 *   HD_OPT_SELECT        work split and median selection at window levels >= 5:
 *                        0 = adaptive: a very short list of pending pixels runs four
 *                        pixels per wave through all its levels; a longer list runs level
 *                        by level, one lane per pixel (bisection) when it fills the
 *                        workgroup, else several pixels per wave (lane groups); 3 = as 0
 *                        with a register sorting network for the 5x5 median and lane
 *                        groups from level 7 on (for dense impulse noise); 1 = one lane per
 *                        pixel with bisection everywhere; 2 = one wave per pixel everywhere
 *                        (ballot radix select); -1 = the autotuned choice (default 0).
 *   HD_OPT_FUSE_MOMENTS  1 = the AMF stage also computes the Wiener noise-power sums on a
 *                        ring around each tile; 0 = a separate pass over the AMF output;
 *                        -1 = autotuned (default).
 *   HD_OPT_GRAPHS        1 = batched calls replay a captured hipGraph (default); 0 = plain
 *                        launches.
 *   HD_OPT_RESIDENT      1 = (default, also -1) when the noise power is estimated, no tile
 *                        list is given, the call holds at most 8 slices and every tile's
 *                        workgroup fits on the device at once, the whole hybrid runs as
 *                        ONE launch: AMF with the Wiener ring,
 *                        window sums, a grid-wide exchange of the slice noise powers, Wiener
 *                        output (the AMF image is written only when the caller asks for it);
 *                        0 = always the staged launches. Concurrent calls sharing a batched
 *                        plan (same slices and parameters) on different streams must not
 *                        overlap, as for every batched call. */
/*   HD_OPT_WAIT_LIMIT_US bound of every wait of the single-launch exchange, in microseconds
 *                        (-1 = default 1 s; 0 = a workgroup that would wait gives up at
 *                        once, for tests of the error path). See hd_check_errors.
 *   HD_OPT_FAIL_ALLOC    fault injector: n > 0 makes the n-th scratch allocation from now
 *                        fail with HD_ERR_NOMEM (nothing is enqueued), then disarms; 0
 *                        disarms. The environment variable HD_FAIL_ALLOC=n arms it at the
 *                        library's first allocation.
 *   HD_OPT_TILE_ROWS     height of the AMF stage's tiles in the staged path without the
 *                        noise-sum fusion: 16, 32 or 64 rows of 64 columns; -1 = the
 *                        autotuned choice (default 32). Every other stage keeps 64 x 32 tiles.
 *   HD_OPT_SURROGATE_FUSED  surrogate inference (surrogate_forward, surrogate_denoise):
 *                        0 = one launch per layer as in training (default); 1 = the whole
 *                        network in one launch that streams down the image rows through
 *                        LDS (5 bytes of HBM traffic per pixel instead of ~640; no
 *                        activation stored); bit-identical.
 */
#define HD_OPT_SELECT 1
#define HD_OPT_FUSE_MOMENTS 2
#define HD_OPT_GRAPHS 3
#define HD_OPT_RESIDENT 4
#define HD_OPT_WAIT_LIMIT_US 5
#define HD_OPT_FAIL_ALLOC 6
#define HD_OPT_SURROGATE_FUSED 7
#define HD_OPT_TILE_ROWS 8
hd_status hd_set_option(int32_t key, int32_t value);

/* Largest number of 64 x 32 output tiles (ceil(w / 64) * ceil(h / 32), summed over the
 * slices of one call) that the single-launch path of HD_OPT_RESIDENT takes on the current
 * device for (dtype, smax, window, select_mode); select_mode as HD_OPT_SELECT, -1 = the
 * tuned or default choice. Returns 0 for invalid arguments or when the device cannot
 * report its occupancy. Calls with more tiles, more than 8 slices, a caller-given noise
 * power or a tile list take the staged launches. Host only; enqueues nothing. */
int32_t hd_resident_capacity(int32_t dt, int32_t smax, int32_t win_h, int32_t win_w,
                             int32_t select_mode);

/* Times every strategy on one image (device memory, `iters` timed runs each, after one
 * warm-up; synchronises `stream`) and records the fastest for (dtype, smax, window).
 * The strategies: selection mode x noise-sum fusion, and for the unfused AMF stage also
 * 16- and 64-row tiles besides the 32-row default (HD_OPT_TILE_ROWS). Later calls with
 * that key use it unless an option overrides it. When the environment variable
 * HD_AUTOTUNE_CACHE names a file, the table is loaded from it on first use and rewritten
 * after each tuning. best_select / best_fuse / best_tile_rows (host, may be NULL) receive
 * the choice. */
hd_status hd_autotune_hybrid(const void *in, int32_t h, int32_t w, int64_t in_pitch,
                             int32_t dt, int32_t max_value, int32_t smax, int32_t win_h,
                             int32_t win_w, int32_t iters, int32_t *best_select,
                             int32_t *best_fuse, int32_t *best_tile_rows, void *stream);

/* The autotuner on a batch as it will run: every strategy (as in hd_autotune_hybrid) times
 * `iters` batched calls (after one warm-up) on these slices, each strategy with a plan of
 * its own that is freed afterwards, and the fastest is recorded for (dtype, smax, window).
 * Writes the slices' outputs; synchronises `stream`; not capturable. best_select /
 * best_fuse / best_tile_rows (host, may be NULL) receive the choice. */
hd_status hd_autotune_batched(const hd_slice *slices, int32_t n, int32_t dt, int32_t max_value,
                              int32_t smax, int32_t win_h, int32_t win_w, int32_t iters,
                              int32_t *best_select, int32_t *best_fuse, int32_t *best_tile_rows,
                              void *stream);

/* ---- learned surrogate ---------------------------------------------------------------
 * A small convolutional stand-in for the hybrid filter, trained on (noisy, plain hybrid
 * output) pairs that the plain method produces; the plain path stays the reference.
 * Network: x = g / max_value; six 3x3 convolutions with zero padding (1 -> 32, four
 * 32 -> 32, 32 -> 1), ReLU after the first five, output y = x + last layer. Weights and
 * activations bf16 (round to nearest even), fp32 accumulation; the 32 -> 32 layers run
 * on the matrix cores in the forward and both backward passes. Parameters: flat fp32
 * vector of surrogate_num_params() values in the order W1 [9][32] (tap = ky*3+kx, out),
 * b1 [32], then for each 32 -> 32 layer W [9][32][32] (tap, out, in) and b [32], then
 * W6 [9][32] (tap, in), b6 [1]. Training: mean squared error to the target, Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on fp32 master weights.
 * Images of one call are a batch of n_img equal-size images: image i starts at
 * in + i * img_stride elements, rows pitch elements apart; n_img, h, w in 1 .. 65535 and
 * n_img * h * w <= 2^31 (HD_ERR_DIMS otherwise). A surrogate object owns device
 * buffers sized for the largest batch it has seen; they are regrown in stream order.
 * Calls on one object must not overlap in time (one stream, or external ordering). */
typedef struct hd_surrogate hd_surrogate;

int32_t surrogate_num_params(void);

/* init_params: host array of surrogate_num_params() floats, or NULL for zeros. */
hd_status surrogate_create(hd_surrogate **out, const float *init_params);
void surrogate_destroy(hd_surrogate *s);

/* Host copies of the parameters, Adam moments and step (any pointer may be NULL); both
 * calls synchronise the device. set_state is also the checkpoint-resume entry point. */
hd_status surrogate_get_state(hd_surrogate *s, float *params, float *m, float *v, int32_t *step);
hd_status surrogate_set_state(hd_surrogate *s, const float *params, const float *m,
                              const float *v, int32_t step);

/* Diagnostics: host copy of the stored activation A_layer (layer 1..5: the output of
 * convolution `layer` after its ReLU, bf16 bit patterns, NHWC [n_img][h][w][32]) of the
 * object's last surrogate_forward or surrogate_train_step; count = n_img * h * w * 32 of
 * that call. HD_ERR_ARG for another count, a layer outside 1..5, or a layer that call did
 * not keep (the one-launch inference of HD_OPT_SURROGATE_FUSED keeps none).
 * Synchronises the device. */
hd_status surrogate_get_activation(hd_surrogate *s, int32_t layer, uint16_t *host, int64_t count);

/* y = network(in) for a batch; out is float32 with its own pitch / image stride. */
hd_status surrogate_forward(hd_surrogate *s, const void *in, int32_t n_img, int32_t h, int32_t w,
                            int64_t pitch, int64_t img_stride, int32_t dt, int32_t max_value,
                            float *out, int64_t out_pitch, int64_t out_img_stride, void *stream);

/* One training step on a batch: forward, loss = mean (y - target)^2 (target: dense device
 * float32 [n_img][h][w]), backward. loss_out / grad_out: optional DEVICE float pointers
 * (grad_out: surrogate_num_params() floats). apply_update != 0: Adam step with rate lr. */
hd_status surrogate_train_step(hd_surrogate *s, const void *in, int32_t n_img, int32_t h,
                               int32_t w, int64_t pitch, int64_t img_stride, int32_t dt,
                               int32_t max_value, const float *target, float lr, float *loss_out,
                               float *grad_out, int32_t apply_update, void *stream);

/* De-noise slices with the surrogate, check every 64 x 64 tile, and send failing tiles to
 * the plain path. Per tile: frac = share of pixels at 0 or max_value, res = mean (x - y)^2
 * over the other pixels (the plain filter's residual statistics, calibrated on training
 * data: p_max, r_lo, r_hi), and, with d_hi > 0, dev = mean (y - p)^2 over the tile, the
 * deviation of the surrogate output y from a proxy p of the plain output: the plain hybrid
 * with the AMF stopped at window check_smax (3 <= check_smax <= smax, odd), computed by the
 * batched call; d_hi is a root-mean-square deviation bound (calibrated as the plain output's
 * typical distance from the same proxy, so that a passing tile's distance from the plain
 * output is at most about (1 + threshold) d_hi). score = max(frac / p_max, res / r_hi,
 * r_lo / res, dev / d_hi^2) (infinite when res = 0); a tile passes when score < threshold
 * (0: every tile falls back; +inf: none). Failing tiles get the plain AMF (Smax) and
 * Wiener (win_h x win_w) output, with the noise power estimated over the failing tiles of
 * their slice, so threshold 0 reproduces hybrid_denoise exactly. n_fallback_out (device
 * int32, may be NULL) receives the number of 64 x 32 work tiles redone; tile_scores_out
 * (device float32, may be NULL) the scores, slice by slice, 64 x 64 tiles row-major.
 * Asynchronous on `stream` (scratch is regrown in stream order; the call waits only for
 * the previous call's table upload before reusing its pinned host buffer). */
hd_status surrogate_denoise(hd_surrogate *s, const hd_slice *slices, int32_t n, int32_t dt,
                            int32_t max_value, int32_t smax, int32_t win_h, int32_t win_w,
                            float p_max, float r_lo, float r_hi, float d_hi, int32_t check_smax,
                            float threshold, int32_t *n_fallback_out, float *tile_scores_out,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HYBRID_DENOISE_H */

/*
 * sar_rda.h -- C ABI of the MI355X (gfx950) SAR Range Doppler Algorithm
 * library, libsar_rda.so.
 *
 * The method is the kernel-fused Range Doppler Algorithm of "From 8 Seconds
 * to 370 ms: Kernel-Fused SAR Imaging on Apple Silicon via Single-Dispatch
 * FFT Pipelines" (arXiv 2604.03585):
 *   Sec. II.B  one line = FFT -> matched-filter multiply -> IFFT, fused so
 *              the line is read once from and written once to device memory;
 *   Sec. II.C  the inverse transform is the conjugated forward transform
 *              scaled by 1/N;
 *   Sec. IV.A  range compression of every range line, azimuth FFT, range
 *              cell migration correction (RCMC) by sinc interpolation in the
 *              range-Doppler domain, azimuth compression (filter multiply +
 *              IFFT); Sec. IV.B the corner turn between the two passes.
 *
 * Conventions shared by every entry point:
 *  - Scene data are interleaved complex64 (float re, float im), row-major.
 *    Raw echo and range-compressed data are [Na][Nr] (one range line per
 *    row); after the corner turn the azimuth pass works on [Nr][Na].
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors), 16-byte aligned.  The caller owns every data and workspace
 *    buffer; a plan owns only its own tables.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every execute call is asynchronous: it validates its arguments on the
 *    host, enqueues kernels and returns.  A returned status reports argument
 *    or launch errors only; faults during execution surface at the caller's
 *    next synchronisation as HIP errors.
 *  - On any non-OK status nothing has been enqueued (validation precedes the
 *    first launch) except for SAR_ERR_HIP, which may follow earlier launches
 *    of the same call.  sar_last_error() then returns a message (per thread).
 *  - Plans are immutable after sar_plan(); one plan may be used from several
 *    streams at once as long as each call has its own data and workspace.
 *  - No C++ exception crosses this interface.
 */
#ifndef SAR_RDA_H
#define SAR_RDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sar_plan_s* sar_plan_t;
typedef struct sar_batch_s* sar_batch_t;

typedef enum {
    SAR_OK = 0,
    SAR_ERR_NULL = 1,        /* a required pointer is NULL                    */
    SAR_ERR_BAD_SIZE = 2,    /* a size is not a power of two / out of range  */
    SAR_ERR_BAD_PARAM = 3,   /* an enum or physical parameter is invalid     */
    SAR_ERR_ALIAS = 4,       /* buffers overlap where they must not          */
    SAR_ERR_NO_MEMORY = 5,   /* a device or host allocation failed           */
    SAR_ERR_HIP = 6,         /* a HIP runtime call or launch failed          */
    SAR_ERR_UNSUPPORTED = 7  /* valid request the library does not implement */
} sar_status;

typedef enum { SAR_AZ_LFM = 0, SAR_AZ_HYPERBOLIC = 1 } sar_az_model;
typedef enum {
    SAR_FP32 = 0,
    SAR_SPLIT_FP16 = 1,
    SAR_SPLIT_BF16 = 2,
    SAR_FP32_HALF_STORAGE = 3
} sar_precision;
typedef enum { SAR_FUSED = 0, SAR_UNFUSED = 1, SAR_TURN_FREE = 2 } sar_schedule;

/*
 * Processing parameters (normalised units: one range cell = 1, one pulse
 * repetition interval = 1, so chirp rates are cycles/sample^2, `v` is in
 * cells/pulse and `lambda` in cells).
 *
 *  Nr, Na          range / azimuth line lengths, powers of two, 64..16384.
 *  range_len       L_r, range replica length, 1..Nr; range_tbp its
 *                  time-bandwidth product (K_r = tbp / L_r^2).  The range
 *                  filter is H_r = conj(DFT(h_r)) of the circularly centred
 *                  up-chirp replica h_r[u mod Nr] = exp(j pi K_r u^2),
 *                  u = -L_r/2 .. L_r/2-1  (Sec. II.B; H_r itself is not
 *                  specified by the paper, this is our reading).
 *  az_model        SAR_AZ_LFM: zero-migration azimuth; H_a is built like H_r
 *                  from the down-chirp exp(-j pi K_a u^2), u over az_len
 *                  samples, K_a = az_tbp / az_len^2.
 *                  SAR_AZ_HYPERBOLIC: exact-geometry azimuth filter
 *                  exp(+j 4 pi R0 D(f) / lambda), D(f) = sqrt(1-(lambda f/2v)^2),
 *                  R0 = r_near + n, after RCMC (Sec. IV.A steps 3-4).
 *  lambda, v, r_near  hyperbolic geometry (ignored for LFM).
 *  rcmc_taps       0 (no RCMC) or 8: Kaiser-windowed sinc, taps -3..4 about
 *                  floor(p), weights normalised to unit sum; rcmc_beta is the
 *                  Kaiser beta (2.5 by default).
 *  precision       SAR_FP32, or the split-FP16 / split-BF16 MFMA butterflies,
 *                  or SAR_FP32_HALF_STORAGE: FP32 arithmetic, but
 *                  sar_rda_execute keeps its intermediates (range-compressed,
 *                  turned and range-Doppler data) in the workspace as FP16
 *                  pairs with one power-of-two exponent per line, chosen so
 *                  the line's largest component lands in [2^14, 2^15).
 *                  That moves 40 instead of 64 bytes per pixel, at the
 *                  precision of two FP16 roundings (the paper's Sec. VI
 *                  mixed-precision future work).  It needs the fused
 *                  schedule, transpose_back = 0 and, for the hyperbolic model,
 *                  8-tap RCMC with stretch < 0.5 (else SAR_ERR_UNSUPPORTED).
 *                  The individual step functions, which take and return
 *                  complex64, run as SAR_FP32.
 *  schedule        SAR_FUSED (one kernel per line pass) or SAR_UNFUSED
 *                  (separate FFT, multiply and IFFT dispatches, Sec. II.B
 *                  Fig. 1 top) -- the comparator -- or SAR_TURN_FREE: the
 *                  fused kernels without the corner turn (Sec. VI, future
 *                  work on the transposes that dominate the azimuth steps):
 *                  sar_rda_execute's azimuth kernel reads strips of adjacent
 *                  azimuth lines straight from the range pass's [Na][Nr]
 *                  output (FP32, Na <= 4096, transpose_back = 0; else
 *                  SAR_ERR_UNSUPPORTED).  Images are bit-identical to
 *                  SAR_FUSED's; the step entry points behave as for
 *                  SAR_FUSED.
 *  transpose_back  0: sar_rda_execute leaves the image as [Nr][Na];
 *                  1: it is turned back to [Na][Nr].
 */
typedef struct {
    uint32_t struct_size;     /* must equal sizeof(sar_params) */
    int32_t  Nr, Na;
    int32_t  range_len;
    double   range_tbp;
    int32_t  az_model;
    int32_t  az_len;
    double   az_tbp;
    double   lambda, v, r_near;
    int32_t  rcmc_taps;
    double   rcmc_beta;
    int32_t  precision, schedule, transpose_back;
} sar_params;

/* Build a plan (Sec. II.B: the matched filter is pre-computed once, outside
 * the per-line pipeline; Sec. II.C: the IFFT's 1/N scale is applied once, here
 * folded into the filter; Sec. IV.A: the filters H_r and H_a(f_a, R0) and the
 * RCMC geometry).  Validates `p`, allocates the plan's device tables and fills
 * them on `stream` with FP64 generator kernels (twiddles exp(-2 pi i k/N),
 * the matched filters with the IFFT's 1/N folded in, and for the hyperbolic
 * model the per-Doppler-bin RCMC stretch 1/D-1 and phase rate 2D/lambda).
 * Synchronises `stream` before returning.  *out receives the plan; on any
 * error *out is left NULL and nothing stays allocated. */
sar_status sar_plan(const sar_params* p, void* stream, sar_plan_t* out);

/* Free a plan.  The caller must have synchronised every stream that used it. */
void sar_plan_destroy(sar_plan_t plan);

/* Bytes of device workspace sar_rda_execute / sar_azimuth_compress need:
 * 8 * Na * Nr (one scene-sized complex64 buffer); for SAR_FP32_HALF_STORAGE
 * two FP16 scene arrays plus 4 * (Na + Nr) bytes of exponents (each block
 * 256-byte aligned). */
size_t sar_workspace_bytes(sar_plan_t plan);

/* Range compression (Sec. IV.A step 1): every row of in_dev [Na][Nr] goes
 * through FFT, times H_r, IFFT into out_dev [Na][Nr].  in_dev == out_dev is
 * allowed; partial overlap is SAR_ERR_ALIAS. */
sar_status sar_range_compress(sar_plan_t plan, const void* in_dev, void* out_dev,
                              void* stream);

/* Corner turn (Sec. IV.B): out_dev[c][r] = in_dev[r][c] for an in_dev of
 * rows x cols complex64 (each 1..2^20, rows*cols <= 2^31).  Bit-exact.
 * Out of place only (overlap is SAR_ERR_ALIAS).  `plan` may be NULL. */
sar_status sar_corner_turn(sar_plan_t plan, const void* in_dev, void* out_dev,
                           int32_t rows, int32_t cols, void* stream);

/* Azimuth compression on range-major data in_dev [Nr][Na] into out_dev
 * [Nr][Na] (Sec. IV.A steps 2-4).  LFM: FFT * H_a * IFFT per row; in_dev ==
 * out_dev allowed and work_dev unused (may be NULL).  Hyperbolic: azimuth
 * FFT into work_dev, then RCMC + azimuth phase + IFFT into out_dev; in_dev
 * may equal out_dev, work_dev (>= sar_workspace_bytes) must overlap neither. */
sar_status sar_azimuth_compress(sar_plan_t plan, const void* in_dev, void* out_dev,
                                void* work_dev, void* stream);

/* Whole RDA (Sec. IV.A): raw_dev [Na][Nr] -> img_dev ([Nr][Na], or [Na][Nr]
 * with transpose_back).  raw_dev is read only.  work_dev holds
 * sar_workspace_bytes(plan).  The three buffers must be pairwise disjoint. */
sar_status sar_rda_execute(sar_plan_t plan, const void* raw_dev, void* img_dev,
                           void* work_dev, void* stream);

/* Bytes of the library's static workspace (one per GPU, held from the first
 * plan on that GPU until the process ends): 128 MiB, the FP32 workspace of
 * a 4096 x 4096 scene (the paper's scene size). */
#define SAR_NOALLOC_WORKSPACE_BYTES ((size_t)128 << 20)

/* sar_rda_execute for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same kernels as sar_rda_execute, with the workspace taken from a
 * static device array of SAR_NOALLOC_WORKSPACE_BYTES instead of a caller's
 * buffer; it calls no hipMalloc, hipFree or other allocating routine (the
 * array's device address is looked up once per GPU by sar_plan).  The caller
 * passes raw_dev and img_dev as for sar_rda_execute (disjoint).  A plan whose
 * sar_workspace_bytes exceed SAR_NOALLOC_WORKSPACE_BYTES gets
 * SAR_ERR_BAD_SIZE; SAR_ERR_HIP if the static array is unavailable on the
 * plan's device.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other threads) race on it and
 * must be serialised by the caller.  Nothing in the array needs to start at
 * zero (every step writes what the next one reads). */
sar_status sar_rda_execute_noalloc(sar_plan_t plan, const void* raw_dev, void* img_dev,
                                   void* stream);

/* Measurement (the per-kernel durations the benchmark reports, the analogue
 * of Sec. V.C Table III's per-step breakdown): the next n kernels launched by
 * the library on the calling thread record start_events[i] when kernel i
 * starts and stop_events[i] when it ends.  The timestamps come from each
 * kernel's own dispatch (hipExtLaunchKernel), so an interval is the kernel's
 * duration as a profiler's kernel trace reports it, without the launch gaps
 * that events recorded between launches include.  The events are
 * hipEvent_t the caller created with timing enabled and keeps alive until
 * they have completed.  n = 0 disarms; n outside 0..16 is SAR_ERR_BAD_SIZE,
 * a NULL array or event SAR_ERR_NULL (nothing armed then).  sar_rda_execute
 * launches 4 kernels for a fused FP32 hyperbolic plan (range, corner turn,
 * azimuth FFT, RCMC), 3 for LFM or for SAR_TURN_FREE hyperbolic, 2 for
 * SAR_TURN_FREE LFM. */
sar_status sar_time_next_launches(void* const* start_events, void* const* stop_events, int32_t n);

/* ---- individual steps, for step-by-step testing and the unfused path ---- */

/* Forward (inverse = 0) or inverse (inverse = 1, including 1/N) FFT of
 * `lines` contiguous lines of length N = Nr (axis 0) or Na (axis 1).
 * in_dev == out_dev allowed. */
sar_status sar_fft_lines(sar_plan_t plan, int32_t axis, int32_t inverse,
                         const void* in_dev, void* out_dev, int32_t lines,
                         void* stream);

/* Azimuth FFT of the range-Doppler pass (Sec. IV.A step 2): every row of
 * in_dev [Nr][Na] -> out_dev [Nr][Na].  Same as sar_fft_lines(axis 1). */
sar_status sar_azimuth_fft(sar_plan_t plan, const void* in_dev, void* out_dev,
                           void* stream);

/* RCMC + exact-geometry azimuth phase + azimuth IFFT (Sec. IV.A steps 3-4)
 * on range-Doppler data A_dev [Nr][Na] -> out_dev [Nr][Na].  Hyperbolic
 * plans only.  A_dev and out_dev must not overlap (RCMC reads rows up to
 * ~18 cells away). */
sar_status sar_rcmc_azimuth(sar_plan_t plan, const void* A_dev, void* out_dev,
                            void* stream);

/* Copy one of the plan's tables to host memory (tests of the FP64
 * generators).  which: 0 H_r (Nr complex64, includes 1/Nr), 1 H_a (Na
 * complex64, includes 1/Na; LFM only), 2 RCMC stretch 1/D-1 (Na doubles;
 * hyperbolic), 3 phase rate 2D/lambda (Na doubles; hyperbolic), 4 RCMC
 * weight coefficients (3072 floats; hyperbolic): 128 intervals of x in
 * [0, 1), on interval b the weight of tap t (t = 0..7 for taps -3..4) is
 * sum_j c[b*24 + t*3 + j] u^j with u = 128 x - b (a quadratic fitted at
 * three Chebyshev nodes to the exact FP64 Kaiser-sinc weights).
 * host_bytes must be at least the table size. Synchronous. */
sar_status sar_plan_get_table(sar_plan_t plan, int32_t which, void* host_dst,
                              size_t host_bytes);

/* ---- batched execution (scenes of uneven size) ----
 *
 * Not in the paper: the batching pattern for many scenes.  Scenes with LFM
 * azimuth and the fused schedule share launches: one line launch per (pass,
 * line length, precision) and one corner-turn launch per turn, each a grid
 * over all scenes' line groups or tiles (task lists in device memory).  Every
 * other scene (hyperbolic, unfused, half storage, and any scene of 2^22
 * pixels or more, which fills the GPU with its own launches) runs as
 * sar_rda_execute in the same stream, in scene order, after the shared
 * launches; those of 2^22 pixels or more with the fused schedule in FP32,
 * Na <= 4096 and no back-turn run the turn-free kernels (SAR_TURN_FREE).
 * Each scene's image is bit-identical to its own sar_rda_execute.
 */

/* Plan `n` scenes (params ps[0..n-1], n >= 1): validates every parameter set
 * (errors as sar_plan, reported for the first invalid scene), builds one plan
 * per distinct parameter set on `stream` (synchronised), and lays out the
 * scenes' workspaces in one buffer.  *out receives the batch. */
sar_status sar_batch_plan(const sar_params* ps, int32_t n, void* stream,
                          sar_batch_t* out);

/* Device workspace bytes for sar_batch_execute: the scenes' workspaces,
 * each 256-byte aligned.  0 for a NULL batch. */
size_t sar_batch_workspace_bytes(sar_batch_t batch);

/* Run every scene: raw_dev[i] [Na_i][Nr_i] -> img_dev[i] (layout as in
 * sar_rda_execute).  raw_dev / img_dev are host arrays of n device pointers
 * (16-byte aligned); work_dev holds sar_batch_workspace_bytes(batch).  The
 * images and the workspace must not overlap each other or any raw input
 * (SAR_ERR_ALIAS); raw inputs are only read and may be shared by scenes.
 * The first call with a set of buffer pointers (and stream) builds the task
 * lists and uploads them synchronously (after synchronising the stream of
 * the previous set, whose replays may still read them); on a non-null stream
 * it then captures the whole batch into a hipGraph, and every later call with
 * the same pointers replays that graph (asynchronous).  On the null stream
 * the launches are issued directly.  Errors: SAR_ERR_NULL, SAR_ERR_BAD_PARAM
 * (misaligned buffers, another device than at planning), SAR_ERR_ALIAS,
 * SAR_ERR_NO_MEMORY (task buffer), SAR_ERR_HIP. */
sar_status sar_batch_execute(sar_batch_t batch, const void* const* raw_dev,
                             void* const* img_dev, void* work_dev, void* stream);

/* Free the batch, its plans, task buffer and graph (NULL is a no-op).  The
 * caller must first synchronise any stream a replay of it was queued on. */
void sar_batch_destroy(sar_batch_t batch);

/* ---- autotuner (the batching/serving pattern: measured kernel choices) ----
 *
 * Kernel variants are chosen per (kind, line length N, precision); every
 * variant computes the same result, they differ in scheduling only:
 *   kind 0 fused FFT*H*IFFT, 1 forward FFT, 2 inverse FFT line kernels:
 *          variant bit 0 = twiddles read from the table (else by products
 *          of two table loads per radix-16 pass; FP32 butterflies only);
 *          kinds 1 and 2 (FP32): bit 1 = real and imaginary parts exchanged
 *          through LDS as two float arrays (the split layout of the MFMA
 *          passes; else one array of complex pairs); bit 2 (FP32, N <= 8192)
 *          = twice the default lines per workgroup (8192 points per
 *          workgroup up to N = 4096, two lines at 8192);
 *   kind 3 RCMC + azimuth kernel: bit 0 as above for its IFFT, bit 1 = one
 *          output row per line slot (else two rows sharing their gathers),
 *          bit 2 = the two rows on two line slots' threads instead of one's
 *          (FP32 and Na = 4096 or 8192 only);
 *   kind 4 batched fused line kernel: bit 0 as above, bits 2-3 = grid
 *          (0: one workgroup per line group; 1, 2, 3: a persistent grid of
 *          1x, 2x, 4x the resident workgroups);
 *   kind 5 corner turn, keyed by the row length of the matrix it turns
 *          (precision 0): variant 0 = a grid of five workgroups per CU,
 *          1 = four per CU, 2 = one workgroup per 64 x 64 tile;
 *   kind 6 turn-free azimuth strips, keyed by the azimuth line length
 *          (precision 0): variant 0 = the default strip width, 1 = half of
 *          it (half the LDS and threads per workgroup, shorter row runs).
 * The process-wide table starts with every variant 0.  A plan copies the
 * table's choices for its sizes when it is created (sar_plan, sar_batch_plan);
 * the first plan of the process loads $SAR_AUTOTUNE_CACHE if that is set.
 *
 * The cache is a JSON-lines text file, one flat object per tuned kernel:
 *   {"arch":"gfx950","kind":"fused","n":4096,"prec":0,"variant":1,
 *    "us_default":64.1,"us_best":61.9}
 * (kind names: "fused", "fwd", "inv", "rcmc", "batch_fused", "turn", "strip").  Lines for
 * other architectures are preserved; malformed lines are ignored.
 */

/* Time every candidate variant of the kernels a plan of *p launches (its
 * line kernels, its corner turns or turn-free strips, and, for fused LFM
 * parameters, the batched fused line kernel for Nr and Na) on
 * the current device, interleaving candidates over five timed rounds of eight
 * launches and keeping the best; a variant other than 0 wins only if it is at
 * least 2 % faster.  The winners enter the process-wide table (plans created
 * afterwards use them) and are merged into the cache at cache_path (NULL:
 * $SAR_AUTOTUNE_CACHE; neither set: table only).  Allocates two scene-sized
 * device buffers for the duration; synchronous.
 * Errors: those of sar_plan; SAR_ERR_NO_MEMORY; SAR_ERR_HIP; SAR_ERR_BAD_PARAM
 * if the cache cannot be written. */
sar_status sar_autotune(const sar_params* p, const char* cache_path);

/* Replace the process-wide table by the entries of the cache at path whose
 * "arch" equals arch (NULL: the current device's gfx name, e.g. "gfx950").
 * path NULL clears the table.  Host-only when arch is given.  After this call
 * $SAR_AUTOTUNE_CACHE is no longer read.  Errors: SAR_ERR_BAD_PARAM if path
 * cannot be read; SAR_ERR_HIP if arch is NULL and there is no device. */
sar_status sar_tune_load(const char* path, const char* arch);

/* The table's variant for (kind, n, precision): 0 when nothing is tuned,
 * -1 for an unknown kind.  Host-only. */
int32_t sar_tune_variant(int32_t kind, int32_t n, int32_t precision);

/* Message for the last non-OK status on the calling thread ("" if none). */
const char* sar_last_error(void);

/* Library version string. */
const char* sar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SAR_RDA_H */

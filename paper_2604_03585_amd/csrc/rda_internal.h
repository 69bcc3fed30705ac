// rda_internal.h -- declarations shared by the host API and the kernel
// launchers inside libsar_rda.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "sar_rda.h"

struct sar_plan_s;

namespace sar {

// Record a message for sar_last_error() on this thread and return `st`.
sar_status set_error(sar_status st, const char* fmt, ...);
void clear_error();

// The next pair of events sar_time_next_launches armed on this thread, if
// any: taken by the next kernel launch, which records them at its start and
// end.
bool take_launch_events(hipEvent_t& start, hipEvent_t& stop);

enum class LineOp { Fused, Forward, Inverse, RcmcAz };

// One scene's share of a batched line launch: `lines` lines of `in` -> `out`
// with this scene's filter and twiddles; group_begin is the index of its
// first line group in the launch (tasks sorted by it).
struct LineTask {
    const float2* in;
    float2* out;
    const float2* H;
    const float2* tw;
    int lines;
    int group_begin;
};

// One matrix of a batched corner turn (rows x cols -> cols x rows).
struct TurnTask {
    const float2* in;
    float2* out;
    int rows, cols;
    int tile_begin;
};

// Host-side description of the hyperbolic azimuth tables and RCMC kernel.
struct RcmcHost {
    const double* stretch;   // device, Na doubles: 1/D_k - 1
    const double* rate;      // device, Na doubles: 2 D_k / lambda
    const float* table;      // device, rcmc_table_floats() weight coefficients
    double r_near;
    double stretch_max;      // largest stretch_k (at |f| = 1/2)
    double x_per_bin;        // lambda / (2 v Na)
    double two_over_lam;     // 2 / lambda
    int taps;                // 0 or 8
    int nr;                  // range lines (rows of the [Nr][Na] data)
};

// Line kernels for line length n in {64, ..., 16384}.
//  Fused:   out = IFFT(FFT(in) * H)   (H includes 1/n)
//  Forward: out = FFT(in) * scale;  Inverse: out = unscaled IFFT(in) * scale
//  RcmcAz:  out[n] = IFFT(RCMC(in)[n] * phase / n), rh required, lines = rh->nr
//  prec: 0 FP32 butterflies, 1 split FP16 / 2 split BF16 radix-16 butterflies on MFMA
//  variant (autotuned): bit 0 twiddles from the table instead of by products
//  (Forward / Inverse FP32 also bit 1: split real/imaginary LDS exchange),
//  bit 1 one RCMC output row per line slot instead of two, bit 2 the two RCMC
//  rows on two line slots' threads instead of one's (FP32, N = 4096 / 8192)
hipError_t launch_line(LineOp op, int n, const void* in, void* out, int lines, const void* H,
                       const void* tw, float scale, const RcmcHost* rh, int prec, int variant,
                       hipStream_t s);
int twiddle_table_size(int n);

// Column-strip azimuth pass (turn-free schedule, FP32, n <= 4096): the n-point
// azimuth lines of range cells 0 .. cols-1, read from in [n][pitch] (the range
// pass's output), transformed (fused: IFFT(FFT * H); else FFT * scale) and
// stored as lines out [cols][n].  cols must be a multiple of the strip width
// min(16, 1024 / (n / 16)).
hipError_t launch_line_strip(bool fused, int n, const void* in, void* out, int cols, int pitch,
                             const void* H, const void* tw, float scale, int variant, hipStream_t s);

// Batched launches (kind: 0 fused, 1 forward, 2 inverse; tasks in device memory).
//  variant bits 0 (twiddles) and 2-3 (grid: one workgroup per line group, or
//  a persistent grid of 1x, 2x, 4x the resident workgroups)
hipError_t launch_line_batch(int kind, int n, const void* tasks, int ntasks, int total_groups,
                             float scale, int prec, int variant, hipStream_t s);

// Autotuned kernel variants, per (kernel kind, line length, precision).  The
// table starts empty (every variant 0) and is filled by sar_autotune or from a
// JSON-lines cache named by SAR_AUTOTUNE_CACHE when the first plan is built.
// TK_TURN is keyed by the turned matrix's row length (precision FP32), TK_STRIP
// by the azimuth line length (FP32).
enum TuneKind { TK_FUSED = 0, TK_FWD = 1, TK_INV = 2, TK_RCMC = 3, TK_BATCH_FUSED = 4, TK_TURN = 5,
                TK_STRIP = 6 };
int tuned_variant(int kind, int n, int prec);
void load_tune_cache_once();

// Half storage (FP32 arithmetic, FP16 intermediates with a power-of-two
// scale per line; see k_line_hs):
//  RangeFused:     complex64 lines -> FP16 lines, ex_out[line] exponents
//  AzimuthFused:   FP16 lines (point j scaled by 2^ex_in[j]) -> complex64
//  AzimuthForward: FP16 lines (as above) -> FFT -> FP16 lines + ex_out
enum class HalfOp { RangeFused, AzimuthFused, AzimuthForward };
hipError_t launch_line_half(HalfOp op, int n, const void* in, void* out, int lines, const void* H,
                            const void* tw, const int* ex_in, int* ex_out, hipStream_t s);
// Two-row RCMC + azimuth from FP16 range-Doppler rows (row r scaled by
// 2^ex[r]) into complex64 (requires taps == 8, stretch_max < 0.5, even nr).
hipError_t launch_rcmc_half(int n, const void* A, const int* ex, void* out, const RcmcHost& rh,
                            const void* tw, hipStream_t s);
// Corner turn of 4-byte elements (FP16 pairs); rows, cols multiples of 64.
hipError_t launch_corner_turn_b4(const void* in, void* out, int rows, int cols, hipStream_t s);

hipError_t launch_corner_turn_batch(const void* tasks, int ntasks, int total_tiles, hipStream_t s);
int line_groups(int n, int lines);        // line groups of `lines` lines of length n

// Device tables of a plan (for the batch runtime).
struct PlanTables {
    const void* Hr;
    const void* Ha;
    const void* tw_r;
    const void* tw_a;
};
PlanTables plan_tables(const sar_plan_s* P);
RcmcHost plan_rcmc(const sar_plan_s* P);   // hyperbolic plans only
int turn_tiles(int rows, int cols);       // 64 x 64 tiles of a corner turn

hipError_t launch_rowmul(const void* in, void* out, int rows, int n, const void* H, hipStream_t s);
hipError_t launch_corner_turn(const void* in, void* out, int rows, int cols, int variant,
                              hipStream_t s);
hipError_t launch_rcmc_interp(const void* A, void* out, int na, const RcmcHost& rh, hipStream_t s);
hipError_t launch_az_phase(const void* in, void* out, int na, const RcmcHost& rh, float scale,
                           hipStream_t s);

hipError_t launch_gen_twiddles(void* tw, int n, hipStream_t s);
hipError_t launch_gen_chirp_filter(void* H, int n, int len, double K, int sign, double scale,
                                   hipStream_t s);
hipError_t launch_gen_rcmc_table(float* tab, double beta, hipStream_t s);
int rcmc_table_floats();
hipError_t launch_gen_hyper_tables(double* stretch, double* rate, int na, double lam, double v,
                                   hipStream_t s);

}  // namespace sar

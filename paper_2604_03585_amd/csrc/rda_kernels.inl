// rda_kernels.inl -- gfx950 kernels of the Range Doppler Algorithm and their
// launchers.  Compiled in four parts (rda_part_*.hip, SAR_PART = 0..3) so that
// the template instantiations build in parallel: part 0 holds the table
// generators, the non-line kernels and the dispatcher, parts 1-3 the line
// and RCMC kernels for FP32, split-FP16 and split-BF16 butterflies.  Every kernel is written for wave64 CDNA4; lines are kept in
// registers (16 complex64 per thread) and LDS between radix passes.
//
// Kernels (paper: arXiv 2604.03585):
//   k_gen_*          FP64 plan-time tables (twiddles, matched filters with
//                    the IFFT's 1/N folded in, hyperbolic per-bin tables).
//   k_line_fused     FFT -> x H -> IFFT per line, one HBM read and one write
//                    (Sec. II.B; range compression and LFM azimuth
//                    compression, Sec. IV.A steps 1 and 4).
//   k_line_fft       FFT or IFFT only (azimuth FFT of Sec. IV.A step 2; the
//                    first/last dispatch of the unfused comparator, Fig. 1).
//   k_rowmul         the unfused comparator's separate filter multiply.
//   k_corner_turn    LDS-tiled [rows][cols] -> [cols][rows] transpose
//                    (Sec. IV.B).
//   k_rcmc_az        RCMC (8-tap Kaiser-sinc) + exact-geometry azimuth phase
//                    + IFFT per output range line, fused (Sec. IV.A steps 3-4).
//   k_rcmc_interp,   the same two steps as separate dispatches for the
//   k_az_phase       unfused comparator.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft_line.hpp"
#include "mfma_fft.hpp"
#include "rda_internal.h"

// Every kernel launch of the library.  When sar_time_next_launch has armed
// two events on this thread, the launch records them at the kernel's start
// and end (hipExtLaunchKernel takes the dispatch's own timestamps, so the
// interval is the kernel's duration alone).
#define SAR_LAUNCH(kernel, grid, block, lds, stream, ...)                                  \
    do {                                                                                   \
        hipEvent_t sar_e0_, sar_e1_;                                                       \
        if (sar::take_launch_events(sar_e0_, sar_e1_))                                     \
            hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, sar_e0_, sar_e1_, 0,   \
                                  __VA_ARGS__);                                            \
        else                                                                               \
            hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);             \
    } while (0)

namespace sar {

#if SAR_PART == 0
// ===================================================== FP64 generators
// exp(-2 pi i * num / den) in FP64, num reduced exactly mod den first.
__device__ __forceinline__ float2 twiddle_fp64(long long num, long long den)
{
    long long r = num % den;
    double s, c;
    sincospi(-2.0 * (double)r / (double)den, &s, &c);
    return make_float2((float)c, (float)s);
}

// Per-N Stockham twiddle table (layout in fft_line.hpp, LineGeom::tw_off),
// for radix-E passes followed by one smaller pass.
__global__ void k_gen_twiddles(float2* __restrict__ tw, int n, int e_pts)
{
    int log = 0, rlog = 0;
    while ((1 << log) < n) ++log;
    while ((1 << rlog) < e_pts) ++rlog;
    const int nfull = log / rlog, rem = 1 << (log % rlog);
    const int np = nfull + (rem > 1 ? 1 : 0);
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int off = 0, ns = 1;
    for (int p = 0; p < np; ++p) {
        const int R = p < nfull ? e_pts : rem;
        if (p >= 1) {
            const int cnt = (R - 1) * ns;
            if (e >= off && e < off + cnt) {
                const int i = (e - off) / ns + 1, jm = (e - off) % ns;
                tw[e] = twiddle_fp64((long long)jm * i, (long long)ns * R);
                return;
            }
            off += cnt;
        }
        ns *= R;
    }
}

// Matched filter H[k] = scale * conj( sum_u exp(j*(sign*pi*K*u^2 - 2*pi*k*u/N)) ),
// u = -L/2 .. L-L/2-1: the DFT of the circularly centred chirp replica,
// evaluated directly (O(N*L)) in FP64 with every phase reduced to turns.
__global__ void k_gen_chirp_filter(float2* __restrict__ H, int n, int len, double K,
                                   int sign, double scale)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double re = 0.0, im = 0.0;
    const int u0 = -(len / 2), u1 = len - len / 2;
    for (int u = u0; u < u1; ++u) {
        // phase in turns: sign*K*u^2/2 - k*u/n
        double a = (double)sign * 0.5 * K * (double)u * (double)u;
        a -= a >= 0.0 ? floor(a) : -floor(-a);       // exact-ish fraction, |a| < 1
        long long ku = ((long long)k * (long long)u) % n;
        double b = a - (double)ku / (double)n;
        double s, c;
        sincospi(2.0 * b, &s, &c);
        re += c;
        im += s;
    }
    H[k] = make_float2((float)(re * scale), (float)(-im * scale));
}


#endif  // SAR_PART == 0

// ===================================================== line kernels
// FP16 storage of intermediates (the half-storage precision mode): a
// complex sample as two _Float16, with a power-of-two scale per line.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 h2_to_f2(h2_t v, float scale)
{
    return make_float2((float)v.x * scale, (float)v.y * scale);
}
// X: a multiple of the default lines per workgroup (the autotuner's 2x
// candidate of the FP32 line kernels).
template <int N, int X = 1> struct LineLaunch {
    static constexpr int T = LineGeom<N>::T;
    static constexpr int LPW = (T >= 256 ? 1 : 256 / T) * X;   // lines per workgroup
    static constexpr int BLOCK = LPW * T;
    // Register policy of the fused FFT*H*IFFT kernels (measured on gfx950):
    // the inverse transform reuses the forward pass's twiddle products when
    // the compiler can prove the addresses equal, which saves VALU work but
    // keeps them live across the multiply.  For N = 4096 that reuse pays once
    // the kernel is held to 128 VGPRs (4 waves per SIMD, as many workgroups
    // as LDS allows; see line_wpe); for N >= 8192 it spills, so the inverse
    // recomputes them.
    static constexpr bool RECOMPUTE_INV_TW = N >= 8192;
    static constexpr int LDS_BYTES = LPW * LineGeom<N>::LDS * (int)sizeof(float2);
};

// Minimum waves per SIMD requested for the line kernels: 4 for the FP32
// 4096-point kernels (register reuse above); 2 for the split-precision
// (MFMA) kernels (left to itself the fused 4096-point one takes 268 VGPRs,
// one wave per SIMD); no request otherwise.
template <int N, int PREC> constexpr int line_wpe()
{
    if constexpr (PREC == 0) return N == 4096 ? 4 : 1;
    else return 2;     // four waves (128 VGPRs) spill in the split transforms, measured slower
}

// Line transform in the requested butterfly precision: FP32 VALU passes, or
// split FP16 / BF16 radix-16 passes on MFMA (twiddles and filters in FP32).
template <int N, bool INV, int PREC, bool TWP = true, bool SPLIT = false, class F = NoOp,
          bool AHEAD = false>
__device__ __forceinline__ void fft_any(float2 (&x)[line_e(N)], float2* __restrict__ lds,
                                        const float2* __restrict__ tw, int sub, int t,
                                        F&& before_last = F())
{
    if constexpr (PREC == PREC_FP32 && AHEAD) {
        fft_line_ahead<N, INV, TWP, SPLIT>(x, lds, tw, t, before_last);
    } else if constexpr (PREC == PREC_FP32) {
        fft_line<N, INV, TWP, SPLIT>(x, lds, tw, t, before_last);
    } else {
        using L = LineLaunch<N>;
        fft_line_mfma<N, INV, PREC, L::LPW, L::BLOCK>(x, lds - sub * LineGeom<N>::LDS, tw, sub,
                                                      t, before_last);
    }
}

// XCD-aware line order: gfx950 hands workgroup b to XCD (b mod 8); giving each
// XCD a contiguous run of line groups keeps neighbouring lines in one L2.
__device__ __forceinline__ int xcd_group(int b, int groups)
{
    if ((groups & 7) != 0) return b;
    return (b & 7) * (groups >> 3) + (b >> 3);
}

template <int N>
__device__ __forceinline__ void load_line(float2 (&x)[line_e(N)], const float2* __restrict__ src,
                                          int t)
{
#pragma unroll
    for (int m = 0; m < line_e(N); ++m) x[m] = src[t + m * LineGeom<N>::T];
}

template <int N>
__device__ __forceinline__ void store_line(const float2 (&x)[line_e(N)], float2* __restrict__ dst,
                                           int t)
{
#pragma unroll
    for (int m = 0; m < line_e(N); ++m) dst[t + m * LineGeom<N>::T] = x[m];
}

// One workgroup per group of LPW lines.
enum LineKind { LK_FUSED = 0, LK_FWD = 1, LK_INV = 2 };

//  LK_FUSED: out = IFFT(FFT(in) * H)      (H carries the 1/N)
//  LK_FWD:   out = FFT(in) * scale;  LK_INV: out = IFFT_unscaled(in) * scale
// One group of LPW lines starting at line g * LPW of `in` / `out`.  TWP:
// twiddles by products (true) or straight table reads (false), chosen per
// line length by the autotuner; SPLIT (FP32 forward / inverse): the split
// real/imaginary exchange layout.
// The transform of one line held by its T threads (thread t: points t + m*T)
// with `lds` its exchange buffer: FFT * H * IFFT, FFT or IFFT (see line_group).
template <int N, int KIND, int PREC, bool TWP, bool SPLIT = false>
__device__ __forceinline__ void line_transform(float2 (&x)[line_e(N)], float2* __restrict__ lds,
                                               const float2* __restrict__ H,
                                               const float2* __restrict__ tw, float scale,
                                               int sub, int t)
{
    using L = LineLaunch<N>;
    constexpr int E = line_e(N);
    if constexpr (KIND == LK_FUSED) {
        // the filter is requested just before the last forward pass.  Lines
        // of 8192 points and more (one or two workgroups per CU) read their
        // twiddles one pass ahead in both transforms, 4096-point lines in the
        // forward one (in the inverse too they spill), shorter ones not at
        // all (registers)
        constexpr bool AHEAD = N >= 8192;
        constexpr bool AHEAD_FWD = AHEAD || N == 4096;
        float2 h[E];
        auto filter = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m) h[m] = H[t + m * L::T];
        };
        fft_any<N, false, PREC, TWP, false, decltype(filter)&, AHEAD_FWD>(x, lds, tw, sub, t, filter);
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = c_mul(x[m], h[m]);
        int ti = t;
        if constexpr (L::RECOMPUTE_INV_TW) asm volatile("" : "+v"(ti));   // hide ti == t
        fft_any<N, true, PREC, TWP, false, NoOp, AHEAD>(x, lds, tw, sub, ti);
    } else {
        fft_any<N, KIND == LK_INV, PREC, TWP, SPLIT, NoOp, true>(x, lds, tw, sub, t);
        if (scale != 1.0f) {
#pragma unroll
            for (int m = 0; m < E; ++m) x[m] = c_scale(x[m], scale);
        }
    }
}

template <int N, int KIND, int PREC, bool TWP, bool SPLIT = false, int X = 1>
__device__ __forceinline__ void line_group(const float2* in, float2* out, int lines,
                                           const float2* __restrict__ H,
                                           const float2* __restrict__ tw, float scale, int g,
                                           float2* smem)
{
    using L = LineLaunch<N, X>;
    constexpr int E = line_e(N);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int line = g * L::LPW + sub;
    const bool live = line < lines;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    float2 x[E];
    if (live) load_line<N>(x, in + (size_t)line * N, t);
    else {
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = make_float2(0.f, 0.f);
    }
    line_transform<N, KIND, PREC, TWP, SPLIT>(x, lds, H, tw, scale, sub, t);
    if (live) store_line<N>(x, out + (size_t)line * N, t);
}

// ---------------------------------------------------------- column strips
// Turn-free schedule: the azimuth lines of a strip of C adjacent range cells
// read straight from the range pass's [Na][Nr] output, so no corner turn is
// needed.  Each row of the strip is C consecutive samples (C * 8 bytes: 32 B
// at 4096 points, 64 B at 2048, 128 B at 1024 and below); the workgroup
// reads the C x N strip with consecutive lanes on consecutive sample pairs,
// regroups it through LDS into one line per slot of T = N/16 threads, runs
// the same line transform as k_line (so the results are bit-identical to
// the turned path) and stores each line contiguously: out is [Nr][Na].
// C = min(16, 1024 / T) lines per workgroup (N <= 4096: 136 KiB of LDS), or
// CW lines (the autotuner's half-width candidate).
template <int N, int CW = 0> struct StripLaunch {
    static constexpr int T = LineGeom<N>::T;
    static constexpr int C_DEFAULT = (1024 / T) < 16 ? 1024 / T : 16;
    static constexpr int C = CW ? CW : C_DEFAULT;
    static constexpr int BLOCK = C * T;
    // line buffers 16 float2 more than a line's exchange buffer apart, so
    // the C samples of one row (consecutive lanes) fall into different banks
    static constexpr int STRIDE = LineGeom<N>::LDS + 16;
    static constexpr int LDS_BYTES = C * STRIDE * (int)sizeof(float2);
    static_assert(N <= 4096 && C >= 2 && C <= C_DEFAULT, "strips of two lines or more");
};

template <int N, int KIND, bool TWP, int CW = 0>
__global__ __launch_bounds__((StripLaunch<N, CW>::BLOCK)) void
k_line_strip(const float2* __restrict__ in, float2* __restrict__ out, int cols, int pitch,
             const float2* __restrict__ H, const float2* __restrict__ tw, float scale)
{
    using S = StripLaunch<N, CW>;
    constexpr int T = S::T, C = S::C, E = line_e(N);
    static_assert(S::BLOCK * E == C * N, "one sample per thread and pass");
    extern __shared__ __align__(16) float2 smem[];
    const int g = xcd_group(blockIdx.x, cols / C);
    const int n0 = g * C;
    const int u = threadIdx.x;
    // 16-byte loads: lanes take pairs of adjacent columns, C / 2 lanes per
    // row (fewer, wider requests for the same short runs)
    static_assert(C % 2 == 0, "pairs of columns");
#pragma unroll
    for (int p = 0; p < E / 2; ++p) {
        const int e = u + p * S::BLOCK;           // pair (row m, columns 2q, 2q+1) of the strip
        const int m = e / (C / 2), q = e % (C / 2);
        const float4 v = *(const float4*)(in + (size_t)m * pitch + n0 + 2 * q);
        smem[(2 * q) * S::STRIDE + lds_pad(m)] = make_float2(v.x, v.y);
        smem[(2 * q + 1) * S::STRIDE + lds_pad(m)] = make_float2(v.z, v.w);
    }
    __syncthreads();
    const int sub = u / T, t = u % T;
    float2* lds = smem + sub * S::STRIDE;
    float2 x[E];
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = lds[lds_pad(t + m * T)];
    __syncthreads();                              // reads done before the exchanges
    line_transform<N, KIND, PREC_FP32, TWP>(x, lds, H, tw, scale, sub, t);
    store_line<N>(x, out + (size_t)(n0 + sub) * N, t);
}

template <int N, int KIND, int PREC, bool TWP, bool SPLIT = false, int X = 1>
__global__ __launch_bounds__((LineLaunch<N, X>::BLOCK))
__attribute__((amdgpu_waves_per_eu(line_wpe<N, PREC>()))) void
k_line(const float2* in, float2* out, int lines, const float2* __restrict__ H,
       const float2* __restrict__ tw, float scale)
{
    static_assert(!SPLIT || (PREC == PREC_FP32 && KIND != LK_FUSED), "split layout: FP32 FFT only");
    static_assert(X == 1 || PREC == PREC_FP32, "more lines per workgroup: FP32 butterflies only");
    extern __shared__ __align__(16) float2 smem[];
    line_group<N, KIND, PREC, TWP, SPLIT, X>(in, out, lines, H, tw, scale, blockIdx.x, smem);
}

// Batched form: the line groups of many scenes (tasks) in one launch.  The
// grid covers min(total groups, resident capacity) workgroups, each walking
// groups gg = blockIdx.x, + gridDim.x, ...; the task of a group is found by
// binary search over the tasks' first-group indices (sorted).
// The task owning line group gg (tasks sorted by group_begin; uniform).
__device__ __forceinline__ const LineTask& find_task(const LineTask* __restrict__ tasks, int ntasks,
                                                      int gg)
{
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].group_begin <= gg) lo = mid;
        else hi = mid - 1;
    }
    return tasks[lo];
}

// PERSIST: a grid smaller than the work loops over line groups; otherwise
// one workgroup per line group (no loop, so nothing is hoisted across
// groups and the register footprint equals k_line's).
template <int N, int KIND, int PREC, bool TWP, bool PERSIST>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK)
__attribute__((amdgpu_waves_per_eu(line_wpe<N, PREC>()))) void
k_line_batch(const LineTask* __restrict__ tasks, int ntasks, int total_groups, float scale)
{
    extern __shared__ __align__(16) float2 smem[];
    if constexpr (!PERSIST) {
        const LineTask& tk = find_task(tasks, ntasks, blockIdx.x);
        line_group<N, KIND, PREC, TWP>(tk.in, tk.out, tk.lines, tk.H, tk.tw, scale,
                                       blockIdx.x - tk.group_begin, smem);
    } else {
        for (int gg = blockIdx.x; gg < total_groups; gg += gridDim.x) {
            const LineTask tk = find_task(tasks, ntasks, gg);
            line_group<N, KIND, PREC, TWP>(tk.in, tk.out, tk.lines, tk.H, tk.tw, scale,
                                           gg - tk.group_begin, smem);
            __syncthreads();                      // LDS reuse by the next group
        }
    }
}

#if SAR_PART == 0
// out[r][k] = in[r][k] * H[k]  (unfused comparator's multiply dispatch)
__global__ __launch_bounds__(256) void k_rowmul(const float4* in, float4* out, long long n_pairs,
                                                int n, const float2* __restrict__ H)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n_pairs; p += stride) {
        float4 a = in[p];
        const int k = (int)((2 * p) & (n - 1));
        const float2 h0 = H[k], h1 = H[k + 1];
        const float2 r0 = c_mul(make_float2(a.x, a.y), h0);
        const float2 r1 = c_mul(make_float2(a.z, a.w), h1);
        out[p] = make_float4(r0.x, r0.y, r1.x, r1.y);
    }
}

// ===================================================== corner turn
// 64 x 64 complex64 tiles through LDS (one pad column against bank
// conflicts); reads and writes are 512-byte contiguous row segments.
constexpr int TT = 64;
__global__ __launch_bounds__(256) void k_corner_turn(const float2* __restrict__ in,
                                                     float2* __restrict__ out, int rows, int cols)
{
    __shared__ float2 tile[TT][TT + 1];
    const int tiles_c = (cols + TT - 1) / TT;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
    const int r0 = tr * TT, c0 = tc * TT;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < TT / 4; ++i) {
        const int r = ty + 4 * i;
        if (r0 + r < rows && c0 + tx < cols)
            tile[r][tx] = in[(size_t)(r0 + r) * cols + c0 + tx];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TT / 4; ++i) {
        const int c = ty + 4 * i;
        if (c0 + c < cols && r0 + tx < rows)
            out[(size_t)(c0 + c) * rows + r0 + tx] = tile[tx][c];
    }
}

// Batched corner turn: the 64 x 64 tiles of many matrices in one launch.
// Whole 64 x 64 tiles only (rows and cols multiples of 64): every global
// access moves 16 bytes (two complex samples), half the instructions of
// k_corner_turn.
// LDS map: element (r, c) of the tile sits at column c ^ ((r >> 1) & 31) of
// row r (no pad).  A bank holds 4 bytes and 64 banks span 32 samples, so a
// sample's banks depend on its column mod 32.  The read phase has lane tx
// take rows 2tx and 2tx+1 at one column c: the swizzle gives the 32 lanes
// 32 different columns mod 32 (with a pad the even rows share 16), and the
// 32 KiB tile lets five workgroups share a CU's LDS instead of four.
__device__ __forceinline__ int turn_swz(int r, int c) { return c ^ ((r >> 1) & 31); }

// Tiles gt = blockIdx.x, + gridDim.x, ... (the launcher keeps gridDim.x <=
// tiles): the next tile's loads are issued before the current tile leaves
// LDS, so they overlap its stores; its LDS writes wait for those loads only
// (vector-memory operations complete in issue order, the stores came after).
// `more` is uniform per workgroup.
__device__ __forceinline__ void turn_tile_to_lds(float2 (*tile)[TT], const float4 (&v)[TT / 8], int tx,
                                                 int ty)
{
#pragma unroll
    for (int i = 0; i < TT / 8; ++i) {
        const int r = ty + 8 * i;
        tile[r][turn_swz(r, 2 * tx)] = make_float2(v[i].x, v[i].y);
        tile[r][turn_swz(r, 2 * tx + 1)] = make_float2(v[i].z, v[i].w);
    }
}

__global__ __launch_bounds__(256) void k_corner_turn_x2(const float4* __restrict__ in,
                                                        float4* __restrict__ out, int rows,
                                                        int cols, int tiles)
{
    __shared__ float2 tile[TT][TT];
    const int tiles_c = cols / TT;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int cols2 = cols / 2, rows2 = rows / 2;
    int gt = blockIdx.x;
    float4 v[TT / 8];
    {
        const int r0 = (gt / tiles_c) * TT, c0 = (gt % tiles_c) * TT;
#pragma unroll
        for (int i = 0; i < TT / 8; ++i) v[i] = in[(size_t)(r0 + ty + 8 * i) * cols2 + c0 / 2 + tx];
    }
    turn_tile_to_lds(tile, v, tx, ty);
    wg_barrier();
    for (;;) {
        const int r0 = (gt / tiles_c) * TT, c0 = (gt % tiles_c) * TT;
        const int next = gt + (int)gridDim.x;
        const bool more = next < tiles;
        if (more) {
            const int nr0 = (next / tiles_c) * TT, nc0 = (next % tiles_c) * TT;
#pragma unroll
            for (int i = 0; i < TT / 8; ++i)
                v[i] = in[(size_t)(nr0 + ty + 8 * i) * cols2 + nc0 / 2 + tx];
        }
#pragma unroll
        for (int i = 0; i < TT / 8; ++i) {
            const int c = ty + 8 * i;
            const float2 a = tile[2 * tx][turn_swz(2 * tx, c)], b = tile[2 * tx + 1][turn_swz(2 * tx + 1, c)];
            out[(size_t)(c0 + c) * rows2 + r0 / 2 + tx] = make_float4(a.x, a.y, b.x, b.y);
        }
        if (!more) break;
        wg_barrier();                             // every read done before the next writes
        turn_tile_to_lds(tile, v, tx, ty);
        wg_barrier();
        gt = next;
    }
}

// k_corner_turn_x2 for 4-byte elements (FP16 pairs): whole 64 x 64 tiles,
// every global access moves two elements (8 bytes).
__global__ __launch_bounds__(256) void k_corner_turn_b4(const uint2* __restrict__ in,
                                                        uint2* __restrict__ out, int rows, int cols)
{
    __shared__ uint32_t tile[TT][TT + 1];
    const int tiles_c = cols / TT;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
    const int r0 = tr * TT, c0 = tc * TT;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int cols2 = cols / 2, rows2 = rows / 2;
#pragma unroll
    for (int i = 0; i < TT / 8; ++i) {
        const int r = ty + 8 * i;
        const uint2 v = in[(size_t)(r0 + r) * cols2 + c0 / 2 + tx];
        tile[r][2 * tx] = v.x;
        tile[r][2 * tx + 1] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TT / 8; ++i) {
        const int c = ty + 8 * i;
        out[(size_t)(c0 + c) * rows2 + r0 / 2 + tx] = make_uint2(tile[2 * tx][c], tile[2 * tx + 1][c]);
    }
}

__global__ __launch_bounds__(256) void k_corner_turn_batch(const TurnTask* __restrict__ tasks,
                                                           int ntasks, int total_tiles)
{
    // every task is whole 64 x 64 tiles (plan sizes are powers of two >= 64);
    // the tile's LDS map is k_corner_turn_x2's
    __shared__ float2 tile[TT][TT];
    for (int gt = blockIdx.x; gt < total_tiles; gt += gridDim.x) {
        int lo = 0, hi = ntasks - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].tile_begin <= gt) lo = mid;
            else hi = mid - 1;
        }
        const TurnTask tk = tasks[lo];
        const int b = gt - tk.tile_begin;
        const int tiles_c = tk.cols / TT;
        const int r0 = (b / tiles_c) * TT, c0 = (b % tiles_c) * TT;
        const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
        const float4* in = (const float4*)tk.in;
        float4* out = (float4*)tk.out;
        const int cols2 = tk.cols / 2, rows2 = tk.rows / 2;
#pragma unroll
        for (int i = 0; i < TT / 8; ++i) {
            const int r = ty + 8 * i;
            const float4 v = in[(size_t)(r0 + r) * cols2 + c0 / 2 + tx];
            tile[r][turn_swz(r, 2 * tx)] = make_float2(v.x, v.y);
            tile[r][turn_swz(r, 2 * tx + 1)] = make_float2(v.z, v.w);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TT / 8; ++i) {
            const int c = ty + 8 * i;
            const float2 a = tile[2 * tx][turn_swz(2 * tx, c)];
            const float2 bb = tile[2 * tx + 1][turn_swz(2 * tx + 1, c)];
            out[(size_t)(c0 + c) * rows2 + r0 / 2 + tx] = make_float4(a.x, a.y, bb.x, bb.y);
        }
        __syncthreads();
    }
}

#endif  // SAR_PART == 0

// ===================================================== RCMC
// The 8-tap Kaiser-windowed sinc (taps t = -3..4 about floor(p), x = p -
// floor(p), weights normalised to unit sum) depends on x alone.  Its eight
// weight functions w_t(x) are smooth on [0, 1), so the plan stores them as
// piecewise quadratics: RCMC_INTERVALS intervals, on each a degree-2
// Chebyshev interpolant of the exact FP64 weights, in monomial form in the
// local variable u = x * RCMC_INTERVALS - b in [0, 1].  Layout (interval-
// major, 24 floats = 96 bytes per interval, read as six 16-byte vectors):
//     tab[b * 24 + t * 3 + j] = coefficient of u^j, tap t.
// The interpolation error is 2.2e-8 in FP64 (below the FP32 rounding of the
// coefficients; tested against the oracle's weights); the kernels copy the
// 12 KiB table into LDS (14 KiB there, see RCMC_LDS_STRIDE).
constexpr int RCMC_INTERVALS = 128;
constexpr int RCMC_PER_INTERVAL = 24;
constexpr int RCMC_TAB = RCMC_INTERVALS * RCMC_PER_INTERVAL;
// The LDS copy places the intervals 7 vectors (28 floats) apart: the lanes of
// a wave read random intervals, and with an odd stride in 16-byte units the
// same vector of different intervals falls into every bank group, where a
// stride of 6 reaches only half of them (twice the bank conflicts).  The
// seventh vector of each interval is padding and never read.
constexpr int RCMC_LDS_STRIDE = 28;
constexpr int RCMC_LDS_FLOATS = RCMC_INTERVALS * RCMC_LDS_STRIDE;

#if SAR_PART == 0
__device__ double i0_fp64(double y)
{
    const double q = 0.25 * y * y;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// Exact normalised weights at x (FP64): K(z) = sinc(z) I0(beta sqrt(1-(z/4)^2)).
__device__ void kaiser_weights_fp64(double x, double beta, double* w)
{
    double sum = 0.0;
    for (int i = 0; i < 8; ++i) {
        const double z = (double)(i - 3) - x;
        const double r = z / 4.0;
        const double sc = (z == 0.0) ? 1.0 : sinpi(z) / (3.14159265358979323846 * z);
        const double arg = 1.0 - r * r;
        w[i] = (arg > 0.0 ? sc * i0_fp64(beta * sqrt(arg)) : 0.0);
        sum += w[i];
    }
    for (int i = 0; i < 8; ++i) w[i] /= sum;
}

// One thread per interval b: three Chebyshev nodes, exact weights, 3x3
// solve per tap for the monomial coefficients in u.
__global__ void k_gen_rcmc_table(float* __restrict__ tab, double beta)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= RCMC_INTERVALS) return;
    double u[3], w[3][8];
    for (int j = 0; j < 3; ++j) {
        u[j] = 0.5 * (1.0 + cospi((2.0 * j + 1.0) / 6.0));
        kaiser_weights_fp64(((double)b + u[j]) / RCMC_INTERVALS, beta, w[j]);
    }
    for (int t = 0; t < 8; ++t) {
        double M[3][4];
        for (int j = 0; j < 3; ++j) {
            M[j][0] = 1.0;
            M[j][1] = u[j];
            M[j][2] = u[j] * u[j];
            M[j][3] = w[j][t];
        }
        for (int c = 0; c < 3; ++c) {             // Gaussian elimination, partial pivot
            int piv = c;
            for (int r = c + 1; r < 3; ++r)
                if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
            for (int q = 0; q < 4; ++q) { double tmp = M[c][q]; M[c][q] = M[piv][q]; M[piv][q] = tmp; }
            for (int r = c + 1; r < 3; ++r) {
                const double f = M[r][c] / M[c][c];
                for (int q = c; q < 4; ++q) M[r][q] -= f * M[c][q];
            }
        }
        double cf[3];
        for (int c = 2; c >= 0; --c) {
            double acc = M[c][3];
            for (int q = c + 1; q < 3; ++q) acc -= M[c][q] * cf[q];
            cf[c] = acc / M[c][c];
        }
        for (int j = 0; j < 3; ++j) tab[b * RCMC_PER_INTERVAL + t * 3 + j] = (float)cf[j];
    }
}

#endif  // SAR_PART == 0

struct RcmcArgs {
    const double* stretch;   // 1/D_k - 1 per Doppler bin
    const double* rate;      // 2 D_k / lambda per Doppler bin
    const float* table;      // RCMC_TAB weight coefficients (global)
    double r_near;
    double stretch_max;      // max_k stretch_k (|f| = 1/2)
    double x_per_bin;        // lambda / (2 v Na): x_k = signed bin * x_per_bin
    double two_over_lam;     // 2 / lambda
    int nr;
    const int* row_exp;      // half storage: per-row exponents of the FP16 input
};

// The per-bin geometry from the bin index: f_k in fftfreq order,
// x = lambda f / (2 v), D = sqrt(1 - x^2), stretch = 1/D - 1, rate = 2 D / lambda.
// r = 1/D comes from the hardware reciprocal square root refined by two
// Newton steps in FP64 (quadratic convergence: full double precision), so
// stretch = r - 1 has an absolute error near 1e-16; the RCMC shift
// R0 * stretch needs it to 1e-12.  The plan's tables use the same function.
__device__ __forceinline__ void bin_geometry_x(double x, double two_over_lam, double& stretch,
                                               double& rate)
{
    const double a = fma(-x, x, 1.0);               // D^2
    double r = __builtin_amdgcn_rsq(a);
    const double ha = 0.5 * a;
#pragma unroll
    for (int i = 0; i < 2; ++i) r = r * fma(-ha * r, r, 1.5);
    stretch = r - 1.0;
    rate = (a * r) * two_over_lam;                  // D = a / sqrt(a)
}

__device__ __forceinline__ void bin_geometry(const RcmcArgs& ra, int k, int na, double& stretch,
                                             double& rate)
{
    const int kk = k < na / 2 ? k : k - na;
    bin_geometry_x((double)kk * ra.x_per_bin, ra.two_over_lam, stretch, rate);
}

#if SAR_PART == 0
// Hyperbolic per-Doppler-bin tables (the unfused and one-row kernels read
// them; the two-row kernel computes the same values in place):
// stretch = 1/D - 1, rate = 2 D / lambda (azimuth phase in turns per cell).
__global__ void k_gen_hyper_tables(double* __restrict__ stretch, double* __restrict__ rate,
                                   int na, double x_per_bin, double two_over_lam)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    const int kk = k < na / 2 ? k : k - na;
    bin_geometry_x((double)kk * x_per_bin, two_over_lam, stretch[k], rate[k]);
}
#endif

// Global table (24 floats per interval) -> LDS (RCMC_LDS_STRIDE floats per
// interval); lds_tab holds RCMC_LDS_FLOATS floats.
__device__ __forceinline__ void load_rcmc_table(float* __restrict__ lds_tab,
                                                const float* __restrict__ tab, int tid, int nthreads)
{
    static_assert(RCMC_PER_INTERVAL == 24 && RCMC_LDS_STRIDE % 4 == 0, "16-byte copies");
    constexpr int V = RCMC_PER_INTERVAL / 4, VS = RCMC_LDS_STRIDE / 4;
    for (int i = tid; i < RCMC_TAB / 4; i += nthreads)
        ((float4*)lds_tab)[(i / V) * VS + i % V] = ((const float4*)tab)[i];
}

// sum_t w_t(x) a_t with the weights from the LDS table.
__device__ __forceinline__ float2 rcmc_combine(float x, const float* __restrict__ tab,
                                               const float2 (&a)[8])
{
    const float xf = x * (float)RCMC_INTERVALS;
    const int b = min((int)xf, RCMC_INTERVALS - 1);
    const float u = xf - (float)b;
    const float4* p = (const float4*)(tab + b * RCMC_LDS_STRIDE);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {                 // taps 4h .. 4h+3: three vectors
        float c[12];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float4 v = p[3 * h + i];
            c[4 * i] = v.x;
            c[4 * i + 1] = v.y;
            c[4 * i + 2] = v.z;
            c[4 * i + 3] = v.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = 4 * h + q;
            const float w = fmaf(fmaf(c[3 * q + 2], u, c[3 * q + 1]), u, c[3 * q]);
            acc.x = fmaf(w, a[t].x, acc.x);
            acc.y = fmaf(w, a[t].y, acc.y);
        }
    }
    return acc;
}

__device__ __forceinline__ float2 ld_off(const float2* __restrict__ base, uint32_t byte_off)
{
    return *(const float2*)((const char*)base + byte_off);
}

// RCMC output y[n][k] from range-Doppler A[Nr][Na]:
//   R0 = r_near + n, s = R0 * stretch_k, i0 = n + floor(s), x = frac(s),
//   y = sum_t w_t(x) A[i0 + t][k] over t = -3..4 (rows outside [0, Nr) add 0).
// `interior` promises that every tap row is inside the scene (checked by
// the caller per line), which removes the per-tap bounds tests.
__device__ __forceinline__ void rcmc_shift(double R0, int n, double stretch, float& x, int& i0)
{
    const double s = R0 * stretch;
    const double fl = floor(s);
    x = (float)(s - fl);
    // shifts beyond +-2^30 cells read nothing but stay defined integers
    i0 = n + (int)fmax(-1073741824.0, fmin(fl, 1073741824.0));
}

__device__ __forceinline__ float2 rcmc_gather(const float2* __restrict__ A, int na, int nr, int k,
                                              float x, int i0, const float* __restrict__ tab,
                                              bool interior)
{
    float2 a[8];
    if (interior) {
        const uint32_t step = (uint32_t)na * 8u;
        uint32_t off = ((uint32_t)(i0 - 3) * (uint32_t)na + (uint32_t)k) * 8u;
#pragma unroll
        for (int i = 0; i < 8; ++i, off += step) a[i] = ld_off(A, off);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int r = i0 + i - 3;
            a[i] = (r >= 0 && r < nr) ? A[(size_t)r * na + k] : make_float2(0.f, 0.f);
        }
    }
    return rcmc_combine(x, tab, a);
}

template <int TAPS>
__device__ __forceinline__ float2 rcmc_value(const float2* __restrict__ A, int na, int n, int k,
                                             const RcmcArgs& ra, const float* __restrict__ tab,
                                             bool interior)
{
    if constexpr (TAPS == 0) {
        return ld_off(A, ((uint32_t)n * (uint32_t)na + (uint32_t)k) * 8u);
    } else {
        float x;
        int i0;
        rcmc_shift(ra.r_near + (double)n, n, ra.stretch[k], x, i0);
        return rcmc_gather(A, na, ra.nr, k, x, i0, tab, interior);
    }
}

// exp(+j 2 pi frac(R0 * rate)) * scale: the phase in turns is reduced in
// FP64, then the hardware sine/cosine (argument in turns, max abs error
// 1.3e-7 on [-1/2, 1/2], measured on gfx950) evaluate it.
__device__ __forceinline__ float2 turns_to_phasor(double ph, float scale)
{
    float f = (float)(ph - floor(ph));
    if (f > 0.5f) f -= 1.0f;
    return make_float2(__builtin_amdgcn_cosf(f) * scale, __builtin_amdgcn_sinf(f) * scale);
}

__device__ __forceinline__ float2 az_phase_of(double R0, double rate, float scale)
{
    return turns_to_phasor(R0 * rate, scale);
}

__device__ __forceinline__ float2 az_phase(const RcmcArgs& ra, int n, int k, float scale)
{
    return az_phase_of(ra.r_near + (double)n, ra.rate[k], scale);
}

// Every tap row of output line n lies inside [0, Nr).
__device__ __forceinline__ bool rcmc_interior(const RcmcArgs& ra, int n)
{
    const double smax = (ra.r_near + (double)n) * ra.stretch_max;
    return n >= 3 && (double)n + smax + 6.0 <= (double)(ra.nr - 1);
}

// Samples y[m] = RCMC(n, k_m) * phase_m for the 16 columns k_m = t + m*T
// of one thread, all tap rows inside the scene.  The eight gathers of
// column m+1 are in flight while column m is combined (vector-memory loads
// complete in order, so the wait for column m leaves m+1's loads pending).
// The eight tap samples A[i0 - 3 + i][k].  EDGE: rows outside [0, nr) are
// read at a clamped (valid) row and replaced by zero, without branches.
template <int N, bool EDGE>
__device__ __forceinline__ void rcmc_gather8(float2 (&a)[8], const float2* __restrict__ A, int k,
                                             int i0, int nr)
{
    if constexpr (!EDGE) {
        constexpr uint32_t step = (uint32_t)N * 8u;
        uint32_t off = ((uint32_t)(i0 - 3) * (uint32_t)N + (uint32_t)k) * 8u;
#pragma unroll
        for (int i = 0; i < 8; ++i, off += step) a[i] = ld_off(A, off);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int r = i0 - 3 + i;
            const int rc = min(max(r, 0), nr - 1);
            const float2 v = ld_off(A, ((uint32_t)rc * (uint32_t)N + (uint32_t)k) * 8u);
            const bool in = (r >= 0) & (r < nr);
            a[i] = make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
        }
    }
}

// Samples y[m] = RCMC(n, k_m) * phase_m for the 16 columns k_m = t + m*T
// of one thread.  The gathers of column m+1 are in flight while column m is
// combined (vector-memory loads complete in order, so waiting for column m
// leaves m+1's loads pending); sched_barrier(0) keeps the scheduler from
// hoisting every gather to the top, which would need ~256 registers.
template <int N, bool EDGE>
__device__ __forceinline__ void rcmc_row(float2 (&x)[line_e(N)], const float2* __restrict__ A, int t,
                                         int nr, const float (&xs)[line_e(N)], const int (&i0s)[line_e(N)],
                                         const float2 (&ph)[line_e(N)], const float* __restrict__ tab)
{
    constexpr int T = LineGeom<N>::T;
    constexpr int E = line_e(N);
    float2 a0[8], a1[8];
    rcmc_gather8<N, EDGE>(a0, A, t, i0s[0], nr);
#pragma unroll
    for (int m = 0; m < E; m += 2) {
        rcmc_gather8<N, EDGE>(a1, A, t + (m + 1) * T, i0s[m + 1], nr);
        __builtin_amdgcn_sched_barrier(0);
        x[m] = c_mul(rcmc_combine(xs[m], tab, a0), ph[m]);
        __builtin_amdgcn_sched_barrier(0);
        if (m + 2 < E) rcmc_gather8<N, EDGE>(a0, A, t + (m + 2) * T, i0s[m + 2], nr);
        __builtin_amdgcn_sched_barrier(0);
        x[m + 1] = c_mul(rcmc_combine(xs[m + 1], tab, a1), ph[m + 1]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int N, int TAPS, int PREC>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK) void
k_rcmc_az(const float2* __restrict__ A, float2* __restrict__ out, RcmcArgs ra,
               const float2* __restrict__ tw)
{
    using L = LineLaunch<N>;
    constexpr int E = line_e(N);
    extern __shared__ __align__(16) float2 smem[];
    // The weight table and the line buffers share LDS: the table is only read
    // while the RCMC samples are formed, before the first FFT exchange.
    float* tab = (float*)smem;
    static_assert(L::LDS_BYTES >= RCMC_LDS_FLOATS * (int)sizeof(float), "table fits the line LDS");
    const int lines = ra.nr;
    const int groups = (lines + L::LPW - 1) / L::LPW;
    const int g = xcd_group(blockIdx.x, groups);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int n = g * L::LPW + sub;
    const bool live = n < lines;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    constexpr float scale = 1.0f / (float)N;
    const double R0 = ra.r_near + (double)n;

    // per-Doppler-bin quantities first: their loads overlap the table copy
    float xs[E];
    int i0s[E];
    float2 ph[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * L::T;
        ph[m] = az_phase_of(R0, ra.rate[k], scale);
        if constexpr (TAPS != 0) rcmc_shift(R0, n, ra.stretch[k], xs[m], i0s[m]);
    }
    if constexpr (TAPS != 0) {
        load_rcmc_table(tab, ra.table, threadIdx.x, L::BLOCK);
        __syncthreads();
    }
    float2 x[E];
    if (!live) {
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = make_float2(0.f, 0.f);
    } else if constexpr (TAPS == 0) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            x[m] = c_mul(ld_off(A, ((uint32_t)n * (uint32_t)N + (uint32_t)(t + m * L::T)) * 8u), ph[m]);
    } else if (rcmc_interior(ra, n)) {
        rcmc_row<N, false>(x, A, t, ra.nr, xs, i0s, ph, tab);
    } else {
        rcmc_row<N, true>(x, A, t, ra.nr, xs, i0s, ph, tab);
    }
    if constexpr (TAPS != 0) __syncthreads();     // table reads done before LDS reuse
    fft_any<N, true, PREC>(x, lds, tw, sub, t);
    if (live) store_line<N>(x, out + (size_t)n * N, t);
}

// Two output rows n, n+1 per line slot.  For each column their 8-tap
// windows start at i0(n) - 3 and i0(n+1) - 3 with i0(n+1) - i0(n) = 1 + d,
// d in {0, 1} (requires stretch < 1), so ten rows i0(n) - 3 .. i0(n) + 6
// cover both: 10 gathers for 2 samples instead of 16.  The per-bin
// geometry is computed, not loaded, so the gathers of the next column can be
// issued before the current column is combined without a load-to-load chain.
// Range-Doppler rows stored as FP16 pairs, row r scaled by 2^-ex[r].
struct HalfRows {
    const h2_t* a;
    const int* ex;
};

template <int N, bool EDGE>
__device__ __forceinline__ void rcmc_gather10(float2 (&w)[10], const HalfRows& A, int k, int i0,
                                              int nr)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const int r = i0 - 3 + i;
        const int rc = EDGE ? min(max(r, 0), nr - 1) : r;
        const h2_t v = *(const h2_t*)((const char*)A.a + ((uint32_t)rc * (uint32_t)N + (uint32_t)k) * 4u);
        const float2 f = h2_to_f2(v, ldexpf(1.0f, A.ex[rc]));
        const bool in = !EDGE || ((r >= 0) & (r < nr));
        w[i] = make_float2(in ? f.x : 0.f, in ? f.y : 0.f);
    }
}

template <int N, bool EDGE>
__device__ __forceinline__ void rcmc_gather10(float2 (&w)[10], const float2* __restrict__ A,
                                              int k, int i0, int nr)
{
    if constexpr (!EDGE) {
        constexpr uint32_t step = (uint32_t)N * 8u;
        uint32_t off = ((uint32_t)(i0 - 3) * (uint32_t)N + (uint32_t)k) * 8u;
#pragma unroll
        for (int i = 0; i < 10; ++i, off += step) w[i] = ld_off(A, off);
    } else {
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            const int r = i0 - 3 + i;
            const int rc = min(max(r, 0), nr - 1);
            const float2 v = ld_off(A, ((uint32_t)rc * (uint32_t)N + (uint32_t)k) * 8u);
            const bool in = (r >= 0) & (r < nr);
            w[i] = make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
        }
    }
}

struct ColPair {
    float xa, xb;        // fractional positions for rows n, n+1
    int i0;              // i0(n)
    bool d;              // i0(n+1) - i0(n) == 2
    float2 pa, pb;       // azimuth phases (with 1/Na) for rows n, n+1
};

// Row n+1 continues row n: its shift is s + stretch and its phase (turns)
// ph + rate, both in FP64 (the same values as R0 * stretch and R0 * rate
// with R0 = r_near + n + 1, up to one rounding).
__device__ __forceinline__ ColPair col_pair(const RcmcArgs& ra, int n, int k, int na, float scale)
{
    double stretch, rate;
    bin_geometry(ra, k, na, stretch, rate);
    const double R0 = ra.r_near + (double)n;
    ColPair c;
    const double sa = R0 * stretch, sb = sa + stretch;
    const double fa = floor(sa), fb = floor(sb);
    c.xa = (float)(sa - fa);
    c.xb = (float)(sb - fb);
    // shifts beyond +-2^30 cells read nothing but stay defined integers
    c.i0 = n + (int)fmax(-1073741824.0, fmin(fa, 1073741824.0));
    c.d = (fb - fa) != 0.0;                       // i0(n+1) - i0(n) == 2
    const double pa = R0 * rate;
    c.pa = turns_to_phasor(pa, scale);
    c.pb = turns_to_phasor(pa + rate, scale);
    return c;
}

template <int N, bool EDGE>
__device__ __forceinline__ void rcmc_pair_combine(float2& ya, float2& yb, const ColPair& c,
                                                  const float2 (&w)[10],
                                                  const float* __restrict__ tab)
{
    float2 ta[8], tb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        ta[i] = w[i];
        tb[i] = c.d ? w[i + 2] : w[i + 1];
    }
    ya = c_mul(rcmc_combine(c.xa, tab, ta), c.pa);
    yb = c_mul(rcmc_combine(c.xb, tab, tb), c.pb);
}

// Columns t + m * S (m < C) of rows n, n+1 of A (FP32 rows, or HalfRows).
template <int N, bool EDGE, int C = line_e(N), int S = LineGeom<N>::T, class Src = const float2*>
__device__ __forceinline__ void rcmc_rows2(float2 (&xa)[C], float2 (&xb)[C], Src A,
                                           const RcmcArgs& ra, int n, int t,
                                           const float* __restrict__ tab)
{
    constexpr int T = S;
    constexpr int E = C;
    static_assert(E % 2 == 0, "columns are processed in pairs");
    constexpr float scale = 1.0f / (float)N;
    // two named buffers, alternated by column parity (no register copies)
    ColPair c0 = col_pair(ra, n, t, N, scale), c1;
    float2 w0[10], w1[10];
    rcmc_gather10<N, EDGE>(w0, A, t, c0.i0, ra.nr);
#pragma unroll
    for (int m = 0; m < E; m += 2) {
        c1 = col_pair(ra, n, t + (m + 1) * T, N, scale);
        rcmc_gather10<N, EDGE>(w1, A, t + (m + 1) * T, c1.i0, ra.nr);
        __builtin_amdgcn_sched_barrier(0);
        rcmc_pair_combine<N, EDGE>(xa[m], xb[m], c0, w0, tab);
        __builtin_amdgcn_sched_barrier(0);
        if (m + 2 < E) {
            c0 = col_pair(ra, n, t + (m + 2) * T, N, scale);
            rcmc_gather10<N, EDGE>(w0, A, t + (m + 2) * T, c0.i0, ra.nr);
        }
        __builtin_amdgcn_sched_barrier(0);
        rcmc_pair_combine<N, EDGE>(xa[m + 1], xb[m + 1], c1, w1, tab);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// HIN: A holds FP16 rows with per-row exponents ra.row_exp (half storage).
template <int N, int PREC, bool HIN = false>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK) void
k_rcmc_az2(const void* __restrict__ A_, float2* __restrict__ out, RcmcArgs ra,
           const float2* __restrict__ tw)
{
    using SrcT = typename std::conditional<HIN, HalfRows, const float2*>::type;
    SrcT A;
    if constexpr (HIN) A = HalfRows{(const h2_t*)A_, ra.row_exp};
    else A = (const float2*)A_;
    using L = LineLaunch<N>;
    constexpr int E = line_e(N);
    extern __shared__ __align__(16) float2 smem[];
    float* tab = (float*)smem;                    // shares LDS with the line buffers
    static_assert(L::LDS_BYTES >= RCMC_LDS_FLOATS * (int)sizeof(float), "table fits the line LDS");
    const int pairs = ra.nr / 2;
    const int groups = (pairs + L::LPW - 1) / L::LPW;
    const int g = xcd_group(blockIdx.x, groups);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int pr = g * L::LPW + sub;
    const bool live = pr < pairs;
    const int n = 2 * pr;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    load_rcmc_table(tab, ra.table, threadIdx.x, L::BLOCK);
    __syncthreads();
    float2 xa[E], xb[E];
    if (!live) {
#pragma unroll
        for (int m = 0; m < E; ++m) xa[m] = xb[m] = make_float2(0.f, 0.f);
    } else {
        const double smax = (ra.r_near + (double)n + 1.0) * ra.stretch_max;
        if (n >= 3 && (double)n + 1.0 + smax + 6.0 <= (double)(ra.nr - 1))
            rcmc_rows2<N, false, line_e(N), LineGeom<N>::T, SrcT>(xa, xb, A, ra, n, t, tab);
        else
            rcmc_rows2<N, true, line_e(N), LineGeom<N>::T, SrcT>(xa, xb, A, ra, n, t, tab);
    }
    __syncthreads();                              // table reads done before LDS reuse
    fft_any<N, true, PREC, true, false, NoOp, true>(xa, lds, tw, sub, t);
    if (live) store_line<N>(xa, out + (size_t)n * N, t);
    fft_any<N, true, PREC, true, false, NoOp, true>(xb, lds, tw, sub, t);
    if (live) store_line<N>(xb, out + (size_t)(n + 1) * N, t);
}

// The same two rows per workgroup on 2T threads (FP32, T = N/16 <= 512):
// the interpolation is spread over all 2T threads (E/2 columns each, half
// the accumulator registers of k_rcmc_az2), the two rows then meet in LDS
// and their IFFTs run side by side, one per half of the workgroup.  LDS:
// two line buffers (the weight table shares the first).
template <int N>
__global__ __launch_bounds__(2 * LineGeom<N>::T) void
k_rcmc_az2w(const float2* __restrict__ A, float2* __restrict__ out, RcmcArgs ra,
            const float2* __restrict__ tw)
{
    using G = LineGeom<N>;
    constexpr int T = G::T, E = line_e(N), C = E / 2, S = 2 * T;
    static_assert(S <= 1024, "two line slots per workgroup");
    extern __shared__ __align__(16) float2 smem[];
    float* tab = (float*)smem;
    static_assert(2 * G::LDS * (int)sizeof(float2) >= RCMC_LDS_FLOATS * (int)sizeof(float),
                  "table fits the two line buffers");
    const int pairs = ra.nr / 2;
    const int pr = xcd_group(blockIdx.x, pairs);
    const int n = 2 * pr;
    const int u = threadIdx.x;
    load_rcmc_table(tab, ra.table, u, S);
    __syncthreads();
    float2 ya[C], yb[C];
    const double smax = (ra.r_near + (double)n + 1.0) * ra.stretch_max;
    if (n >= 3 && (double)n + 1.0 + smax + 6.0 <= (double)(ra.nr - 1))
        rcmc_rows2<N, false, C, S>(ya, yb, A, ra, n, u, tab);
    else
        rcmc_rows2<N, true, C, S>(ya, yb, A, ra, n, u, tab);
    __syncthreads();                              // table reads done before LDS reuse
    float2* row_a = smem;
    float2* row_b = smem + G::LDS;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        row_a[lds_pad(u + m * S)] = ya[m];
        row_b[lds_pad(u + m * S)] = yb[m];
    }
    __syncthreads();
    const int sub = u / T, t = u % T;
    float2* lds = smem + sub * G::LDS;
    float2 x[E];
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = lds[lds_pad(t + m * T)];
    __syncthreads();                              // reads done before the IFFT writes
    fft_line<N, true>(x, lds, tw, t);
    store_line<N>(x, out + (size_t)(n + sub) * N, t);
}

#if SAR_PART == 0
// Unfused comparator: RCMC interpolation alone (grid-stride, one sample per
// thread per iteration).
template <int TAPS>
__global__ __launch_bounds__(256) void k_rcmc_interp(const float2* __restrict__ A,
                                                     float2* __restrict__ out, int na, RcmcArgs ra)
{
    __shared__ __align__(16) float tab[RCMC_LDS_FLOATS];
    if constexpr (TAPS != 0) {
        load_rcmc_table(tab, ra.table, threadIdx.x, 256);
        __syncthreads();
    }
    const long long total = (long long)ra.nr * na;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int n = (int)(e / na), k = (int)(e % na);
        out[e] = rcmc_value<TAPS>(A, na, n, k, ra, tab, false);
    }
}

// Unfused comparator: azimuth phase multiply exp(+j 2 pi frac(R0 rate_k)) * scale.
__global__ __launch_bounds__(256) void k_az_phase(const float2* __restrict__ in,
                                                  float2* __restrict__ out, int na, RcmcArgs ra,
                                                  float scale)
{
    const long long total = (long long)ra.nr * na;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int n = (int)(e / na), k = (int)(e % na);
        out[e] = c_mul(in[e], az_phase(ra, n, k, scale));
    }
}

#endif  // SAR_PART == 0

#if SAR_PART == 1
// ===================================================== half storage (FP32 math)
// Largest |re|, |im| of one line's samples (the line's T threads: aligned
// lane segments of a wave when T < 64, else whole waves combined through
// `scratch`, 16 floats of LDS that no thread still reads).
template <int N>
__device__ __forceinline__ float line_absmax(const float2 (&x)[line_e(N)], float* scratch, int sub)
{
    using L = LineLaunch<N>;
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < line_e(N); ++i) m = fmaxf(m, fmaxf(fabsf(x[i].x), fabsf(x[i].y)));
    constexpr int W = L::T < 64 ? L::T : 64;
#pragma unroll
    for (int off = 1; off < W; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    if constexpr (L::T > 64) {
        constexpr int WPL = L::T / 64;            // waves per line
        static_assert(L::BLOCK / 64 <= 16, "scratch holds one float per wave");
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0) scratch[wave] = m;
        __syncthreads();
        m = 0.f;
#pragma unroll
        for (int w = 0; w < WPL; ++w) m = fmaxf(m, scratch[sub * WPL + w]);
    }
    return m;
}

// Exponent e of a line whose largest component is amax: the stored values
// x * 2^-e have their largest component in [2^14, 2^15) (FP16 holds up to
// 65504); empty, non-finite or all-zero lines keep e = 0.
__device__ __forceinline__ int half_exponent(float amax)
{
    if (!(amax > 0.f) || !(amax < INFINITY)) return 0;
    return max(ilogbf(amax) - 14, -100);
}

// FP32 line transform with FP16 storage on either side.
//  IN_H:  `in` holds lines of FP16 pairs; point j of every line carries the
//         scale 2^ex_in[j] (the exponent of the range line the point came
//         from, after the corner turn);
//  OUT_H: `out` receives FP16 pairs x * 2^-e, e = ex_out[line] chosen per
//         line by half_exponent; else `out` is complex64.
template <int N, int KIND, bool IN_H, bool OUT_H>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK)
__attribute__((amdgpu_waves_per_eu(line_wpe<N, PREC_FP32>()))) void
k_line_hs(const void* __restrict__ in, void* __restrict__ out, int lines,
          const float2* __restrict__ H, const float2* __restrict__ tw,
          const int* __restrict__ ex_in, int* __restrict__ ex_out)
{
    using L = LineLaunch<N>;
    constexpr int E = line_e(N);
    extern __shared__ __align__(16) float2 smem[];
    const int groups = (lines + L::LPW - 1) / L::LPW;
    const int g = xcd_group(blockIdx.x, groups);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int line = g * L::LPW + sub;
    const bool live = line < lines;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    float2 x[E];
    if (live) {
        if constexpr (IN_H) {
            const h2_t* src = (const h2_t*)in + (size_t)line * N;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int j = t + m * L::T;
                x[m] = h2_to_f2(src[j], ldexpf(1.0f, ex_in[j]));
            }
        } else {
            load_line<N>(x, (const float2*)in + (size_t)line * N, t);
        }
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = make_float2(0.f, 0.f);
    }
    // twiddle reads one pass ahead where registers allow, as in line_group
    // (fused: forward from 4096 points, inverse from 8192)
    if constexpr (KIND == LK_FUSED) {
        float2 h[E];
        auto filter = [&] {
#pragma unroll
            for (int m = 0; m < E; ++m) h[m] = H[t + m * L::T];
        };
        if constexpr (N >= 4096) fft_line_ahead<N, false>(x, lds, tw, t, filter);
        else fft_line<N, false>(x, lds, tw, t, filter);
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = c_mul(x[m], h[m]);
        int ti = t;
        if constexpr (L::RECOMPUTE_INV_TW) asm volatile("" : "+v"(ti));
        if constexpr (N >= 8192) fft_line_ahead<N, true>(x, lds, tw, ti);
        else fft_line<N, true>(x, lds, tw, ti);
    } else {
        static_assert(KIND == LK_FWD, "fused or forward");
        fft_line_ahead<N, false>(x, lds, tw, t);
    }
    if constexpr (OUT_H) {
        const int e = half_exponent(line_absmax<N>(x, (float*)smem, sub));
        const float sc = ldexpf(1.0f, -e);
        if (live) {
            h2_t* dst = (h2_t*)out + (size_t)line * N;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                h2_t v;
                v.x = (_Float16)(x[m].x * sc);
                v.y = (_Float16)(x[m].y * sc);
                dst[t + m * L::T] = v;
            }
            if (t == 0) ex_out[line] = e;
        }
    } else if (live) {
        store_line<N>(x, (float2*)out + (size_t)line * N, t);
    }
}
#endif  // SAR_PART == 1

// ===================================================== launchers
static RcmcArgs make_rcmc_args(const RcmcHost& rh)
{
    RcmcArgs ra{};
    ra.stretch = rh.stretch;
    ra.rate = rh.rate;
    ra.table = rh.table;
    ra.r_near = rh.r_near;
    ra.stretch_max = rh.stretch_max;
    ra.x_per_bin = rh.x_per_bin;
    ra.two_over_lam = rh.two_over_lam;
    ra.nr = rh.nr;
    return ra;
}

[[maybe_unused]] static int grid_for(long long work, int per_block)
{
    long long g = (work + per_block - 1) / per_block;
    const long long cap = 256LL * 64;   // grid-stride kernels: 64 workgroups per CU
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

template <int N, int PREC>
static hipError_t set_lds_limit()
{
    using L = LineLaunch<N>;
    if (L::LDS_BYTES <= 64 * 1024) return hipSuccess;
    const void* fns[] = {(const void*)k_line<N, LK_FUSED, PREC, true>,
                         (const void*)k_line<N, LK_FWD, PREC, true>,
                         (const void*)k_line<N, LK_INV, PREC, true>,
                         (const void*)k_line<N, LK_FUSED, PREC, false>,
                         (const void*)k_line<N, LK_FWD, PREC, false>,
                         (const void*)k_line<N, LK_INV, PREC, false>,
                         (const void*)k_rcmc_az<N, 0, PREC>, (const void*)k_rcmc_az<N, 8, PREC>,
                         (const void*)k_rcmc_az2<N, PREC>,
                         (const void*)k_line_batch<N, LK_FUSED, PREC, true, true>,
                         (const void*)k_line_batch<N, LK_FWD, PREC, true, true>,
                         (const void*)k_line_batch<N, LK_INV, PREC, true, true>,
                         (const void*)k_line_batch<N, LK_FUSED, PREC, false, true>,
                         (const void*)k_line_batch<N, LK_FWD, PREC, false, true>,
                         (const void*)k_line_batch<N, LK_INV, PREC, false, true>,
                         (const void*)k_line_batch<N, LK_FUSED, PREC, true, false>,
                         (const void*)k_line_batch<N, LK_FWD, PREC, true, false>,
                         (const void*)k_line_batch<N, LK_INV, PREC, true, false>,
                         (const void*)k_line_batch<N, LK_FUSED, PREC, false, false>,
                         (const void*)k_line_batch<N, LK_FWD, PREC, false, false>,
                         (const void*)k_line_batch<N, LK_INV, PREC, false, false>};
    for (const void* f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
        if (e != hipSuccess) return e;
    }
    if constexpr (PREC == PREC_FP32) {
        const void* split[] = {(const void*)k_line<N, LK_FWD, PREC, true, true>,
                               (const void*)k_line<N, LK_FWD, PREC, false, true>,
                               (const void*)k_line<N, LK_INV, PREC, true, true>,
                               (const void*)k_line<N, LK_INV, PREC, false, true>};
        for (const void* f : split) {
            const hipError_t e =
                hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// FP32 line kernel with X times the default lines per workgroup.
template <int N, int KIND, bool TWP, bool SPLIT, int X>
static hipError_t launch_k_line_x(const float2* in, float2* out, int lines, const float2* H,
                                  const float2* tw, float scale, hipStream_t s)
{
    using L = LineLaunch<N, X>;
    static const hipError_t attr =
        L::LDS_BYTES <= 64 * 1024
            ? hipSuccess
            : hipFuncSetAttribute((const void*)k_line<N, KIND, PREC_FP32, TWP, SPLIT, X>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
    if (attr != hipSuccess) return attr;
    const int groups = (lines + L::LPW - 1) / L::LPW;
    if (groups == 0) return hipSuccess;
    SAR_LAUNCH((k_line<N, KIND, PREC_FP32, TWP, SPLIT, X>), dim3(groups), dim3(L::BLOCK),
               L::LDS_BYTES, s, in, out, lines, H, tw, scale);
    return hipGetLastError();
}

template <int N, int KIND, int PREC>
static hipError_t launch_k_line(const float2* in, float2* out, int lines, const float2* H,
                                const float2* tw, float scale, int variant, hipStream_t s)
{
    using L = LineLaunch<N>;
    const int groups = (lines + L::LPW - 1) / L::LPW;
    if (groups == 0) return hipSuccess;
    // variant bit 0: twiddles from the table (FP32 butterflies only); bit 1
    // (FP32 forward / inverse): the split real/imaginary exchange layout;
    // bit 2 (FP32, N <= 8192): twice the lines per workgroup
    if constexpr (PREC == PREC_FP32 && N <= 8192) {
        if (variant & 4) {
            const bool tab = variant & 1;
            if constexpr (KIND != LK_FUSED) {
                if (variant & 2)
                    return tab ? launch_k_line_x<N, KIND, false, true, 2>(in, out, lines, H, tw, scale, s)
                               : launch_k_line_x<N, KIND, true, true, 2>(in, out, lines, H, tw, scale, s);
            }
            return tab ? launch_k_line_x<N, KIND, false, false, 2>(in, out, lines, H, tw, scale, s)
                       : launch_k_line_x<N, KIND, true, false, 2>(in, out, lines, H, tw, scale, s);
        }
    }
    if constexpr (PREC == PREC_FP32 && KIND != LK_FUSED) {
        if (variant & 2) {
            if (variant & 1)
                SAR_LAUNCH((k_line<N, KIND, PREC, false, true>), dim3(groups), dim3(L::BLOCK),
                                   L::LDS_BYTES, s, in, out, lines, H, tw, scale);
            else
                SAR_LAUNCH((k_line<N, KIND, PREC, true, true>), dim3(groups), dim3(L::BLOCK),
                                   L::LDS_BYTES, s, in, out, lines, H, tw, scale);
            return hipGetLastError();
        }
    }
    if (PREC == PREC_FP32 && (variant & 1))
        SAR_LAUNCH((k_line<N, KIND, PREC, false>), dim3(groups), dim3(L::BLOCK),
                           L::LDS_BYTES, s, in, out, lines, H, tw, scale);
    else
        SAR_LAUNCH((k_line<N, KIND, PREC, true>), dim3(groups), dim3(L::BLOCK),
                           L::LDS_BYTES, s, in, out, lines, H, tw, scale);
    return hipGetLastError();
}

template <int N, int PREC>
static hipError_t launch_line_n(LineOp op, const float2* in, float2* out, int lines,
                                const float2* H, const float2* tw, float scale,
                                const RcmcArgs* ra, int taps, int variant, hipStream_t s)
{
    using L = LineLaunch<N>;
    static const hipError_t attr = set_lds_limit<N, PREC>();
    if (attr != hipSuccess) return attr;
    switch (op) {
    case LineOp::Fused:
        return launch_k_line<N, LK_FUSED, PREC>(in, out, lines, H, tw, 1.0f, variant, s);
    case LineOp::Forward:
        return launch_k_line<N, LK_FWD, PREC>(in, out, lines, nullptr, tw, scale, variant, s);
    case LineOp::Inverse:
        return launch_k_line<N, LK_INV, PREC>(in, out, lines, nullptr, tw, scale, variant, s);
    case LineOp::RcmcAz: {
        const int groups = (lines + L::LPW - 1) / L::LPW;
        if (groups == 0) return hipSuccess;
        static_assert(L::LDS_BYTES >= RCMC_LDS_FLOATS * (int)sizeof(float), "table fits the line LDS");
        // variant bit 1: one output row per line slot instead of two; bit 2
        // (FP32, N = 4096 or 8192): the two rows on two line slots' threads
        // (k_rcmc_az2w) instead of one's
        const bool two_rows = taps == 8 && ra->stretch_max < 0.5 && (lines & 1) == 0 && !(variant & 2);
        if constexpr (PREC == PREC_FP32 && (N == 4096 || N == 8192)) {
            if (two_rows && (variant & 4)) {
                constexpr int lds2 = 2 * LineGeom<N>::LDS * (int)sizeof(float2);
                static const hipError_t wa =
                    lds2 <= 64 * 1024 ? hipSuccess
                                      : hipFuncSetAttribute((const void*)k_rcmc_az2w<N>,
                                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                                            lds2);
                if (wa != hipSuccess) return wa;
                SAR_LAUNCH((k_rcmc_az2w<N>), dim3(lines / 2), dim3(2 * LineGeom<N>::T), lds2,
                                   s, in, out, *ra, tw);
                return hipGetLastError();
            }
        }
        if (two_rows) {
            const int g2 = (lines / 2 + L::LPW - 1) / L::LPW;
            SAR_LAUNCH((k_rcmc_az2<N, PREC>), dim3(g2), dim3(L::BLOCK), L::LDS_BYTES, s, in,
                               out, *ra, tw);
        } else if (taps == 8)
            SAR_LAUNCH((k_rcmc_az<N, 8, PREC>), dim3(groups), dim3(L::BLOCK), L::LDS_BYTES,
                               s, in, out, *ra, tw);
        else
            SAR_LAUNCH((k_rcmc_az<N, 0, PREC>), dim3(groups), dim3(L::BLOCK), L::LDS_BYTES,
                               s, in, out, *ra, tw);
        return hipGetLastError();
    }
    }
    return hipErrorInvalidValue;
}

template <int N, int PREC, bool TWP, bool PERSIST>
static void launch_line_batch_k(int kind, int grid, const LineTask* tasks, int ntasks,
                                int total_groups, float scale, hipStream_t s)
{
    using L = LineLaunch<N>;
    switch (kind) {
    case LK_FUSED:
        SAR_LAUNCH((k_line_batch<N, LK_FUSED, PREC, TWP, PERSIST>), dim3(grid),
                           dim3(L::BLOCK), L::LDS_BYTES, s, tasks, ntasks, total_groups, scale);
        break;
    case LK_FWD:
        SAR_LAUNCH((k_line_batch<N, LK_FWD, PREC, TWP, PERSIST>), dim3(grid),
                           dim3(L::BLOCK), L::LDS_BYTES, s, tasks, ntasks, total_groups, scale);
        break;
    default:
        SAR_LAUNCH((k_line_batch<N, LK_INV, PREC, TWP, PERSIST>), dim3(grid),
                           dim3(L::BLOCK), L::LDS_BYTES, s, tasks, ntasks, total_groups, scale);
        break;
    }
}

template <int N, int PREC, bool TWP>
static hipError_t launch_line_batch_t(int kind, const LineTask* tasks, int ntasks, int total_groups,
                                      float scale, int grid_sel, hipStream_t s)
{
    using L = LineLaunch<N>;
    static const hipError_t attr = set_lds_limit<N, PREC>();
    if (attr != hipSuccess) return attr;
    if (total_groups == 0) return hipSuccess;
    // grid_sel 0: one workgroup per line group; 1, 2, 3: a persistent grid of
    // 1x, 2x, 4x the resident workgroups (LDS-limited per CU x 256 CUs)
    if ((grid_sel & 3) == 0) {
        launch_line_batch_k<N, PREC, TWP, false>(kind, total_groups, tasks, ntasks, total_groups,
                                                 scale, s);
        return hipGetLastError();
    }
    const int per_cu = (160 * 1024) / L::LDS_BYTES;
    const int resident = (per_cu < 1 ? 1 : per_cu) * 256;
    const int cap = resident << ((grid_sel & 3) - 1);
    const int grid = total_groups < cap ? total_groups : cap;
    launch_line_batch_k<N, PREC, TWP, true>(kind, grid, tasks, ntasks, total_groups, scale, s);
    return hipGetLastError();
}

template <int N, int PREC>
static hipError_t launch_line_batch_n(int kind, const LineTask* tasks, int ntasks, int total_groups,
                                      float scale, int variant, hipStream_t s)
{
    // variant bit 0: table twiddles (FP32); bits 2-3: persistent grid size
    const int grid_sel = (variant >> 2) & 3;
    if (PREC == PREC_FP32 && (variant & 1))
        return launch_line_batch_t<N, PREC, false>(kind, tasks, ntasks, total_groups, scale,
                                                   grid_sel, s);
    return launch_line_batch_t<N, PREC, true>(kind, tasks, ntasks, total_groups, scale, grid_sel, s);
}

template <int PREC>
static hipError_t launch_line_batch_prec(int kind, int n, const LineTask* tasks, int ntasks,
                                         int total_groups, float scale, int v, hipStream_t s)
{
    switch (n) {
    case 64: return launch_line_batch_n<64, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 128: return launch_line_batch_n<128, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 256: return launch_line_batch_n<256, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 512: return launch_line_batch_n<512, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 1024: return launch_line_batch_n<1024, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 2048: return launch_line_batch_n<2048, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 4096: return launch_line_batch_n<4096, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 8192: return launch_line_batch_n<8192, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    case 16384: return launch_line_batch_n<16384, PREC>(kind, tasks, ntasks, total_groups, scale, v, s);
    default: return hipErrorInvalidValue;
    }
}

template <int PREC>
static hipError_t launch_line_prec(LineOp op, int n, const float2* i, float2* o, int lines,
                                   const float2* h, const float2* w, float scale,
                                   const RcmcArgs* ra, int taps, int v, hipStream_t s)
{
    switch (n) {
    case 64: return launch_line_n<64, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 128: return launch_line_n<128, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 256: return launch_line_n<256, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 512: return launch_line_n<512, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 1024: return launch_line_n<1024, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 2048: return launch_line_n<2048, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 4096: return launch_line_n<4096, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 8192: return launch_line_n<8192, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    case 16384: return launch_line_n<16384, PREC>(op, i, o, lines, h, w, scale, ra, taps, v, s);
    default: return hipErrorInvalidValue;
    }
}

// One instantiation of launch_line_prec / launch_line_batch_prec per part
// (defined in parts 1-3).
hipError_t launch_line_batch_p1(int, int, const LineTask*, int, int, float, int, hipStream_t);
hipError_t launch_line_batch_p2(int, int, const LineTask*, int, int, float, int, hipStream_t);
hipError_t launch_line_batch_p3(int, int, const LineTask*, int, int, float, int, hipStream_t);
hipError_t launch_line_fp32(LineOp, int, const float2*, float2*, int, const float2*, const float2*,
                            float, const RcmcArgs*, int, int, hipStream_t);
hipError_t launch_line_f16(LineOp, int, const float2*, float2*, int, const float2*, const float2*,
                           float, const RcmcArgs*, int, int, hipStream_t);
hipError_t launch_line_bf16(LineOp, int, const float2*, float2*, int, const float2*, const float2*,
                            float, const RcmcArgs*, int, int, hipStream_t);

#if SAR_PART >= 1
hipError_t SAR_LINE_BATCH_FN(int kind, int n, const LineTask* tasks, int ntasks, int total_groups,
                             float scale, int v, hipStream_t s)
{
    return launch_line_batch_prec<SAR_PART - 1>(kind, n, tasks, ntasks, total_groups, scale, v, s);
}
#endif

#if SAR_PART == 1
hipError_t launch_line_fp32(LineOp op, int n, const float2* i, float2* o, int lines,
                            const float2* h, const float2* w, float scale, const RcmcArgs* ra,
                            int taps, int v, hipStream_t s)
{
    return launch_line_prec<PREC_FP32>(op, n, i, o, lines, h, w, scale, ra, taps, v, s);
}

template <int N, int KIND, int CW>
static hipError_t launch_strip_k(const float2* in, float2* out, int cols, int pitch,
                                 const float2* H, const float2* tw, float scale, hipStream_t s)
{
    using S = StripLaunch<N, CW>;
    static const hipError_t attr =
        S::LDS_BYTES <= 64 * 1024
            ? hipSuccess
            : hipFuncSetAttribute((const void*)k_line_strip<N, KIND, true, CW>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS_BYTES);
    if (attr != hipSuccess) return attr;
    // whole strips; 16-byte pair loads need an even pitch and an aligned base
    if (cols % S::C != 0 || (pitch & 1) || ((uintptr_t)in & 15u)) return hipErrorInvalidValue;
    if (cols == 0) return hipSuccess;
    SAR_LAUNCH((k_line_strip<N, KIND, true, CW>), dim3(cols / S::C), dim3(S::BLOCK), S::LDS_BYTES,
               s, in, out, cols, pitch, H, tw, scale);
    return hipGetLastError();
}

// Twiddles by products only: the strips' 1024-thread workgroups hold 128
// VGPRs, where the table-twiddle transforms spill.  Variant 1: strips of
// half the default width (C / 2 lines: half the LDS and threads per
// workgroup, runs of C / 2 samples).
template <int N>
static hipError_t launch_strip_n(bool fused, const float2* in, float2* out, int cols, int pitch,
                                 const float2* H, const float2* tw, float scale, int variant,
                                 hipStream_t s)
{
    constexpr int HALF = StripLaunch<N>::C_DEFAULT / 2;
    if (variant == 1) {
        if (fused) return launch_strip_k<N, LK_FUSED, HALF>(in, out, cols, pitch, H, tw, 1.f, s);
        return launch_strip_k<N, LK_FWD, HALF>(in, out, cols, pitch, nullptr, tw, scale, s);
    }
    if (fused) return launch_strip_k<N, LK_FUSED, 0>(in, out, cols, pitch, H, tw, 1.f, s);
    return launch_strip_k<N, LK_FWD, 0>(in, out, cols, pitch, nullptr, tw, scale, s);
}

hipError_t launch_line_strip(bool fused, int n, const void* in, void* out, int cols, int pitch,
                             const void* H, const void* tw, float scale, int variant, hipStream_t s)
{
    auto i = (const float2*)in;
    auto o = (float2*)out;
    auto h = (const float2*)H;
    auto w = (const float2*)tw;
    switch (n) {
    case 64: return launch_strip_n<64>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    case 128: return launch_strip_n<128>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    case 256: return launch_strip_n<256>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    case 512: return launch_strip_n<512>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    case 1024: return launch_strip_n<1024>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    case 2048: return launch_strip_n<2048>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    case 4096: return launch_strip_n<4096>(fused, i, o, cols, pitch, h, w, scale, variant, s);
    default: return hipErrorInvalidValue;
    }
}

template <const void* (*KERNEL)(), int BYTES>
static hipError_t allow_lds()
{
    static const hipError_t e =
        BYTES <= 64 * 1024
            ? hipSuccess
            : hipFuncSetAttribute(KERNEL(), hipFuncAttributeMaxDynamicSharedMemorySize, BYTES);
    return e;
}

template <int N, int KIND, bool IN_H, bool OUT_H>
static const void* hs_kernel() { return (const void*)k_line_hs<N, KIND, IN_H, OUT_H>; }

template <int N, int KIND, bool IN_H, bool OUT_H>
static hipError_t launch_hs_n(const void* in, void* out, int lines, const void* H, const void* tw,
                              const int* ex_in, int* ex_out, hipStream_t s)
{
    using L = LineLaunch<N>;
    const hipError_t attr = allow_lds<hs_kernel<N, KIND, IN_H, OUT_H>, L::LDS_BYTES>();
    if (attr != hipSuccess) return attr;
    const int groups = (lines + L::LPW - 1) / L::LPW;
    if (groups == 0) return hipSuccess;
    SAR_LAUNCH((k_line_hs<N, KIND, IN_H, OUT_H>), dim3(groups), dim3(L::BLOCK),
                       L::LDS_BYTES, s, in, out, lines, (const float2*)H, (const float2*)tw, ex_in,
                       ex_out);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_hs_op(HalfOp op, const void* in, void* out, int lines, const void* H,
                               const void* tw, const int* ex_in, int* ex_out, hipStream_t s)
{
    switch (op) {
    case HalfOp::RangeFused:
        return launch_hs_n<N, LK_FUSED, false, true>(in, out, lines, H, tw, ex_in, ex_out, s);
    case HalfOp::AzimuthFused:
        return launch_hs_n<N, LK_FUSED, true, false>(in, out, lines, H, tw, ex_in, ex_out, s);
    case HalfOp::AzimuthForward:
        return launch_hs_n<N, LK_FWD, true, true>(in, out, lines, H, tw, ex_in, ex_out, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_line_half(HalfOp op, int n, const void* in, void* out, int lines, const void* H,
                            const void* tw, const int* ex_in, int* ex_out, hipStream_t s)
{
    switch (n) {
    case 64: return launch_hs_op<64>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 128: return launch_hs_op<128>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 256: return launch_hs_op<256>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 512: return launch_hs_op<512>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 1024: return launch_hs_op<1024>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 2048: return launch_hs_op<2048>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 4096: return launch_hs_op<4096>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 8192: return launch_hs_op<8192>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    case 16384: return launch_hs_op<16384>(op, in, out, lines, H, tw, ex_in, ex_out, s);
    default: return hipErrorInvalidValue;
    }
}

template <int N>
static const void* rcmc_half_kernel() { return (const void*)k_rcmc_az2<N, PREC_FP32, true>; }

template <int N>
static hipError_t launch_rcmc_half_n(const void* A, const int* ex, void* out, const RcmcArgs& ra0,
                                     const void* tw, hipStream_t s)
{
    using L = LineLaunch<N>;
    const hipError_t attr = allow_lds<rcmc_half_kernel<N>, L::LDS_BYTES>();
    if (attr != hipSuccess) return attr;
    RcmcArgs ra = ra0;
    ra.row_exp = ex;
    const int g2 = (ra.nr / 2 + L::LPW - 1) / L::LPW;
    if (g2 == 0) return hipSuccess;
    SAR_LAUNCH((k_rcmc_az2<N, PREC_FP32, true>), dim3(g2), dim3(L::BLOCK), L::LDS_BYTES, s,
                       A, (float2*)out, ra, (const float2*)tw);
    return hipGetLastError();
}

hipError_t launch_rcmc_half(int n, const void* A, const int* ex, void* out, const RcmcHost& rh,
                            const void* tw, hipStream_t s)
{
    if (rh.taps != 8 || !(rh.stretch_max < 0.5) || (rh.nr & 1)) return hipErrorInvalidValue;
    const RcmcArgs ra = make_rcmc_args(rh);
    switch (n) {
    case 64: return launch_rcmc_half_n<64>(A, ex, out, ra, tw, s);
    case 128: return launch_rcmc_half_n<128>(A, ex, out, ra, tw, s);
    case 256: return launch_rcmc_half_n<256>(A, ex, out, ra, tw, s);
    case 512: return launch_rcmc_half_n<512>(A, ex, out, ra, tw, s);
    case 1024: return launch_rcmc_half_n<1024>(A, ex, out, ra, tw, s);
    case 2048: return launch_rcmc_half_n<2048>(A, ex, out, ra, tw, s);
    case 4096: return launch_rcmc_half_n<4096>(A, ex, out, ra, tw, s);
    case 8192: return launch_rcmc_half_n<8192>(A, ex, out, ra, tw, s);
    case 16384: return launch_rcmc_half_n<16384>(A, ex, out, ra, tw, s);
    default: return hipErrorInvalidValue;
    }
}
#elif SAR_PART == 2
hipError_t launch_line_f16(LineOp op, int n, const float2* i, float2* o, int lines,
                           const float2* h, const float2* w, float scale, const RcmcArgs* ra,
                           int taps, int v, hipStream_t s)
{
    return launch_line_prec<PREC_F16>(op, n, i, o, lines, h, w, scale, ra, taps, v, s);
}
#elif SAR_PART == 3
hipError_t launch_line_bf16(LineOp op, int n, const float2* i, float2* o, int lines,
                            const float2* h, const float2* w, float scale, const RcmcArgs* ra,
                            int taps, int v, hipStream_t s)
{
    return launch_line_prec<PREC_BF16>(op, n, i, o, lines, h, w, scale, ra, taps, v, s);
}
#endif

#if SAR_PART == 0
hipError_t launch_line(LineOp op, int n, const void* in, void* out, int lines, const void* H,
                       const void* tw, float scale, const RcmcHost* rh, int prec, int variant,
                       hipStream_t s)
{
    RcmcArgs ra{};
    int taps = 0;
    if (rh) {
        ra = make_rcmc_args(*rh);
        taps = rh->taps;
    }
    auto i = (const float2*)in;
    auto o = (float2*)out;
    auto h = (const float2*)H;
    auto w = (const float2*)tw;
    switch (prec) {
    case PREC_FP32: return launch_line_fp32(op, n, i, o, lines, h, w, scale, &ra, taps, variant, s);
    case PREC_F16: return launch_line_f16(op, n, i, o, lines, h, w, scale, &ra, taps, variant, s);
    case PREC_BF16: return launch_line_bf16(op, n, i, o, lines, h, w, scale, &ra, taps, variant, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_line_batch(int kind, int n, const void* tasks, int ntasks, int total_groups,
                             float scale, int prec, int variant, hipStream_t s)
{
    const LineTask* t = (const LineTask*)tasks;
    switch (prec) {
    case PREC_FP32: return launch_line_batch_p1(kind, n, t, ntasks, total_groups, scale, variant, s);
    case PREC_F16: return launch_line_batch_p2(kind, n, t, ntasks, total_groups, scale, variant, s);
    case PREC_BF16: return launch_line_batch_p3(kind, n, t, ntasks, total_groups, scale, variant, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_corner_turn_batch(const void* tasks, int ntasks, int total_tiles, hipStream_t s)
{
    if (total_tiles == 0) return hipSuccess;
    const int grid = total_tiles < 256 * 16 ? total_tiles : 256 * 16;
    SAR_LAUNCH(k_corner_turn_batch, dim3(grid), dim3(256), 0, s, (const TurnTask*)tasks,
                       ntasks, total_tiles);
    return hipGetLastError();
}

int line_groups(int n, int lines)
{
    const int T = n / line_e(n);
    const int lpw = T >= 256 ? 1 : 256 / T;
    return (lines + lpw - 1) / lpw;
}

int turn_tiles(int rows, int cols) { return ((rows + TT - 1) / TT) * ((cols + TT - 1) / TT); }

int twiddle_table_size(int n)
{
    switch (n) {
    case 64: return LineGeom<64>::TW_SIZE;
    case 128: return LineGeom<128>::TW_SIZE;
    case 256: return LineGeom<256>::TW_SIZE;
    case 512: return LineGeom<512>::TW_SIZE;
    case 1024: return LineGeom<1024>::TW_SIZE;
    case 2048: return LineGeom<2048>::TW_SIZE;
    case 4096: return LineGeom<4096>::TW_SIZE;
    case 8192: return LineGeom<8192>::TW_SIZE;
    case 16384: return LineGeom<16384>::TW_SIZE;
    default: return -1;
    }
}

hipError_t launch_rowmul(const void* in, void* out, int rows, int n, const void* H, hipStream_t s)
{
    const long long pairs = (long long)rows * n / 2;
    SAR_LAUNCH(k_rowmul, dim3(grid_for(pairs, 256)), dim3(256), 0, s, (const float4*)in,
                       (float4*)out, pairs, n, (const float2*)H);
    return hipGetLastError();
}

hipError_t launch_corner_turn_b4(const void* in, void* out, int rows, int cols, hipStream_t s)
{
    if (rows % TT != 0 || cols % TT != 0 || (((uintptr_t)in | (uintptr_t)out) & 7u) != 0)
        return hipErrorInvalidValue;
    const long long tiles = (long long)(rows / TT) * (cols / TT);
    if (tiles == 0) return hipSuccess;
    SAR_LAUNCH(k_corner_turn_b4, dim3((unsigned)tiles), dim3(256), 0, s, (const uint2*)in,
                       (uint2*)out, rows, cols);
    return hipGetLastError();
}

hipError_t launch_corner_turn(const void* in, void* out, int rows, int cols, int variant,
                              hipStream_t s)
{
    const long long tiles = (long long)((rows + TT - 1) / TT) * ((cols + TT - 1) / TT);
    if (tiles == 0) return hipSuccess;
    const bool whole = rows % TT == 0 && cols % TT == 0 &&
                       (((uintptr_t)in | (uintptr_t)out) & 15u) == 0;
    if (whole) {
        // a grid of at most 1280 workgroups (five per CU, as many as LDS
        // holds), each taking the same number of tiles (the last round
        // ragged); variant 1: at most 1024 (four per CU); variant 2: one
        // workgroup per tile.  The tiles and their order within a workgroup
        // do not change the result.
        const long long cap = variant == 1 ? 1024 : (variant == 2 ? tiles : 1280);
        const long long per = (tiles + cap - 1) / cap;
        const long long grid = (tiles + per - 1) / per;
        SAR_LAUNCH(k_corner_turn_x2, dim3((unsigned)grid), dim3(256), 0, s,
                           (const float4*)in, (float4*)out, rows, cols, (int)tiles);
    }
    else
        SAR_LAUNCH(k_corner_turn, dim3((unsigned)tiles), dim3(256), 0, s,
                           (const float2*)in, (float2*)out, rows, cols);
    return hipGetLastError();
}

hipError_t launch_rcmc_interp(const void* A, void* out, int na, const RcmcHost& rh, hipStream_t s)
{
    const RcmcArgs ra = make_rcmc_args(rh);
    const long long total = (long long)rh.nr * na;
    if (rh.taps == 8)
        SAR_LAUNCH(k_rcmc_interp<8>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                           (const float2*)A, (float2*)out, na, ra);
    else
        SAR_LAUNCH(k_rcmc_interp<0>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                           (const float2*)A, (float2*)out, na, ra);
    return hipGetLastError();
}

hipError_t launch_az_phase(const void* in, void* out, int na, const RcmcHost& rh, float scale,
                           hipStream_t s)
{
    const RcmcArgs ra = make_rcmc_args(rh);
    const long long total = (long long)rh.nr * na;
    SAR_LAUNCH(k_az_phase, dim3(grid_for(total, 256)), dim3(256), 0, s, (const float2*)in,
                       (float2*)out, na, ra, scale);
    return hipGetLastError();
}

hipError_t launch_gen_twiddles(void* tw, int n, hipStream_t s)
{
    const int cnt = twiddle_table_size(n);
    if (cnt <= 0) return hipSuccess;
    SAR_LAUNCH(k_gen_twiddles, dim3((cnt + 255) / 256), dim3(256), 0, s, (float2*)tw, n,
                       line_e(n));
    return hipGetLastError();
}

hipError_t launch_gen_chirp_filter(void* H, int n, int len, double K, int sign, double scale,
                                   hipStream_t s)
{
    SAR_LAUNCH(k_gen_chirp_filter, dim3((n + 255) / 256), dim3(256), 0, s, (float2*)H, n,
                       len, K, sign, scale);
    return hipGetLastError();
}

hipError_t launch_gen_rcmc_table(float* tab, double beta, hipStream_t s)
{
    SAR_LAUNCH(k_gen_rcmc_table, dim3(1), dim3(RCMC_INTERVALS), 0, s, tab, beta);
    return hipGetLastError();
}

int rcmc_table_floats() { return RCMC_TAB; }

hipError_t launch_gen_hyper_tables(double* stretch, double* rate, int na, double lam, double v,
                                   hipStream_t s)
{
    // the same expressions as the kernels' RcmcArgs (x_per_bin, two_over_lam)
    SAR_LAUNCH(k_gen_hyper_tables, dim3((na + 255) / 256), dim3(256), 0, s, stretch, rate,
                       na, lam / (2.0 * v * (double)na), 2.0 / lam);
    return hipGetLastError();
}

#endif  // SAR_PART == 0

}  // namespace sar

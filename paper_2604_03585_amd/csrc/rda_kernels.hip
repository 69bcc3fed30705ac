// rda_kernels.hip -- gfx950 kernels of the Range Doppler Algorithm and their
// launchers.  Every kernel is written for wave64 CDNA4; lines are kept in
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
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_line.hpp"
#include "rda_internal.h"

namespace sar {

// ===================================================== FP64 generators
// exp(-2 pi i * num / den) in FP64, num reduced exactly mod den first.
__device__ __forceinline__ float2 twiddle_fp64(long long num, long long den)
{
    long long r = num % den;
    double s, c;
    sincospi(-2.0 * (double)r / (double)den, &s, &c);
    return make_float2((float)c, (float)s);
}

// Per-N Stockham twiddle table (layout in fft_line.hpp, LineGeom::tw_off).
__global__ void k_gen_twiddles(float2* __restrict__ tw, int n)
{
    int log = 0;
    while ((1 << log) < n) ++log;
    const int n16 = log / 4, rem = 1 << (log % 4);
    const int np = n16 + (rem > 1 ? 1 : 0);
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int off = 0, ns = 1;
    for (int p = 0; p < np; ++p) {
        const int R = p < n16 ? 16 : rem;
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

// Hyperbolic per-Doppler-bin tables: f_k in fftfreq order (PRF = 1),
// x = lam f / (2 v), D = sqrt(1 - x^2); stretch = x^2 / (D (1 + D)) (= 1/D - 1
// without cancellation); rate = 2 D / lam (azimuth phase in turns per cell).
__global__ void k_gen_hyper_tables(double* __restrict__ stretch, double* __restrict__ rate,
                                   int na, double lam, double v)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= na) return;
    const double f = (k < na / 2) ? (double)k / na : (double)(k - na) / na;
    const double x = lam * f / (2.0 * v);
    const double D = sqrt(1.0 - x * x);
    stretch[k] = x * x / (D * (1.0 + D));
    rate[k] = 2.0 * D / lam;
}

// ===================================================== line kernels
template <int N> struct LineLaunch {
    static constexpr int T = LineGeom<N>::T;
    static constexpr int LPW = T >= 256 ? 1 : 256 / T;     // lines per workgroup
    static constexpr int BLOCK = LPW * T;
    static constexpr int LDS_BYTES = LPW * LineGeom<N>::LDS * (int)sizeof(float2);
};

// XCD-aware line order: gfx950 hands workgroup b to XCD (b mod 8); giving each
// XCD a contiguous run of line groups keeps neighbouring lines in one L2.
__device__ __forceinline__ int xcd_group(int b, int groups)
{
    if ((groups & 7) != 0) return b;
    return (b & 7) * (groups >> 3) + (b >> 3);
}

template <int N>
__device__ __forceinline__ void load_line(float2 (&x)[16], const float2* __restrict__ src, int t)
{
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = src[t + m * LineGeom<N>::T];
}

template <int N>
__device__ __forceinline__ void store_line(const float2 (&x)[16], float2* __restrict__ dst, int t)
{
#pragma unroll
    for (int m = 0; m < 16; ++m) dst[t + m * LineGeom<N>::T] = x[m];
}

template <int N>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK) void
k_line_fused(const float2* in, float2* out, int lines, const float2* __restrict__ H,
             const float2* __restrict__ tw)
{
    using L = LineLaunch<N>;
    extern __shared__ float2 smem[];
    const int groups = (lines + L::LPW - 1) / L::LPW;
    const int g = xcd_group(blockIdx.x, groups);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int line = g * L::LPW + sub;
    const bool live = line < lines;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    float2 x[16];
    if (live) load_line<N>(x, in + (size_t)line * N, t);
    else {
#pragma unroll
        for (int m = 0; m < 16; ++m) x[m] = make_float2(0.f, 0.f);
    }
    fft_line<N, false>(x, lds, tw, t);
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = c_mul(x[m], H[t + m * L::T]);
    fft_line<N, true>(x, lds, tw, t);
    if (live) store_line<N>(x, out + (size_t)line * N, t);
}

template <int N, bool INV>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK) void
k_line_fft(const float2* in, float2* out, int lines, const float2* __restrict__ tw, float scale)
{
    using L = LineLaunch<N>;
    extern __shared__ float2 smem[];
    const int groups = (lines + L::LPW - 1) / L::LPW;
    const int g = xcd_group(blockIdx.x, groups);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int line = g * L::LPW + sub;
    const bool live = line < lines;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    float2 x[16];
    if (live) load_line<N>(x, in + (size_t)line * N, t);
    else {
#pragma unroll
        for (int m = 0; m < 16; ++m) x[m] = make_float2(0.f, 0.f);
    }
    fft_line<N, INV>(x, lds, tw, t);
    if (scale != 1.0f) {
#pragma unroll
        for (int m = 0; m < 16; ++m) x[m] = c_scale(x[m], scale);
    }
    if (live) store_line<N>(x, out + (size_t)line * N, t);
}

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

// ===================================================== RCMC
// Interpolation weights of the 8-tap Kaiser-windowed sinc (taps t = -3..4
// about floor(p), x = p - floor(p)), in a division-free form: with
// z_t = t - x, sinc(z_t) = -(-1)^t sin(pi x) / (pi z_t), so after the unit-sum
// normalisation the weights are proportional to
//     q_t = (-1)^t * Win(z_t) * prod_{t' != t} z_t',
//     Win(z) = I0(beta * sqrt(1 - z^2/16)) = sum_k u^k / (k!)^2,
//     u = (beta^2 / 4) (1 - z^2 / 16),
// which also collapses to the identity at x = 0 with no special case.
// Returns sum_t q_t * a_t / sum_t q_t for the eight samples a[].
__device__ __forceinline__ float2 kaiser_sinc8(float x, float b4, float b64, const float2 (&a)[8])
{
    float z[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (float)(i - 3) - x;
    float pre[8], suf[8];
    pre[0] = 1.0f;
#pragma unroll
    for (int i = 1; i < 8; ++i) pre[i] = pre[i - 1] * z[i - 1];
    suf[7] = 1.0f;
#pragma unroll
    for (int i = 6; i >= 0; --i) suf[i] = suf[i + 1] * z[i + 1];
    float den = 0.0f;
    float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float u = fmaf(-b64, z[i] * z[i], b4);
        // Horner of sum_{k=0}^{8} u^k / (k!)^2
        float w = 1.0f / 1625702400.0f;
        w = fmaf(w, u, 1.0f / 25401600.0f);
        w = fmaf(w, u, 1.0f / 518400.0f);
        w = fmaf(w, u, 1.0f / 14400.0f);
        w = fmaf(w, u, 1.0f / 576.0f);
        w = fmaf(w, u, 1.0f / 36.0f);
        w = fmaf(w, u, 0.25f);
        w = fmaf(w, u, 1.0f);
        w = fmaf(w, u, 1.0f);
        float q = w * pre[i] * suf[i];
        if ((i - 3) & 1) q = -q;
        den += q;
        acc.x = fmaf(q, a[i].x, acc.x);
        acc.y = fmaf(q, a[i].y, acc.y);
    }
    const float inv = 1.0f / den;
    return make_float2(acc.x * inv, acc.y * inv);
}

struct RcmcArgs {
    const double* stretch;   // 1/D_k - 1 per Doppler bin
    const double* rate;      // 2 D_k / lambda per Doppler bin
    double r_near;
    float b4, b64;           // beta^2/4, beta^2/64
    int nr;
};

// RCMC output sample y[n][k] from range-Doppler A[Nr][Na] (rows outside
// [0, Nr) contribute nothing), times exp(+j 2 pi frac(R0 * rate_k)) * scale.
template <int TAPS>
__device__ __forceinline__ float2 rcmc_sample(const float2* __restrict__ A, int na, int n, int k,
                                              const RcmcArgs& ra, float scale, bool phase)
{
    const double R0 = ra.r_near + (double)n;
    float2 y;
    if constexpr (TAPS == 0) {
        y = A[(size_t)n * na + k];
    } else {
        const double s = R0 * ra.stretch[k];
        const double fl = floor(s);
        const float x = (float)(s - fl);
        // shifts beyond +-2^30 cells read nothing but stay defined integers
        const int i0 = n + (int)fmax(-1073741824.0, fmin(fl, 1073741824.0));
        float2 a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int r = i0 + i - 3;
            a[i] = (r >= 0 && r < ra.nr) ? A[(size_t)r * na + k] : make_float2(0.f, 0.f);
        }
        y = kaiser_sinc8(x, ra.b4, ra.b64, a);
    }
    if (phase) {
        const double ph = R0 * ra.rate[k];
        float f = (float)(ph - floor(ph));
        if (f > 0.5f) f -= 1.0f;
        float sn, cs;
        sincospif(2.0f * f, &sn, &cs);
        y = c_mul(y, make_float2(cs * scale, sn * scale));
    }
    return y;
}

template <int N, int TAPS>
__global__ __launch_bounds__(LineLaunch<N>::BLOCK) void
k_rcmc_az(const float2* __restrict__ A, float2* __restrict__ out, RcmcArgs ra,
          const float2* __restrict__ tw)
{
    using L = LineLaunch<N>;
    extern __shared__ float2 smem[];
    const int lines = ra.nr;
    const int groups = (lines + L::LPW - 1) / L::LPW;
    const int g = xcd_group(blockIdx.x, groups);
    const int sub = threadIdx.x / L::T, t = threadIdx.x % L::T;
    const int n = g * L::LPW + sub;
    const bool live = n < lines;
    float2* lds = smem + sub * LineGeom<N>::LDS;
    float2 x[16];
    constexpr float scale = 1.0f / (float)N;
#pragma unroll
    for (int m = 0; m < 16; ++m)
        x[m] = live ? rcmc_sample<TAPS>(A, N, n, t + m * L::T, ra, scale, true)
                    : make_float2(0.f, 0.f);
    fft_line<N, true>(x, lds, tw, t);
    if (live) store_line<N>(x, out + (size_t)n * N, t);
}

// Unfused comparator: RCMC interpolation alone (one sample per thread).
template <int TAPS>
__global__ __launch_bounds__(256) void k_rcmc_interp(const float2* __restrict__ A,
                                                     float2* __restrict__ out, int na, RcmcArgs ra)
{
    const long long total = (long long)ra.nr * na;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int n = (int)(e / na), k = (int)(e % na);
        out[e] = rcmc_sample<TAPS>(A, na, n, k, ra, 1.0f, false);
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
        const double ph = (ra.r_near + (double)n) * ra.rate[k];
        float f = (float)(ph - floor(ph));
        if (f > 0.5f) f -= 1.0f;
        float sn, cs;
        sincospif(2.0f * f, &sn, &cs);
        out[e] = c_mul(in[e], make_float2(cs * scale, sn * scale));
    }
}

// ===================================================== launchers
static int grid_for(long long work, int per_block)
{
    long long g = (work + per_block - 1) / per_block;
    const long long cap = 256LL * 64;   // grid-stride kernels: 64 workgroups per CU
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

template <int N>
static hipError_t set_lds_limit()
{
    using L = LineLaunch<N>;
    hipError_t e = hipSuccess;
    if (L::LDS_BYTES > 64 * 1024) {
        e = hipFuncSetAttribute((const void*)k_line_fused<N>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_line_fft<N, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_line_fft<N, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_rcmc_az<N, 0>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_rcmc_az<N, 8>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, L::LDS_BYTES);
    }
    return e;
}

template <int N>
static hipError_t launch_line_n(LineOp op, const float2* in, float2* out, int lines,
                                const float2* H, const float2* tw, float scale,
                                const RcmcArgs* ra, int taps, hipStream_t s)
{
    using L = LineLaunch<N>;
    static const hipError_t attr = set_lds_limit<N>();
    if (attr != hipSuccess) return attr;
    const int groups = (lines + L::LPW - 1) / L::LPW;
    if (groups == 0) return hipSuccess;
    dim3 grid(groups), block(L::BLOCK);
    switch (op) {
    case LineOp::Fused:
        hipLaunchKernelGGL(k_line_fused<N>, grid, block, L::LDS_BYTES, s, in, out, lines, H, tw);
        break;
    case LineOp::Forward:
        hipLaunchKernelGGL((k_line_fft<N, false>), grid, block, L::LDS_BYTES, s, in, out, lines, tw,
                           scale);
        break;
    case LineOp::Inverse:
        hipLaunchKernelGGL((k_line_fft<N, true>), grid, block, L::LDS_BYTES, s, in, out, lines, tw,
                           scale);
        break;
    case LineOp::RcmcAz:
        if (taps == 8)
            hipLaunchKernelGGL((k_rcmc_az<N, 8>), grid, block, L::LDS_BYTES, s, in, out, *ra, tw);
        else
            hipLaunchKernelGGL((k_rcmc_az<N, 0>), grid, block, L::LDS_BYTES, s, in, out, *ra, tw);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_line(LineOp op, int n, const void* in, void* out, int lines, const void* H,
                       const void* tw, float scale, const RcmcHost* rh, hipStream_t s)
{
    RcmcArgs ra{};
    int taps = 0;
    if (rh) {
        ra.stretch = rh->stretch;
        ra.rate = rh->rate;
        ra.r_near = rh->r_near;
        ra.b4 = (float)(rh->beta * rh->beta / 4.0);
        ra.b64 = (float)(rh->beta * rh->beta / 64.0);
        ra.nr = rh->nr;
        taps = rh->taps;
    }
    auto i = (const float2*)in;
    auto o = (float2*)out;
    auto h = (const float2*)H;
    auto w = (const float2*)tw;
    switch (n) {
    case 64: return launch_line_n<64>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 128: return launch_line_n<128>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 256: return launch_line_n<256>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 512: return launch_line_n<512>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 1024: return launch_line_n<1024>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 2048: return launch_line_n<2048>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 4096: return launch_line_n<4096>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 8192: return launch_line_n<8192>(op, i, o, lines, h, w, scale, &ra, taps, s);
    case 16384: return launch_line_n<16384>(op, i, o, lines, h, w, scale, &ra, taps, s);
    default: return hipErrorInvalidValue;
    }
}

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
    hipLaunchKernelGGL(k_rowmul, dim3(grid_for(pairs, 256)), dim3(256), 0, s, (const float4*)in,
                       (float4*)out, pairs, n, (const float2*)H);
    return hipGetLastError();
}

hipError_t launch_corner_turn(const void* in, void* out, int rows, int cols, hipStream_t s)
{
    const long long tiles = (long long)((rows + TT - 1) / TT) * ((cols + TT - 1) / TT);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_corner_turn, dim3((unsigned)tiles), dim3(256), 0, s, (const float2*)in,
                       (float2*)out, rows, cols);
    return hipGetLastError();
}

hipError_t launch_rcmc_interp(const void* A, void* out, int na, const RcmcHost& rh, hipStream_t s)
{
    RcmcArgs ra{rh.stretch, rh.rate, rh.r_near, (float)(rh.beta * rh.beta / 4.0),
                (float)(rh.beta * rh.beta / 64.0), rh.nr};
    const long long total = (long long)rh.nr * na;
    if (rh.taps == 8)
        hipLaunchKernelGGL(k_rcmc_interp<8>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                           (const float2*)A, (float2*)out, na, ra);
    else
        hipLaunchKernelGGL(k_rcmc_interp<0>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                           (const float2*)A, (float2*)out, na, ra);
    return hipGetLastError();
}

hipError_t launch_az_phase(const void* in, void* out, int na, const RcmcHost& rh, float scale,
                           hipStream_t s)
{
    RcmcArgs ra{rh.stretch, rh.rate, rh.r_near, 0.f, 0.f, rh.nr};
    const long long total = (long long)rh.nr * na;
    hipLaunchKernelGGL(k_az_phase, dim3(grid_for(total, 256)), dim3(256), 0, s, (const float2*)in,
                       (float2*)out, na, ra, scale);
    return hipGetLastError();
}

hipError_t launch_gen_twiddles(void* tw, int n, hipStream_t s)
{
    const int cnt = twiddle_table_size(n);
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_twiddles, dim3((cnt + 255) / 256), dim3(256), 0, s, (float2*)tw, n);
    return hipGetLastError();
}

hipError_t launch_gen_chirp_filter(void* H, int n, int len, double K, int sign, double scale,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_gen_chirp_filter, dim3((n + 255) / 256), dim3(256), 0, s, (float2*)H, n,
                       len, K, sign, scale);
    return hipGetLastError();
}

hipError_t launch_gen_hyper_tables(double* stretch, double* rate, int na, double lam, double v,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_gen_hyper_tables, dim3((na + 255) / 256), dim3(256), 0, s, stretch, rate,
                       na, lam, v);
    return hipGetLastError();
}

}  // namespace sar

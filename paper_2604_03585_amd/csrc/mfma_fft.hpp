// mfma_fft.hpp -- split-precision radix-16 butterflies on gfx950 MFMA.
//
// The precision variant computes every radix-16 DFT of a Stockham pass as a
// small dense matrix product (the paper's DFT_8 as four real MMAs, Sec. III.A
// eqs. 1-2, widened to radix 16 and to the 16x16x32 MFMA shape):
//
//     [Yr]   [Fr  -Fi] [Xr]          F[k][n] = exp(-+2 pi i k n / 16) / 16
//     [Yi] = [Fi   Fr] [Xi] ,        (32 x 32 real, applied to 16 DFTs at once)
//
// with v_mfma_f32_16x16x32_{f16,bf16}: D(16x16) = A(16x32) B(32x16), where a
// wave's lane l holds A[l%16][8(l/16)+i], B[8(l/16)+i][l%16] (i < 8) and
// D[4(l/16)+i][l%16] (i < 4) -- the layout was checked on the device.  The
// rows of B interleave the parts, B[2n][b] = Re x_n, B[2n+1][b] = Im x_n of
// butterfly b, and the columns of A follow: one MFMA gives Yr (A[k][2n] =
// Fr, A[k][2n+1] = -Fi), the other Yi (Fi, Fr).  A lane's B values are then
// the complete samples x_4q .. x_4q+3 (q = l/16), four 8-byte LDS reads, and
// its D values the complete outputs Y_4q .. Y_4q+3, four 8-byte writes.
//
// Each FP32 operand is split as x = hi + lo (hi = round(x), lo =
// round(x - hi)) and the product is accumulated in FP32 as
// F_hi X_hi + F_hi X_lo + F_lo X_hi (the lo*lo term is dropped).
//
// Range.  FP16 holds magnitudes up to 65504, and its lo parts keep full
// precision only while |x| >= 2^-3 (below that they go subnormal).  So every
// line is first scaled by a power of two 2^-e of its own (exact), chosen from
// the line's largest component so that it lies in [2^14, 2^15).  F carries a
// factor 1/16 (exact): then |Y_k| = |sum_n F[k][n] x_n| <= max_n |x_n| for
// every output of a pass, and the twiddles keep magnitudes, so no component
// ever exceeds sqrt(2) * 2^15 < 65504 whatever the input's scale; the
// transform's values stay within the line's own dynamic range of 2^15.  The
// scale 2^e * 16^passes is restored at the end.  Twiddles are applied in
// FP32 between passes, on the output side of a pass (where a lane holds
// complete complex values), already for the next pass.
//
// LDS holds the WG's lines as complex values (float2), one pad slot per 16
// entries: the exchange layout of the FP32 path.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_line.hpp"

namespace sar {

enum Prec { PREC_FP32 = 0, PREC_F16 = 1, PREC_BF16 = 2 };

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <int PREC> struct MfmaT;
template <> struct MfmaT<PREC_F16> {
    using scalar = _Float16;
    using vec = h8_t;
    __device__ __forceinline__ static f4_t mma(vec a, vec b, f4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct MfmaT<PREC_BF16> {
    using scalar = __bf16;
    using vec = b8_t;
    __device__ __forceinline__ static f4_t mma(vec a, vec b, f4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

typedef float f8_t __attribute__((ext_vector_type(8)));

// hi + lo split of eight FP32 values: hi = round(v) by packed conversions,
// lo = round(v - hi), where v - hi is exact in FP32 (hi is v rounded to
// fewer bits in the same binade or a subnormal).  FP16: v - hi is one
// v_fma_mix_f32 per value (hi widened inside the FMA, times a -1 held in a
// register so that the compiler keeps the mixed form); BF16: hi widens by a
// shift or a mask, then a plain subtraction.
template <int PREC>
__device__ __forceinline__ void split8(const float (&v)[8], typename MfmaT<PREC>::vec& hi,
                                       typename MfmaT<PREC>::vec& lo)
{
    using S = typename MfmaT<PREC>::scalar;
    using V = typename MfmaT<PREC>::vec;
    f8_t x;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = v[i];
    hi = __builtin_convertvector(x, V);
    if constexpr (PREC == PREC_F16) {
        int m1 = 0xBC00;                          // -1.0 in FP16
        asm volatile("" : "+s"(m1));
        const float neg1 = (float)__builtin_bit_cast(_Float16, (unsigned short)m1);
#pragma unroll
        for (int i = 0; i < 8; ++i) lo[i] = (S)__builtin_fmaf((float)hi[i], neg1, v[i]);
    } else {
        // BF16 widens by placing its bits in the top half of a float: two
        // bit operations per packed pair
        typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
        const u4_t hb = __builtin_bit_cast(u4_t, hi);
        f8_t back;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            back[2 * i] = __uint_as_float(hb[i] << 16);
            back[2 * i + 1] = __uint_as_float(hb[i] & 0xffff0000u);
        }
        lo = __builtin_convertvector(x - back, V);
    }
}

// The constant DFT operands of one wave: A_r = [Fr -Fi], A_i = [Fi Fr] (x 1/16),
// each split in hi/lo, in the MFMA A layout for this lane.
template <int PREC> struct DftOperands {
    typename MfmaT<PREC>::vec rh, rl, ih, il;
};

template <int PREC, bool INV>
__device__ __forceinline__ DftOperands<PREC> dft16_operands(int lane)
{
    // cos / sin of 2 pi m / 16, m = 0..15
    constexpr float C[16] = {1.0f, 0.92387953251128675613f, 0.70710678118654752440f,
                             0.38268343236508977173f, 0.0f, -0.38268343236508977173f,
                             -0.70710678118654752440f, -0.92387953251128675613f, -1.0f,
                             -0.92387953251128675613f, -0.70710678118654752440f,
                             -0.38268343236508977173f, 0.0f, 0.38268343236508977173f,
                             0.70710678118654752440f, 0.92387953251128675613f};
    const int k = lane & 15, q = lane >> 4;
    float ar[8], ai[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int n = 4 * q + (i >> 1);                 // column 8q + i = 2n + (i & 1)
        const int m = (k * n) & 15;
        const float fr = C[m] * 0.0625f;
        const float s = C[(m + 12) & 15] * 0.0625f;    // sin(2 pi m/16) = cos(2 pi (m - 4)/16)
        const float fi = INV ? s : -s;                  // F = exp(-+ i 2 pi m / 16)
        ar[i] = (i & 1) ? -fi : fr;                     // Yr: Fr Re x_n - Fi Im x_n
        ai[i] = (i & 1) ? fr : fi;                      // Yi: Fi Re x_n + Fr Im x_n
    }
    DftOperands<PREC> d;
    split8<PREC>(ar, d.rh, d.rl);
    split8<PREC>(ai, d.ih, d.il);
    return d;
}

__device__ __forceinline__ int mf_pad(int i) { return i + (i >> 4); }

// Exponent e of a line whose largest component is amax: amax * 2^-e lies in
// [2^14, 2^15); zero, non-finite and empty lines keep e = 0.
__device__ __forceinline__ int mfma_line_exponent(float amax)
{
    if (!(amax > 0.f) || !(amax < INFINITY)) return 0;
    return max(ilogbf(amax) - 14, -126);
}

// The line's exponent, from the largest |re|, |im| over its T threads: lane
// segments of a wave when T <= 64, else whole waves combined through the
// line's LDS pad slots (entries 17 w + 16 of its line, which the passes never
// touch since mf_pad skips them).  On entry no wave may still read the
// workgroup's LDS (the callers end every earlier LDS use with a barrier).
template <int T, int LL>
__device__ __forceinline__ int mfma_line_scale_exp(const float2 (&x)[16], float2* __restrict__ lds,
                                                   int sub)
{
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) m = fmaxf(m, fmaxf(fabsf(x[i].x), fabsf(x[i].y)));
    constexpr int W = T < 64 ? T : 64;
#pragma unroll
    for (int off = 1; off < W; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    if constexpr (T > 64) {
        constexpr int WPL = T / 64;               // waves per line
        static_assert(17 * (WPL - 1) + 16 < LL, "pad slots of the line");
        const int lane = threadIdx.x & 63, wl = (threadIdx.x >> 6) % WPL;
        float2* slots = lds + sub * LL;
        if (lane == 0) slots[17 * wl + 16].x = m;
        __syncthreads();
        m = 0.f;
#pragma unroll
        for (int w = 0; w < WPL; ++w) m = fmaxf(m, slots[17 * w + 16].x);
    }
    const int e = mfma_line_exponent(m);
    // a wave holds one line when T >= 64: the exponent is wave-uniform
    if constexpr (T >= 64) return __builtin_amdgcn_readfirstlane(e);
    else return e;
}

// All radix-16 passes of the lines of one workgroup on MFMA, followed by the
// trailing smaller pass (if any) in FP32.  On entry each thread holds its
// line's x in the strided register layout (see fft_line.hpp); on exit it
// holds the transform (scaled back to the plain unnormalised DFT).
//   lds:   the workgroup's LDS (LPW lines, N + N/16 float2 each)
//   sub:   this thread's line within the workgroup, t its index in the line
//   before_last: runs as the last MFMA pass starts (callers issue the loads
//          they need right after the transform there, e.g. a filter)
template <int N, bool INV, int PREC, int LPW, int BLOCK, class Pre = NoOp>
__device__ __forceinline__ void fft_line_mfma(float2 (&x)[16], float2* __restrict__ lds,
                                              const float2* __restrict__ tw, int sub, int t,
                                              Pre&& before_last = Pre())
{
    using G = LineGeom<N, 16>;
    static_assert(line_e(N) == 16, "the MFMA path uses 16 points per thread");
    constexpr int T = G::T;
    constexpr int LL = G::LDS;                   // float2 per line
    constexpr int NB = N / 16;                   // butterflies per line and pass
    constexpr int NMF = G::NFULL;                // radix-16 (MFMA) passes
    constexpr int GROUPS = LPW * NB / 16;        // 16-butterfly groups per workgroup
    constexpr int WAVES = BLOCK / 64;
    constexpr int GPW = GROUPS / WAVES;          // groups per wave
    static_assert(GROUPS % WAVES == 0 && GPW >= 1, "group split");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    const int c = lane & 15, q = lane >> 4;

    // registers -> LDS, scaled by the line's 2^-ex
    const int ex = mfma_line_scale_exp<T, LL>(x, lds, sub);
#pragma unroll
    for (int m = 0; m < 16; ++m)
        lds[sub * LL + mf_pad(t + m * T)] = make_float2(ldexpf(x[m].x, -ex), ldexpf(x[m].y, -ex));
    __syncthreads();

    const DftOperands<PREC> F = dft16_operands<PREC, INV>(lane);

#pragma unroll
    for (int p = 0; p < NMF; ++p) {
        if (p == NMF - 1) before_last();
        const int NS = p == 0 ? 1 : (p == 1 ? 16 : (p == 2 ? 256 : 4096));
        const bool next_mfma = (p + 1 < NMF);
        // Next-pass twiddles of a lane's outputs k = 4q .. 4q+3 of butterfly j
        // (output e = base + k NS, base = (j / NS) 16 NS + j mod NS): with
        // 16 NS <= N / 16 the row i2 = e / (N/16) is the same for the four k and
        // the column (e mod N/16) mod 16 NS is j mod NS + k NS, so the twiddles
        // W^(i2 (j mod NS + k NS)) form a geometric sequence: the first and the
        // step W^(i2 NS) are read from the table (at the start of the pass, so
        // that the reads overlap it), the other three are products.  Row 0
        // needs none (its twiddles are 1); its reads go to the table's row 1.
        float2 w0[GPW], wst[GPW];
        bool won[GPW];
        if (next_mfma) {
            const float2* tab = tw + G::tw_off(p + 1);
#pragma unroll
            for (int gi = 0; gi < GPW; ++gi) {
                const int b = (wave * GPW + gi) * 16 + c;
                const int j = b % NB, jm = j & (NS - 1);
                const int i2 = ((j / NS) * NS * 16 + jm + 4 * q * NS) / NB;
                const float2* row = tab + (i2 > 0 ? i2 - 1 : 0) * (NS * 16);
                w0[gi] = row[jm + 4 * q * NS];
                wst[gi] = row[NS];
                won[gi] = i2 > 0;
            }
        }
        float2 y[GPW][4];
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi) {
            const int b = (wave * GPW + gi) * 16 + c;          // butterfly in the WG
            const int s = b / NB, j = b % NB;
            const float2* src = lds + s * LL;
            float v[8];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const float2 u = src[mf_pad(j + (4 * q + h) * NB)];
                v[2 * h] = u.x;
                v[2 * h + 1] = u.y;
            }
            typename MfmaT<PREC>::vec bh, bl;
            split8<PREC>(v, bh, bl);
            f4_t ar = {0.f, 0.f, 0.f, 0.f}, ai = {0.f, 0.f, 0.f, 0.f};
            ar = MfmaT<PREC>::mma(F.rh, bh, ar);
            ar = MfmaT<PREC>::mma(F.rh, bl, ar);
            ar = MfmaT<PREC>::mma(F.rl, bh, ar);
            ai = MfmaT<PREC>::mma(F.ih, bh, ai);
            ai = MfmaT<PREC>::mma(F.ih, bl, ai);
            ai = MfmaT<PREC>::mma(F.il, bh, ai);
            float2 w = w0[gi], d = wst[gi];
            if (INV) {
                w.y = -w.y;
                d.y = -d.y;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float2 o = make_float2(ar[i], ai[i]);
                if (next_mfma) {                  // pre-twiddle for the next radix-16 pass
                    const float2 ow = c_mul(o, w);
                    o = won[gi] ? ow : o;
                    if (i < 3) w = c_mul(w, d);
                }
                y[gi][i] = o;
            }
        }
        __syncthreads();                          // every read of this pass is done
#pragma unroll
        for (int gi = 0; gi < GPW; ++gi) {
            const int b = (wave * GPW + gi) * 16 + c;
            const int s = b / NB, j = b % NB;
            const int base = (j / NS) * NS * 16 + (j & (NS - 1));
#pragma unroll
            for (int i = 0; i < 4; ++i) lds[s * LL + mf_pad(base + (4 * q + i) * NS)] = y[gi][i];
        }
        __syncthreads();
    }

    // LDS -> registers, undo the 1/16 per MFMA pass and the line's scale
    const int undo = ex + 4 * NMF;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const float2 u = lds[sub * LL + mf_pad(t + m * T)];
        x[m] = make_float2(ldexpf(u.x, undo), ldexpf(u.y, undo));
    }
    __syncthreads();                              // LDS free for the caller's next use
    if constexpr (G::NP > NMF) {
        // trailing radix-2/4/8 pass in FP32 (its twiddles applied on input)
        PassTw<N, G::NP - 1> pt;
        load_tw<N, G::NP - 1, false>(pt, tw, t);
        fft_pass<N, G::NP - 1, INV>(x, (float2*)nullptr, pt, t);
    }
}

}  // namespace sar

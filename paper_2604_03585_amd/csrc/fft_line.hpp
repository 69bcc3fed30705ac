// fft_line.hpp -- register/LDS line FFT building blocks for gfx950.
//
// One line of N complex64 points (64 <= N <= 16384, power of two) is held by
// T = N/E threads, E points per thread (E = 8 or 16), in the "strided"
// register layout:
//
//     thread t, register m  <->  element t + m*T .
//
// The transform is a sequence of self-sorting (Stockham) passes: radix-E
// passes followed by at most one smaller power-of-two pass (N = E^a * r).
// A pass with radix R and span Ns (product of the earlier radices) computes,
// for every butterfly j in [0, N/R),
//
//     v_i = x[j + i*N/R] * W_{Ns*R}^{(j mod Ns)*i},   i = 0..R-1
//     y[(j/Ns)*Ns*R + (j mod Ns) + k*Ns] = DFT_R(v)_k,
//
// and thread t owns butterflies j = t + q*T (q < E/R), whose inputs are its
// own registers q + i*(E/R).  Between passes the data go through LDS once
// (scatter write, barrier, strided read).  The last pass writes y in natural
// order straight back to the same registers, so a forward transform ends in
// the layout in which the next step (filter multiply, inverse transform,
// store) starts: FFT -> x H -> IFFT needs no extra exchange.
//
// The inverse transform (INV = true) uses conjugated twiddles and butterflies,
// i.e. computes sum_k X[k] exp(+2 pi i k n / N) without the 1/N, which the
// callers fold into the filter.  This equals the paper's conj(FFT(conj(.)))
// form of the IFFT (Sec. II.C) up to rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace sar {

// Workgroup barrier for LDS exchanges.  The compiler models the barrier and
// its fences as side effects that do not write memory, so LDS reads issued
// before a barrier may be sunk below it into a following branch, where they
// race with other waves' writes of the next exchange.  The empty asm that
// clobbers memory counts as a store and keeps every memory access on its
// side of the barrier.
__device__ __forceinline__ void wg_barrier()
{
    __syncthreads();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }

// a * (-j) for the forward transform, a * (+j) for the inverse.
template <bool INV>
__device__ __forceinline__ float2 c_mul_mj(float2 a)
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// a * exp(-+ j pi/4) = a * (1 -+ j)/sqrt(2)
template <bool INV>
__device__ __forceinline__ float2 c_mul_w8(float2 a)
{
    constexpr float r = 0.70710678118654752440f;
    return INV ? make_float2(r * (a.x - a.y), r * (a.y + a.x))
               : make_float2(r * (a.x + a.y), r * (a.y - a.x));
}

// a * exp(-+ j 3pi/4) = a * (-1 -+ j)/sqrt(2)
template <bool INV>
__device__ __forceinline__ float2 c_mul_w8_3(float2 a)
{
    constexpr float r = 0.70710678118654752440f;
    return INV ? make_float2(-r * (a.x + a.y), r * (a.x - a.y))
               : make_float2(r * (a.y - a.x), -r * (a.x + a.y));
}

// a * (c, -+ s)
template <bool INV>
__device__ __forceinline__ float2 c_mul_cs(float2 a, float c, float s)
{
    return c_mul(a, make_float2(c, INV ? s : -s));
}

// ---------------------------------------------------------- small DFTs
// All take natural-order input in v[] and leave natural-order output.
template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b)
{
    float2 t = a;
    a = c_add(t, b);
    b = c_sub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3)
{
    float2 s0 = c_add(a0, a2), d0 = c_sub(a0, a2);
    float2 s1 = c_add(a1, a3), d1 = c_mul_mj<INV>(c_sub(a1, a3));
    a0 = c_add(s0, s1);
    a2 = c_sub(s0, s1);
    a1 = c_add(d0, d1);
    a3 = c_sub(d0, d1);
}

template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
    __device__ __forceinline__ static void run(float2* v) { dft2<INV>(v[0], v[1]); }
};

template <bool INV> struct Dft<4, INV> {
    __device__ __forceinline__ static void run(float2* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }
};

// DFT8 = DFT2 (stride 4) x twiddle W8^{n2 k1} x DFT4.
template <bool INV> struct Dft<8, INV> {
    __device__ __forceinline__ static void run(float2* v)
    {
        dft2<INV>(v[0], v[4]);
        dft2<INV>(v[1], v[5]);
        dft2<INV>(v[2], v[6]);
        dft2<INV>(v[3], v[7]);
        v[5] = c_mul_w8<INV>(v[5]);
        v[6] = c_mul_mj<INV>(v[6]);
        v[7] = c_mul_w8_3<INV>(v[7]);
        // y[n2][k1] sits in v[n2 + 4 k1]; DFT4 over n2 gives X[k1 + 2 k2]
        float2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
        float2 b0 = v[4], b1 = v[5], b2 = v[6], b3 = v[7];
        dft4<INV>(a0, a1, a2, a3);
        dft4<INV>(b0, b1, b2, b3);
        v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
        v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
    }
};

// DFT16 = DFT4 (stride 4) x twiddle W16^{n2 k1} x DFT4.
template <bool INV> struct Dft<16, INV> {
    __device__ __forceinline__ static void run(float2* v)
    {
        constexpr float c1 = 0.92387953251128675613f;   // cos(pi/8)
        constexpr float s1 = 0.38268343236508977173f;   // sin(pi/8)
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
        // y[n2][k1] is in v[n2 + 4 k1]
        v[5] = c_mul_cs<INV>(v[5], c1, s1);     // n2=1 k1=1: W16^1
        v[9] = c_mul_w8<INV>(v[9]);             // n2=1 k1=2: W16^2
        v[13] = c_mul_cs<INV>(v[13], s1, c1);   // n2=1 k1=3: W16^3
        v[6] = c_mul_w8<INV>(v[6]);             // n2=2 k1=1: W16^2
        v[10] = c_mul_mj<INV>(v[10]);           // n2=2 k1=2: W16^4
        v[14] = c_mul_w8_3<INV>(v[14]);         // n2=2 k1=3: W16^6
        v[7] = c_mul_cs<INV>(v[7], s1, c1);     // n2=3 k1=1: W16^3
        v[11] = c_mul_w8_3<INV>(v[11]);         // n2=3 k1=2: W16^6
        v[15] = c_mul_cs<INV>(v[15], -c1, -s1); // n2=3 k1=3: W16^9 = (-c1, +s1)
        float2 o[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
            dft4<INV>(a0, a1, a2, a3);
            o[k1] = a0; o[k1 + 4] = a1; o[k1 + 8] = a2; o[k1 + 12] = a3;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = o[i];
    }
};

// ------------------------------------------------------------ pass plan
__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Points per thread for a line of length N.  16 (radix-16 passes) needs one
// LDS exchange fewer per transform than 8 at N = 4096 and measured faster.
__host__ __device__ constexpr int line_e(int n) { return n > 0 ? 16 : 16; }

template <int N, int E = line_e(N)> struct LineGeom {
    static_assert(N >= 64 && N <= 16384 && (N & (N - 1)) == 0, "line length");
    static_assert(E == 8 || E == 16, "points per thread");
    static_assert(N / E <= 1024, "threads per line");
    static constexpr int T = N / E;                        // threads per line
    static constexpr int LOG = ilog2(N);
    static constexpr int RLOG = ilog2(E);
    static constexpr int NFULL = LOG / RLOG;               // radix-E passes
    static constexpr int REM = 1 << (LOG % RLOG);          // trailing radix (1 = none)
    static constexpr int NP = NFULL + (REM > 1 ? 1 : 0);   // number of passes
    __host__ __device__ static constexpr int radix(int p) { return p < NFULL ? E : REM; }
    __host__ __device__ static constexpr int span(int p)   // Ns of pass p
    {
        return p == 0 ? 1 : span(p - 1) * radix(p - 1);
    }
    // offset of pass p's twiddles in the per-N table (pass 0 has none)
    __host__ __device__ static constexpr int tw_off(int p)
    {
        return p <= 1 ? 0 : tw_off(p - 1) + (radix(p - 1) - 1) * span(p - 1);
    }
    static constexpr int TW_SIZE = tw_off(NP);
    // LDS words (float2) per line: one pad slot every 16 entries
    static constexpr int LDS = N + N / 16;
};

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

// Twiddles a thread needs in pass P: for butterfly q (j = t + q*T) and
// i = 1..R-1, exp(-2 pi i * (j mod Ns) * i / (Ns * R)), read from this N's
// table (entry tw_off(P) + (i-1)*Ns + (j mod Ns)); passes with Ns == 1 need
// none.
template <int N, int P> struct PassTw {
    using G = LineGeom<N>;
    static constexpr bool ANY = P < G::NP && G::span(P) > 1;
    static constexpr int COUNT = ANY ? (line_e(N) / G::radix(P)) * (G::radix(P) - 1) : 1;
    float2 w[COUNT];
};

// TWP, radix-16 pass: W^1 and W^4 come from the table, the other powers are
// products (at most four roundings deep, ~3e-7 relative).  Thirteen complex
// products replace thirteen table reads, for kernels bound by vector-memory
// issue rather than by VALU.  w[i-1] = W^i, w[0] and w[3] given.
__device__ __forceinline__ void tw_products16(float2* w)
{
    w[1] = c_mul(w[0], w[0]);
    w[2] = c_mul(w[1], w[0]);
    w[4] = c_mul(w[3], w[0]);
    w[5] = c_mul(w[3], w[1]);
    w[6] = c_mul(w[3], w[2]);
    w[7] = c_mul(w[3], w[3]);
#pragma unroll
    for (int i = 8; i < 15; ++i) w[i] = c_mul(w[7], w[i - 8]);
}

template <int N, int P, bool TWP>
__device__ __forceinline__ void load_tw(PassTw<N, P>& pt, const float2* __restrict__ tw, int t)
{
    using G = LineGeom<N>;
    if constexpr (TWP && PassTw<N, P>::ANY && G::radix(P) == 16) {
        constexpr int NS = G::span(P), B = line_e(N) / 16, OFF = G::tw_off(P);
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int jm = (t + q * G::T) & (NS - 1);
            float2* w = pt.w + q * 15;
            w[0] = tw[OFF + jm];
            w[3] = tw[OFF + 3 * NS + jm];
            tw_products16(w);
        }
    } else if constexpr (PassTw<N, P>::ANY) {
        constexpr int R = G::radix(P), NS = G::span(P), B = line_e(N) / R, OFF = G::tw_off(P);
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int jm = (t + q * G::T) & (NS - 1);
#pragma unroll
            for (int i = 1; i < R; ++i) pt.w[q * (R - 1) + i - 1] = tw[OFF + (i - 1) * NS + jm];
        }
    }
}

// The table reads of a TWP radix-16 pass (W^1, W^4 per butterfly), issued
// one pass ahead so that their latency overlaps the previous pass and its
// LDS exchange; other passes read their twiddles when they start.
template <int N, int P, bool TWP> struct TwAhead {
    static constexpr bool ON = TWP && PassTw<N, P>::ANY && LineGeom<N>::radix(P) == 16;
    static constexpr int B = ON ? line_e(N) / 16 : 1;
    float2 w1[B], w4[B];
};

template <int N, int P, bool TWP>
__device__ __forceinline__ void tw_issue(TwAhead<N, P, TWP>& a, const float2* __restrict__ tw, int t)
{
    if constexpr (TwAhead<N, P, TWP>::ON) {
        using G = LineGeom<N>;
        constexpr int NS = G::span(P), OFF = G::tw_off(P);
#pragma unroll
        for (int q = 0; q < TwAhead<N, P, TWP>::B; ++q) {
            const int jm = (t + q * G::T) & (NS - 1);
            a.w1[q] = tw[OFF + jm];
            a.w4[q] = tw[OFF + 3 * NS + jm];
        }
    }
}

template <int N, int P, bool TWP>
__device__ __forceinline__ void tw_form(PassTw<N, P>& pt, const TwAhead<N, P, TWP>& a,
                                        const float2* __restrict__ tw, int t)
{
    if constexpr (TwAhead<N, P, TWP>::ON) {
#pragma unroll
        for (int q = 0; q < TwAhead<N, P, TWP>::B; ++q) {
            float2* w = pt.w + q * 15;
            w[0] = a.w1[q];
            w[3] = a.w4[q];
            tw_products16(w);
        }
    } else {
        load_tw<N, P, TWP>(pt, tw, t);
    }
}

// One Stockham pass P of an N-point line (see the header comment), with its
// twiddles already loaded.
// SPLIT: the exchange keeps real and imaginary parts in two float arrays of
// the line's LDS (re[0, LDS), im[LDS, 2 LDS)), two 4-byte accesses per point
// instead of one 8-byte access: the layout the MFMA passes need, here with
// FP32 butterflies, so that the two can be compared at equal layout.
template <int N, int P, bool INV, bool SPLIT = false>
__device__ __forceinline__ void fft_pass(float2 (&x)[line_e(N)], float2* __restrict__ lds,
                                         const PassTw<N, P>& pt, int t)
{
    using G = LineGeom<N>;
    constexpr int E = line_e(N);
    constexpr int R = G::radix(P);
    constexpr int NS = G::span(P);
    constexpr int B = E / R;
    constexpr bool LAST = (P == G::NP - 1);
#pragma unroll
    for (int q = 0; q < B; ++q) {
        float2 v[R];
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = x[q + i * B];
        const int j = t + q * G::T;
        const int jm = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
            for (int i = 1; i < R; ++i) {
                float2 w = pt.w[q * (R - 1) + i - 1];
                if (INV) w.y = -w.y;
                v[i] = c_mul(v[i], w);
            }
        }
        Dft<R, INV>::run(v);
        if constexpr (LAST) {
#pragma unroll
            for (int i = 0; i < R; ++i) x[q + i * B] = v[i];
        } else {
            const int base = (j / NS) * NS * R + jm;
            if constexpr (SPLIT) {
                float* re = (float*)lds;
                float* im = re + G::LDS;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    re[lds_pad(base + i * NS)] = v[i].x;
                    im[lds_pad(base + i * NS)] = v[i].y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < R; ++i) lds[lds_pad(base + i * NS)] = v[i];
            }
        }
    }
    if constexpr (!LAST) {
        wg_barrier();
        if constexpr (SPLIT) {
            const float* re = (const float*)lds;
            const float* im = re + G::LDS;
#pragma unroll
            for (int m = 0; m < E; ++m)
                x[m] = make_float2(re[lds_pad(t + m * G::T)], im[lds_pad(t + m * G::T)]);
        } else {
#pragma unroll
            for (int m = 0; m < E; ++m) x[m] = lds[lds_pad(t + m * G::T)];
        }
        wg_barrier();
    }
}

// Passes P.. of the line.  `before_last` runs just before the last pass
// (callers use it to request data needed right after the transform, e.g.
// the matched filter, so that its latency overlaps the last pass).
struct NoOp {
    __device__ __forceinline__ void operator()() const {}
};

// AHEAD: a TWP radix-16 pass's table reads are issued one pass early, so
// they are in flight during the previous pass and its exchange (and, for
// the last pass, ahead of the `before_last` loads).  They cost four
// registers across the previous pass: the forward / inverse-only, RCMC and
// long-line fused kernels have them, the shorter fused kernels do not.
template <int N, bool INV, bool TWP, int P, bool SPLIT, bool AHEAD, class F>
__device__ __forceinline__ void fft_from(float2 (&x)[line_e(N)], float2* __restrict__ lds,
                                         const float2* __restrict__ tw, int t, F&& before_last,
                                         const TwAhead<N, P, TWP>& ahead)
{
    if constexpr (P < LineGeom<N>::NP) {
        if constexpr (P == LineGeom<N>::NP - 1) before_last();
        PassTw<N, P> cur;
        TwAhead<N, P + 1, TWP> next;
        if constexpr (AHEAD) {
            tw_form<N, P, TWP>(cur, ahead, tw, t);
            tw_issue<N, P + 1, TWP>(next, tw, t);
        } else {
            load_tw<N, P, TWP>(cur, tw, t);
        }
        fft_pass<N, P, INV, SPLIT>(x, lds, cur, t);
        fft_from<N, INV, TWP, P + 1, SPLIT, AHEAD>(x, lds, tw, t, before_last, next);
    }
}

// TWP selects twiddles by products (fewer loads, more VALU) or table reads;
// SPLIT the split real/imaginary exchange layout (see fft_pass).
template <int N, bool INV, bool TWP = true, bool SPLIT = false, class F = NoOp>
__device__ __forceinline__ void fft_line(float2 (&x)[line_e(N)], float2* __restrict__ lds,
                                         const float2* __restrict__ tw, int t, F&& before_last = F())
{
    TwAhead<N, 0, TWP> first;
    fft_from<N, INV, TWP, 0, SPLIT, false>(x, lds, tw, t, before_last, first);
}

// The same transform with every TWP radix-16 pass's table reads issued one
// pass ahead.
template <int N, bool INV, bool TWP = true, bool SPLIT = false, class F = NoOp>
__device__ __forceinline__ void fft_line_ahead(float2 (&x)[line_e(N)], float2* __restrict__ lds,
                                               const float2* __restrict__ tw, int t,
                                               F&& before_last = F())
{
    TwAhead<N, 0, TWP> first;
    tw_issue<N, 0, TWP>(first, tw, t);
    fft_from<N, INV, TWP, 0, SPLIT, true>(x, lds, tw, t, before_last, first);
}

}  // namespace sar

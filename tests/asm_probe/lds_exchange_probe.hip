// Probe kernel for the LDS exchange barrier test: a fused line transform
// (forward, filter loads in the last-pass hook, inverse) whose store is
// conditional on a per-workgroup flag, the shape in which the compiler may
// move an exchange's LDS reads below the barrier that closes it.  Compiled
// to assembly only, never run.
#include "fft_line.hpp"

using namespace sar;

template <int N>
__global__ __launch_bounds__(LineGeom<N>::T) void
lds_exchange_probe(const float2* in, float2* out, const float2* __restrict__ H,
                   const float2* __restrict__ tw, int lines)
{
    constexpr int E = line_e(N), T = LineGeom<N>::T;
    extern __shared__ __align__(16) float2 lds[];
    const int t = threadIdx.x, line = blockIdx.x;
    const bool live = line < lines;                 // uniform per workgroup
    float2 x[E], h[E];
    if (live) {
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = in[(size_t)line * N + t + m * T];
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = make_float2(0.f, 0.f);
    }
    fft_line<N, false>(x, lds, tw, t, [&] {
#pragma unroll
        for (int m = 0; m < E; ++m) h[m] = H[t + m * T];
    });
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = c_mul(x[m], h[m]);
    fft_line<N, true>(x, lds, tw, t);
    if (live) {
#pragma unroll
        for (int m = 0; m < E; ++m) out[(size_t)line * N + t + m * T] = x[m];
    }
}

template __global__ void lds_exchange_probe<4096>(const float2*, float2*, const float2*,
                                                  const float2*, int);
template __global__ void lds_exchange_probe<16384>(const float2*, float2*, const float2*,
                                                   const float2*, int);

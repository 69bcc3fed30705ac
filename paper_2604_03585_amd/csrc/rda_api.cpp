// rda_api.cpp -- host side of libsar_rda.so: parameter validation, plans
// (device tables built by FP64 generator kernels), and the execute entry
// points declared in include/sar_rda.h.
//
// Dataflow of sar_rda_execute (Sec. IV.A / IV.B of arXiv 2604.03585), with
// two scene-sized buffers `img` and `work` used alternately so every step
// reads one and writes the other (the range pass reads the untouched raw):
//
//   LFM:        range [Na][Nr] -> turn -> azimuth FFT*H_a*IFFT    ([Nr][Na])
//   hyperbolic: range [Na][Nr] -> turn -> azimuth FFT -> RCMC*phase*IFFT
//   optional:   -> turn back to [Na][Nr]
//
// With SAR_UNFUSED every "FFT*H*IFFT" is three dispatches and RCMC*phase*IFFT
// is three dispatches as well (the comparator of Sec. II.B, Fig. 1).
#include "sar_rda.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rda_internal.h"

namespace {

thread_local std::string g_err;

sar_status fail(sar_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

sar_status hip_fail(hipError_t e, const char* what)
{
    return fail(SAR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

bool finite(double x) { return std::isfinite(x); }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    auto pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

bool misaligned(const void* p) { return ((uintptr_t)p & 15u) != 0; }

// Workspace of sar_rda_execute_noalloc: one array per GPU, held by the loaded
// code object for the life of the process.  `scratch` names the host-side
// stand-in of the array; kernels get its device address, which
// hipGetSymbolAddress returns per device (each device has its own copy).
// The lookup runs at set-up (sar_plan, with the plan's device current) so the
// entry point itself calls nothing but the kernels' launches.
static __device__ __align__(256) unsigned char scratch[SAR_NOALLOC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};

// Once per device (the device must be current): look up and keep the
// device address of `scratch`.  A failure is kept for the entry point to
// report; plans themselves do not depend on it.
void setup_noalloc_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device] || g_scratch_err[device] != hipSuccess) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        (void)hipGetLastError();          // do not leave the error for the caller's next call
        return;
    }
    g_scratch_ptr[device] = ptr;
}

}  // namespace

namespace {
constexpr int MAX_TIMED = 16;
thread_local hipEvent_t g_time_start[MAX_TIMED], g_time_stop[MAX_TIMED];
thread_local int g_time_next = 0, g_time_count = 0;
}  // namespace

namespace sar {
bool take_launch_events(hipEvent_t& start, hipEvent_t& stop)
{
    if (g_time_next >= g_time_count) return false;
    start = g_time_start[g_time_next];
    stop = g_time_stop[g_time_next];
    if (++g_time_next == g_time_count) g_time_next = g_time_count = 0;
    return true;
}

sar_status set_error(sar_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}
void clear_error() { g_err.clear(); }
}  // namespace sar

struct sar_plan_s {
    sar_params p;
    int device = 0;
    void* block = nullptr;        // one device allocation for all tables
    float2* tw_r = nullptr;       // Stockham twiddles for Nr
    float2* tw_a = nullptr;       // Stockham twiddles for Na
    float2* Hr = nullptr;         // range filter, includes 1/Nr
    float2* Ha = nullptr;         // LFM azimuth filter, includes 1/Na
    double* stretch = nullptr;    // hyperbolic: 1/D - 1
    double* rate = nullptr;       // hyperbolic: 2 D / lambda
    float* rcmc_tab = nullptr;    // hyperbolic: interpolation weight coefficients
    double stretch_max = 0.0;     // hyperbolic: 1/D - 1 at |f| = 1/2
    int var_r[3] = {0, 0, 0};     // tuned variants of the Nr line kernels (fused, fwd, inv)
    int var_a[4] = {0, 0, 0, 0};  // ... of the Na line kernels (fused, fwd, inv, RCMC)
    int var_turn = 0;             // corner turn of [Na][Nr]
    int var_back = 0;             // back-turn of [Nr][Na]
    int var_strip = 0;            // turn-free azimuth strips
};

namespace {
// Butterfly precision of the line kernels: half storage computes in FP32.
int arith(const sar_plan_s* P) { return P->p.precision == SAR_FP32_HALF_STORAGE ? SAR_FP32 : P->p.precision; }

// Workspace layout of a half-storage plan: two FP16 scene arrays, then the
// per-line exponents of the range lines (Na ints) and of the range-Doppler
// rows (Nr ints), each block 256-byte aligned.
struct HalfLayout {
    size_t wa, wb, e1, e2, total;
};
HalfLayout half_layout(int Na, int Nr)
{
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t px = (size_t)Na * (size_t)Nr;
    HalfLayout h;
    h.wa = 0;
    h.wb = al(4 * px);
    h.e1 = h.wb + al(4 * px);
    h.e2 = h.e1 + al(4 * (size_t)Na);
    h.total = h.e2 + al(4 * (size_t)Nr);
    return h;
}
}  // namespace

namespace sar {
PlanTables plan_tables(const sar_plan_s* P)
{
    return PlanTables{P->Hr, P->Ha, P->tw_r, P->tw_a};
}
}  // namespace sar

namespace {

sar_status validate_params(const sar_params* p)
{
    if (!p) return fail(SAR_ERR_NULL, "params is NULL");
    if (p->struct_size != sizeof(sar_params))
        return fail(SAR_ERR_BAD_PARAM, "struct_size %u != sizeof(sar_params) %zu", p->struct_size,
                    sizeof(sar_params));
    if (!pow2_in(p->Nr, 64, 16384)) return fail(SAR_ERR_BAD_SIZE, "Nr=%d: need a power of two in [64, 16384]", p->Nr);
    if (!pow2_in(p->Na, 64, 16384)) return fail(SAR_ERR_BAD_SIZE, "Na=%d: need a power of two in [64, 16384]", p->Na);
    if (p->range_len < 1 || p->range_len > p->Nr)
        return fail(SAR_ERR_BAD_SIZE, "range_len=%d outside [1, Nr]", p->range_len);
    if (!finite(p->range_tbp)) return fail(SAR_ERR_BAD_PARAM, "range_tbp is not finite");
    if (p->az_model == SAR_AZ_LFM) {
        if (p->az_len < 1 || p->az_len > p->Na)
            return fail(SAR_ERR_BAD_SIZE, "az_len=%d outside [1, Na]", p->az_len);
        if (!finite(p->az_tbp)) return fail(SAR_ERR_BAD_PARAM, "az_tbp is not finite");
    } else if (p->az_model == SAR_AZ_HYPERBOLIC) {
        if (!(finite(p->lambda) && p->lambda > 0.0)) return fail(SAR_ERR_BAD_PARAM, "lambda must be > 0");
        if (!(finite(p->v) && p->v > 0.0)) return fail(SAR_ERR_BAD_PARAM, "v must be > 0");
        if (!(finite(p->r_near) && p->r_near >= 0.0)) return fail(SAR_ERR_BAD_PARAM, "r_near must be >= 0");
        if (!(p->lambda < 4.0 * p->v))
            return fail(SAR_ERR_BAD_PARAM, "lambda/(4 v) >= 1: Doppler band exceeds the geometry");
        if (p->rcmc_taps != 0 && p->rcmc_taps != 8)
            return fail(SAR_ERR_BAD_PARAM, "rcmc_taps=%d: only 0 or 8", p->rcmc_taps);
        if (!(finite(p->rcmc_beta) && p->rcmc_beta >= 0.0 && p->rcmc_beta <= 20.0))
            return fail(SAR_ERR_BAD_PARAM, "rcmc_beta must be in [0, 20]");
    } else {
        return fail(SAR_ERR_BAD_PARAM, "az_model=%d unknown", p->az_model);
    }
    if (p->precision < SAR_FP32 || p->precision > SAR_FP32_HALF_STORAGE)
        return fail(SAR_ERR_BAD_PARAM, "precision=%d unknown", p->precision);
    if (p->schedule != SAR_FUSED && p->schedule != SAR_UNFUSED && p->schedule != SAR_TURN_FREE)
        return fail(SAR_ERR_BAD_PARAM, "schedule=%d unknown", p->schedule);
    if (p->schedule == SAR_TURN_FREE &&
        (p->precision != SAR_FP32 || p->transpose_back != 0 || p->Na > 4096))
        return fail(SAR_ERR_UNSUPPORTED,
                    "the turn-free schedule runs FP32 with Na <= 4096 and transpose_back = 0");
    if (p->transpose_back != 0 && p->transpose_back != 1)
        return fail(SAR_ERR_BAD_PARAM, "transpose_back must be 0 or 1");
    if (p->precision == SAR_FP32_HALF_STORAGE) {
        if (p->schedule != SAR_FUSED || p->transpose_back != 0)
            return fail(SAR_ERR_UNSUPPORTED, "half storage runs the fused schedule without transpose_back");
        if (p->az_model == SAR_AZ_HYPERBOLIC) {
            const double x = p->lambda * 0.5 / (2.0 * p->v);
            const double D = std::sqrt(1.0 - x * x);
            if (p->rcmc_taps != 8 || !(x * x / (D * (1.0 + D)) < 0.5))
                return fail(SAR_ERR_UNSUPPORTED, "half storage needs 8-tap RCMC with stretch < 0.5");
        }
    }
    return SAR_OK;
}

size_t scene_bytes(const sar_plan_s* P) { return (size_t)P->p.Na * (size_t)P->p.Nr * 8; }

sar_status check_plan(const sar_plan_s* P)
{
    if (!P) return fail(SAR_ERR_NULL, "plan is NULL");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != P->device)
        return fail(SAR_ERR_BAD_PARAM, "plan was built on device %d, current device is %d", P->device, dev);
    return SAR_OK;
}

sar_status check_ptr(const void* p, const char* name)
{
    if (!p) return fail(SAR_ERR_NULL, "%s is NULL", name);
    if (misaligned(p)) return fail(SAR_ERR_BAD_PARAM, "%s is not 16-byte aligned", name);
    return SAR_OK;
}

sar::RcmcHost rcmc_host(const sar_plan_s* P)
{
    sar::RcmcHost h{};
    h.stretch = P->stretch;
    h.rate = P->rate;
    h.table = P->rcmc_tab;
    h.r_near = P->p.r_near;
    h.stretch_max = P->stretch_max;
    h.x_per_bin = P->p.lambda / (2.0 * P->p.v * (double)P->p.Na);
    h.two_over_lam = 2.0 / P->p.lambda;
    h.taps = P->p.rcmc_taps;
    h.nr = P->p.Nr;
    return h;
}

using sar::LineOp;

}  // namespace

namespace sar {
RcmcHost plan_rcmc(const sar_plan_s* P) { return rcmc_host(P); }
}  // namespace sar

namespace {

// ---- steps (no validation; callers validated) ----
sar_status step_range(const sar_plan_s* P, const void* in, void* out, hipStream_t s)
{
    const int Nr = P->p.Nr, Na = P->p.Na;
    if (P->p.schedule != SAR_UNFUSED) {
        HIP_TRY(sar::launch_line(LineOp::Fused, Nr, in, out, Na, P->Hr, P->tw_r, 1.f, nullptr, arith(P),
                                 P->var_r[sar::TK_FUSED], s),
                "range fused launch");
    } else {
        HIP_TRY(sar::launch_line(LineOp::Forward, Nr, in, out, Na, nullptr, P->tw_r, 1.f, nullptr,
                                 arith(P), P->var_r[sar::TK_FWD], s),
                "range FFT launch");
        HIP_TRY(sar::launch_rowmul(out, out, Na, Nr, P->Hr, s), "range multiply launch");
        HIP_TRY(sar::launch_line(LineOp::Inverse, Nr, out, out, Na, nullptr, P->tw_r, 1.f, nullptr,
                                 arith(P), P->var_r[sar::TK_INV], s),
                "range IFFT launch");
    }
    return SAR_OK;
}

sar_status step_turn(const void* in, void* out, int rows, int cols, int variant, hipStream_t s)
{
    HIP_TRY(sar::launch_corner_turn(in, out, rows, cols, variant, s), "corner turn launch");
    return SAR_OK;
}

// Azimuth compression on [Nr][Na]: in -> out, `work` scratch (hyperbolic).
sar_status step_azimuth(const sar_plan_s* P, const void* in, void* out, void* work, hipStream_t s)
{
    const int Nr = P->p.Nr, Na = P->p.Na;
    if (P->p.az_model == SAR_AZ_LFM) {
        if (P->p.schedule != SAR_UNFUSED) {
            HIP_TRY(sar::launch_line(LineOp::Fused, Na, in, out, Nr, P->Ha, P->tw_a, 1.f, nullptr,
                                     arith(P), P->var_a[sar::TK_FUSED], s),
                    "azimuth fused launch");
        } else {
            HIP_TRY(sar::launch_line(LineOp::Forward, Na, in, out, Nr, nullptr, P->tw_a, 1.f, nullptr,
                                     arith(P), P->var_a[sar::TK_FWD], s),
                    "azimuth FFT launch");
            HIP_TRY(sar::launch_rowmul(out, out, Nr, Na, P->Ha, s), "azimuth multiply launch");
            HIP_TRY(sar::launch_line(LineOp::Inverse, Na, out, out, Nr, nullptr, P->tw_a, 1.f, nullptr,
                                     arith(P), P->var_a[sar::TK_INV], s),
                    "azimuth IFFT launch");
        }
        return SAR_OK;
    }
    const sar::RcmcHost rh = rcmc_host(P);
    HIP_TRY(sar::launch_line(LineOp::Forward, Na, in, work, Nr, nullptr, P->tw_a, 1.f, nullptr,
                             arith(P), P->var_a[sar::TK_FWD], s),
            "azimuth FFT launch");
    if (P->p.schedule != SAR_UNFUSED) {
        HIP_TRY(sar::launch_line(LineOp::RcmcAz, Na, work, out, Nr, nullptr, P->tw_a, 1.f, &rh,
                                 arith(P), P->var_a[sar::TK_RCMC], s),
                "RCMC+azimuth launch");
    } else {
        HIP_TRY(sar::launch_rcmc_interp(work, out, Na, rh, s), "RCMC launch");
        HIP_TRY(sar::launch_az_phase(out, out, Na, rh, 1.0f / (float)Na, s), "azimuth phase launch");
        HIP_TRY(sar::launch_line(LineOp::Inverse, Na, out, out, Nr, nullptr, P->tw_a, 1.f, nullptr,
                                     arith(P), P->var_a[sar::TK_INV], s),
                "azimuth IFFT launch");
    }
    return SAR_OK;
}

// Turn-free schedule: no corner turn.  The azimuth pass reads strips of
// adjacent azimuth lines straight from the range pass's [Na][Nr] output.
//   LFM:        raw -> range -> work [Na][Nr] -> strips FFT*H*IFFT -> img [Nr][Na]
//   hyperbolic: raw -> range -> img [Na][Nr] -> strips FFT -> work [Nr][Na]
//               -> RCMC*phase*IFFT -> img [Nr][Na]
sar_status execute_turn_free(const sar_plan_s* P, const void* raw, void* img, void* work,
                             hipStream_t s)
{
    const int Nr = P->p.Nr, Na = P->p.Na;
    sar_status st;
    if (P->p.az_model == SAR_AZ_LFM) {
        if ((st = step_range(P, raw, work, s))) return st;
        HIP_TRY(sar::launch_line_strip(true, Na, work, img, Nr, Nr, P->Ha, P->tw_a, 1.f, P->var_strip, s),
                "azimuth strip launch");
        return SAR_OK;
    }
    if ((st = step_range(P, raw, img, s))) return st;
    HIP_TRY(sar::launch_line_strip(false, Na, img, work, Nr, Nr, nullptr, P->tw_a, 1.f, P->var_strip,
                                   s),
            "azimuth strip FFT launch");
    const sar::RcmcHost rh = rcmc_host(P);
    HIP_TRY(sar::launch_line(LineOp::RcmcAz, Na, work, img, Nr, nullptr, P->tw_a, 1.f, &rh, arith(P),
                             P->var_a[sar::TK_RCMC], s),
            "RCMC+azimuth launch");
    return SAR_OK;
}

// Half storage (fused schedule): the intermediates live in the workspace as
// FP16 pairs with one power-of-two exponent per line (see half_layout):
//   range      raw (complex64) -> Wa [Na][Nr] FP16, E1[Na]
//   turn       Wa -> Wb [Nr][Na] FP16 (4-byte elements; point m keeps E1[m])
//   LFM:       azimuth FFT*H*IFFT  Wb -> img (complex64)
//   hyperbolic azimuth FFT  Wb -> Wa [Nr][Na] FP16, E2[Nr];
//              RCMC + phase + IFFT  Wa -> img (complex64)
sar_status execute_half(const sar_plan_s* P, const void* raw, void* img, void* work, hipStream_t s)
{
    const int Nr = P->p.Nr, Na = P->p.Na;
    const HalfLayout L = half_layout(Na, Nr);
    char* w = (char*)work;
    void* Wa = w + L.wa;
    void* Wb = w + L.wb;
    int* E1 = (int*)(w + L.e1);
    int* E2 = (int*)(w + L.e2);
    HIP_TRY(sar::launch_line_half(sar::HalfOp::RangeFused, Nr, raw, Wa, Na, P->Hr, P->tw_r, nullptr, E1, s),
            "range launch (half storage)");
    HIP_TRY(sar::launch_corner_turn_b4(Wa, Wb, Na, Nr, s), "corner turn launch (half storage)");
    if (P->p.az_model == SAR_AZ_LFM) {
        HIP_TRY(sar::launch_line_half(sar::HalfOp::AzimuthFused, Na, Wb, img, Nr, P->Ha, P->tw_a, E1, nullptr,
                                      s),
                "azimuth launch (half storage)");
        return SAR_OK;
    }
    HIP_TRY(sar::launch_line_half(sar::HalfOp::AzimuthForward, Na, Wb, Wa, Nr, nullptr, P->tw_a, E1, E2, s),
            "azimuth FFT launch (half storage)");
    HIP_TRY(sar::launch_rcmc_half(Na, Wa, E2, img, rcmc_host(P), P->tw_a, s), "RCMC launch (half storage)");
    return SAR_OK;
}

}  // namespace

extern "C" {

const char* sar_last_error(void) { return g_err.c_str(); }

const char* sar_version(void)
{
    return "sar_rda 0.2 (gfx950: FP32 and split FP16/BF16 MFMA, fused/unfused, batched, autotuned)";
}

sar_status sar_plan(const sar_params* p, void* stream, sar_plan_t* out)
{
    g_err.clear();
    if (!out) return fail(SAR_ERR_NULL, "out is NULL");
    *out = nullptr;
    sar_status st = validate_params(p);
    if (st != SAR_OK) return st;
    hipStream_t s = (hipStream_t)stream;

    sar_plan_s* P = new (std::nothrow) sar_plan_s;
    if (!P) return fail(SAR_ERR_NO_MEMORY, "host allocation of the plan failed");
    P->p = *p;
    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) {
        delete P;
        return hip_fail(e, "hipGetDevice");
    }
    const int Nr = p->Nr, Na = p->Na;
    const bool hyper = p->az_model == SAR_AZ_HYPERBOLIC;
    sar::load_tune_cache_once();
    const int ap = p->precision == SAR_FP32_HALF_STORAGE ? SAR_FP32 : p->precision;
    for (int k = 0; k < 3; ++k) P->var_r[k] = sar::tuned_variant(k, Nr, ap);
    for (int k = 0; k < 4; ++k) P->var_a[k] = sar::tuned_variant(k, Na, ap);
    P->var_turn = sar::tuned_variant(sar::TK_TURN, Nr, SAR_FP32);
    P->var_back = sar::tuned_variant(sar::TK_TURN, Na, SAR_FP32);
    P->var_strip = sar::tuned_variant(sar::TK_STRIP, Na, SAR_FP32);
    const size_t A = 256;
    size_t off = 0;
    const size_t o_twr = off; off = align_up(off + sizeof(float2) * (size_t)sar::twiddle_table_size(Nr), A);
    const size_t o_twa = off; off = align_up(off + sizeof(float2) * (size_t)sar::twiddle_table_size(Na), A);
    const size_t o_hr = off;  off = align_up(off + sizeof(float2) * (size_t)Nr, A);
    const size_t o_ha = off;  off = align_up(off + (hyper ? 0 : sizeof(float2) * (size_t)Na), A);
    const size_t o_st = off;  off = align_up(off + (hyper ? sizeof(double) * (size_t)Na : 0), A);
    const size_t o_rt = off;  off = align_up(off + (hyper ? sizeof(double) * (size_t)Na : 0), A);
    const size_t o_tb = off;  off = align_up(off + (hyper ? sizeof(float) * (size_t)sar::rcmc_table_floats() : 0), A);
    e = hipMalloc(&P->block, off);
    if (e != hipSuccess) {
        delete P;
        return fail(SAR_ERR_NO_MEMORY, "hipMalloc of %zu plan bytes failed: %s", off, hipGetErrorString(e));
    }
    char* b = (char*)P->block;
    P->tw_r = (float2*)(b + o_twr);
    P->tw_a = (float2*)(b + o_twa);
    P->Hr = (float2*)(b + o_hr);
    P->Ha = hyper ? nullptr : (float2*)(b + o_ha);
    P->stretch = hyper ? (double*)(b + o_st) : nullptr;
    P->rate = hyper ? (double*)(b + o_rt) : nullptr;
    P->rcmc_tab = hyper ? (float*)(b + o_tb) : nullptr;
    if (hyper) {
        const double x = p->lambda * 0.5 / (2.0 * p->v);
        const double D = std::sqrt(1.0 - x * x);
        P->stretch_max = x * x / (D * (1.0 + D));
    }

    auto cleanup_fail = [&](sar_status code) {
        (void)hipFree(P->block);
        delete P;
        return code;
    };
    if ((e = sar::launch_gen_twiddles(P->tw_r, Nr, s)) != hipSuccess ||
        (e = sar::launch_gen_twiddles(P->tw_a, Na, s)) != hipSuccess)
        return cleanup_fail(hip_fail(e, "twiddle generator"));
    const double Kr = p->range_tbp / ((double)p->range_len * (double)p->range_len);
    if ((e = sar::launch_gen_chirp_filter(P->Hr, Nr, p->range_len, Kr, +1, 1.0 / Nr, s)) != hipSuccess)
        return cleanup_fail(hip_fail(e, "range filter generator"));
    if (!hyper) {
        const double Ka = p->az_tbp / ((double)p->az_len * (double)p->az_len);
        if ((e = sar::launch_gen_chirp_filter(P->Ha, Na, p->az_len, Ka, -1, 1.0 / Na, s)) != hipSuccess)
            return cleanup_fail(hip_fail(e, "azimuth filter generator"));
    } else {
        if ((e = sar::launch_gen_hyper_tables(P->stretch, P->rate, Na, p->lambda, p->v, s)) != hipSuccess)
            return cleanup_fail(hip_fail(e, "hyperbolic table generator"));
        if ((e = sar::launch_gen_rcmc_table(P->rcmc_tab, p->rcmc_beta, s)) != hipSuccess)
            return cleanup_fail(hip_fail(e, "RCMC weight table generator"));
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup_fail(hip_fail(e, "plan synchronisation"));
    setup_noalloc_scratch(P->device);
    *out = P;
    return SAR_OK;
}

void sar_plan_destroy(sar_plan_t plan)
{
    if (!plan) return;
    (void)hipFree(plan->block);
    delete plan;
}

size_t sar_workspace_bytes(sar_plan_t plan)
{
    if (!plan) return 0;
    if (plan->p.precision == SAR_FP32_HALF_STORAGE) return half_layout(plan->p.Na, plan->p.Nr).total;
    return scene_bytes(plan);
}

sar_status sar_range_compress(sar_plan_t P, const void* in, void* out, void* stream)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P)) || (st = check_ptr(in, "in")) || (st = check_ptr(out, "out"))) return st;
    const size_t n = scene_bytes(P);
    if (in != out && overlap(in, n, out, n)) return fail(SAR_ERR_ALIAS, "in and out partially overlap");
    return step_range(P, in, out, (hipStream_t)stream);
}

sar_status sar_corner_turn(sar_plan_t P, const void* in, void* out, int32_t rows, int32_t cols,
                           void* stream)
{
    g_err.clear();
    sar_status st;
    if (P && (st = check_plan(P))) return st;
    if ((st = check_ptr(in, "in")) || (st = check_ptr(out, "out"))) return st;
    if (rows < 1 || cols < 1 || rows > (1 << 20) || cols > (1 << 20) ||
        (long long)rows * cols > (1LL << 31))
        return fail(SAR_ERR_BAD_SIZE, "rows=%d cols=%d out of range", rows, cols);
    const size_t n = (size_t)rows * (size_t)cols * 8;
    if (overlap(in, n, out, n)) return fail(SAR_ERR_ALIAS, "corner turn must be out of place");
    // a plan's own turns use its tuned grid; other shapes the default
    int v = 0;
    if (P && rows == P->p.Na && cols == P->p.Nr) v = P->var_turn;
    else if (P && rows == P->p.Nr && cols == P->p.Na) v = P->var_back;
    return step_turn(in, out, rows, cols, v, (hipStream_t)stream);
}

sar_status sar_azimuth_compress(sar_plan_t P, const void* in, void* out, void* work, void* stream)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P)) || (st = check_ptr(in, "in")) || (st = check_ptr(out, "out"))) return st;
    const size_t n = scene_bytes(P);
    if (in != out && overlap(in, n, out, n)) return fail(SAR_ERR_ALIAS, "in and out partially overlap");
    if (P->p.az_model == SAR_AZ_HYPERBOLIC) {
        if ((st = check_ptr(work, "work"))) return st;
        if (overlap(work, n, in, n) || overlap(work, n, out, n))
            return fail(SAR_ERR_ALIAS, "work overlaps in or out");
    }
    return step_azimuth(P, in, out, work, (hipStream_t)stream);
}

sar_status sar_rda_execute(sar_plan_t P, const void* raw, void* img, void* work, void* stream)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P)) || (st = check_ptr(raw, "raw")) || (st = check_ptr(img, "img")) ||
        (st = check_ptr(work, "work")))
        return st;
    const size_t n = scene_bytes(P), nw = sar_workspace_bytes(P);
    if (overlap(raw, n, img, n) || overlap(raw, n, work, nw) || overlap(img, n, work, nw))
        return fail(SAR_ERR_ALIAS, "raw, img and work must be pairwise disjoint");
    hipStream_t s = (hipStream_t)stream;
    if (P->p.precision == SAR_FP32_HALF_STORAGE) return execute_half(P, raw, img, work, s);
    if (P->p.schedule == SAR_TURN_FREE) return execute_turn_free(P, raw, img, work, s);
    const int Nr = P->p.Nr, Na = P->p.Na;
    const bool back = P->p.transpose_back != 0;
    // Buffers alternate so that the last step writes img.
    void* A = back ? img : work;     // range output [Na][Nr]
    void* B = back ? work : img;     // turned [Nr][Na]
    if ((st = step_range(P, raw, A, s))) return st;
    if ((st = step_turn(A, B, Na, Nr, P->var_turn, s))) return st;
    void* C;                          // azimuth output [Nr][Na]
    if (P->p.az_model == SAR_AZ_LFM) {
        C = B;                        // in place
        if ((st = step_azimuth(P, B, C, nullptr, s))) return st;
    } else {
        C = B;                        // FFT B -> A, RCMC A -> B
        if ((st = step_azimuth(P, B, C, A, s))) return st;
    }
    if (back) {
        if ((st = step_turn(C, C == img ? work : img, Nr, Na, P->var_back, s))) return st;
    }
    return SAR_OK;
}

sar_status sar_time_next_launches(void* const* start_events, void* const* stop_events, int32_t n)
{
    g_err.clear();
    g_time_next = g_time_count = 0;
    if (n == 0) return SAR_OK;
    if (n < 0 || n > MAX_TIMED)
        return fail(SAR_ERR_BAD_SIZE, "sar_time_next_launches: n=%d outside 0..%d", n, MAX_TIMED);
    if (!start_events || !stop_events) return fail(SAR_ERR_NULL, "sar_time_next_launches: NULL array");
    for (int i = 0; i < n; ++i)
        if (!start_events[i] || !stop_events[i])
            return fail(SAR_ERR_NULL, "sar_time_next_launches: event %d is NULL", i);
    for (int i = 0; i < n; ++i) {
        g_time_start[i] = (hipEvent_t)start_events[i];
        g_time_stop[i] = (hipEvent_t)stop_events[i];
    }
    g_time_count = n;
    return SAR_OK;
}

sar_status sar_rda_execute_noalloc(sar_plan_t P, const void* raw, void* img, void* stream)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P))) return st;
    const size_t need = sar_workspace_bytes(P);
    if (need > SAR_NOALLOC_WORKSPACE_BYTES)
        return fail(SAR_ERR_BAD_SIZE,
                    "sar_rda_execute_noalloc: the plan needs %zu workspace bytes, the library's "
                    "static workspace holds %zu (use sar_rda_execute with a workspace)",
                    need, (size_t)SAR_NOALLOC_WORKSPACE_BYTES);
    void* ptr = nullptr;
    hipError_t e = hipSuccess;
    if (P->device >= 0 && P->device < MAX_DEVICES) {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        ptr = g_scratch_ptr[P->device];
        e = g_scratch_err[P->device];
    }
    if (!ptr)
        return fail(SAR_ERR_HIP, "sar_rda_execute_noalloc: no static workspace on device %d (%s)",
                    P->device, e != hipSuccess ? hipGetErrorString(e) : "set-up did not run");
    return sar_rda_execute(P, raw, img, ptr, stream);
}

sar_status sar_fft_lines(sar_plan_t P, int32_t axis, int32_t inverse, const void* in, void* out,
                         int32_t lines, void* stream)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P)) || (st = check_ptr(in, "in")) || (st = check_ptr(out, "out"))) return st;
    if (axis != 0 && axis != 1) return fail(SAR_ERR_BAD_PARAM, "axis must be 0 (range) or 1 (azimuth)");
    if (inverse != 0 && inverse != 1) return fail(SAR_ERR_BAD_PARAM, "inverse must be 0 or 1");
    if (lines < 0) return fail(SAR_ERR_BAD_SIZE, "lines < 0");
    const int N = axis == 0 ? P->p.Nr : P->p.Na;
    const size_t n = (size_t)lines * N * 8;
    if (in != out && overlap(in, n, out, n)) return fail(SAR_ERR_ALIAS, "in and out partially overlap");
    HIP_TRY(sar::launch_line(inverse ? LineOp::Inverse : LineOp::Forward, N, in, out, lines, nullptr,
                             axis == 0 ? P->tw_r : P->tw_a, inverse ? 1.0f / (float)N : 1.0f, nullptr,
                             arith(P), (axis == 0 ? P->var_r : P->var_a)[inverse ? sar::TK_INV : sar::TK_FWD],
                             (hipStream_t)stream),
            "FFT launch");
    return SAR_OK;
}

sar_status sar_azimuth_fft(sar_plan_t P, const void* in, void* out, void* stream)
{
    if (!P) {
        g_err.clear();
        return fail(SAR_ERR_NULL, "plan is NULL");
    }
    return sar_fft_lines(P, 1, 0, in, out, P->p.Nr, stream);
}

sar_status sar_rcmc_azimuth(sar_plan_t P, const void* A, void* out, void* stream)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P)) || (st = check_ptr(A, "A")) || (st = check_ptr(out, "out"))) return st;
    if (P->p.az_model != SAR_AZ_HYPERBOLIC)
        return fail(SAR_ERR_BAD_PARAM, "sar_rcmc_azimuth needs a hyperbolic plan");
    const size_t n = scene_bytes(P);
    if (overlap(A, n, out, n)) return fail(SAR_ERR_ALIAS, "A and out must not overlap");
    const sar::RcmcHost rh = rcmc_host(P);
    hipStream_t s = (hipStream_t)stream;
    if (P->p.schedule == SAR_FUSED) {
        HIP_TRY(sar::launch_line(LineOp::RcmcAz, P->p.Na, A, out, P->p.Nr, nullptr, P->tw_a, 1.f, &rh,
                                 arith(P), P->var_a[sar::TK_RCMC], s),
                "RCMC+azimuth launch");
    } else {
        HIP_TRY(sar::launch_rcmc_interp(A, out, P->p.Na, rh, s), "RCMC launch");
        HIP_TRY(sar::launch_az_phase(out, out, P->p.Na, rh, 1.0f / (float)P->p.Na, s), "phase launch");
        HIP_TRY(sar::launch_line(LineOp::Inverse, P->p.Na, out, out, P->p.Nr, nullptr, P->tw_a, 1.f,
                                 nullptr, arith(P), P->var_a[sar::TK_INV], s),
                "azimuth IFFT launch");
    }
    return SAR_OK;
}

sar_status sar_plan_get_table(sar_plan_t P, int32_t which, void* host, size_t bytes)
{
    g_err.clear();
    sar_status st;
    if ((st = check_plan(P))) return st;
    if (!host) return fail(SAR_ERR_NULL, "host_dst is NULL");
    const void* src = nullptr;
    size_t need = 0;
    switch (which) {
    case 0: src = P->Hr; need = sizeof(float2) * (size_t)P->p.Nr; break;
    case 1: src = P->Ha; need = sizeof(float2) * (size_t)P->p.Na; break;
    case 2: src = P->stretch; need = sizeof(double) * (size_t)P->p.Na; break;
    case 3: src = P->rate; need = sizeof(double) * (size_t)P->p.Na; break;
    case 4: src = P->rcmc_tab; need = sizeof(float) * (size_t)sar::rcmc_table_floats(); break;
    default: return fail(SAR_ERR_BAD_PARAM, "table %d unknown", which);
    }
    if (!src) return fail(SAR_ERR_BAD_PARAM, "table %d does not exist for this azimuth model", which);
    if (bytes < need) return fail(SAR_ERR_BAD_SIZE, "host buffer holds %zu bytes, need %zu", bytes, need);
    HIP_TRY(hipMemcpy(host, src, need, hipMemcpyDeviceToHost), "table copy");
    return SAR_OK;
}

}  // extern "C"

// rda_tune.cpp -- the autotuner: measured choice of kernel variants.
//
// Tuned per (kernel kind, line length, precision):
//   line kernels (fused FFT*H*IFFT, forward, inverse):  twiddles computed by
//       products of two table loads per radix-16 pass, or read from the table
//       (FP32 butterflies only; the MFMA variants share one scheme);
//   RCMC + azimuth kernel: the same twiddle choice for its IFFT, and two
//       output rows per workgroup (shared interpolation gathers; on one or
//       on two line slots' threads) or one row;
//   batched fused line kernel: twiddles and the grid (one workgroup per line
//       group, or a persistent grid of 1x, 2x or 4x the resident workgroups).
// Every candidate computes the same result (they differ in instruction mix and
// scheduling only); the tests check each one against the oracle.
//
// Cache: a JSON-lines text file, one object per tuned kernel, e.g.
//   {"arch":"gfx950","kind":"fused","n":4096,"prec":0,"variant":1,
//    "us_default":64.1,"us_best":61.9}
// Lines for other architectures are kept; malformed or out-of-range lines are
// skipped.  A new result replaces the line with the same key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "rda_internal.h"
#include "sar_rda.h"

namespace {

const char* const KIND_NAME[] = {"fused", "fwd", "inv", "rcmc", "batch_fused", "turn", "strip"};
constexpr int NKIND = 7;

struct Key {
    int kind, n, prec;
    bool operator<(const Key& o) const
    {
        return std::tie(kind, n, prec) < std::tie(o.kind, o.n, o.prec);
    }
};

std::mutex g_mu;
std::map<Key, int> g_table;
std::once_flag g_env_once;

// Variants a cache entry may select.  Split precisions have the default
// kernels plus the one-row RCMC kernel only: table twiddles, the split
// exchange layout and the wide RCMC kernel are FP32 kernels, and the
// persistent batch grids spill in the split transforms (never faster).
// The corner turn (grid of five or four workgroups per CU, or one per tile)
// and the turn-free strips (default or half width) are keyed as FP32.
bool valid_variant(int kind, int prec, int v)
{
    if (kind == sar::TK_TURN) return prec == SAR_FP32 && v >= 0 && v <= 2;
    if (kind == sar::TK_STRIP) return prec == SAR_FP32 && (v == 0 || v == 1);
    if (prec != SAR_FP32) return v == 0 || (kind == sar::TK_RCMC && v == 2);
    switch (kind) {
    case sar::TK_FUSED: return v == 0 || v == 1 || v == 4 || v == 5;
    case sar::TK_FWD:
    case sar::TK_INV: return v >= 0 && v <= 7;
    case sar::TK_RCMC: return v >= 0 && v <= 7;
    case sar::TK_BATCH_FUSED: return v >= 0 && v <= 15 && (v & 2) == 0;
    default: return false;
    }
}

bool valid_n(int n) { return n >= 64 && n <= 16384 && (n & (n - 1)) == 0; }

// Value of "key": as a string or an integer on one JSON line (flat objects only).
bool json_str(const std::string& line, const char* key, std::string& out)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return false;
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return false;
    p = line.find('"', p);
    if (p == std::string::npos) return false;
    const size_t e = line.find('"', p + 1);
    if (e == std::string::npos) return false;
    out = line.substr(p + 1, e - p - 1);
    return true;
}

bool json_int(const std::string& line, const char* key, long& out)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return false;
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return false;
    const char* c = line.c_str() + p + 1;
    char* end = nullptr;
    out = std::strtol(c, &end, 10);
    return end != c;
}

struct Entry {
    std::string arch;
    Key key;
    int variant;
    std::string line;   // the original text
};

// Parse one cache line; false if it is not a valid entry.
bool parse_line(const std::string& line, Entry& e)
{
    std::string kind;
    long n = 0, prec = 0, v = 0;
    if (!json_str(line, "arch", e.arch) || !json_str(line, "kind", kind) ||
        !json_int(line, "n", n) || !json_int(line, "prec", prec) || !json_int(line, "variant", v))
        return false;
    int k = -1;
    for (int i = 0; i < NKIND; ++i)
        if (kind == KIND_NAME[i]) k = i;
    if (k < 0 || !valid_n((int)n) || prec < SAR_FP32 || prec > SAR_SPLIT_BF16 ||
        !valid_variant(k, (int)prec, (int)v))
        return false;
    e.key = Key{k, (int)n, (int)prec};
    e.variant = (int)v;
    e.line = line;
    return true;
}

std::vector<Entry> read_cache(const char* path, bool& found)
{
    std::vector<Entry> out;
    std::ifstream f(path);
    found = (bool)f;
    std::string line;
    while (std::getline(f, line)) {
        Entry e;
        if (parse_line(line, e)) out.push_back(e);
    }
    return out;
}

// gcnArchName up to the first ':' ("gfx950:sramecc+:xnack-" -> "gfx950").
sar_status device_arch(std::string& arch)
{
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return sar::set_error(SAR_ERR_HIP, "device properties: %s", hipGetErrorString(e));
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    return SAR_OK;
}

int load_into_table(const char* path, const std::string& arch, bool& found)
{
    const std::vector<Entry> es = read_cache(path, found);
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
    int used = 0;
    for (const Entry& e : es)
        if (e.arch == arch) {
            g_table[e.key] = e.variant;
            ++used;
        }
    return used;
}

// ---- measurement ----

struct Candidate {
    int variant;
    float best_ms;
};

template <class Launch>
sar_status time_candidates(std::vector<Candidate>& cs, Launch&& launch, hipStream_t s)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return sar::set_error(SAR_ERR_HIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return sar::set_error(SAR_ERR_HIP, "hipEventCreate");
    }
    sar_status st = SAR_OK;
    const int reps = 8, rounds = 5;
    for (Candidate& c : cs) c.best_ms = 1e30f;
    for (int r = 0; r < rounds + 1 && st == SAR_OK; ++r) {
        // candidates interleaved per round, so cache warmth is shared fairly;
        // round 0 is warm-up
        for (Candidate& c : cs) {
            hipError_t e = hipEventRecord(e0, s);
            for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch(c.variant);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = sar::set_error(SAR_ERR_HIP, "autotune launch: %s", hipGetErrorString(e));
                break;
            }
            if (r > 0) c.best_ms = std::min(c.best_ms, ms / reps);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

struct Result {
    Key key;
    int variant;
    float us_default, us_best;
};

// Default (variant 0) unless a candidate is at least 2% faster.
Result pick(const Key& k, const std::vector<Candidate>& cs)
{
    Result r{k, 0, cs[0].best_ms * 1e3f, cs[0].best_ms * 1e3f};
    for (const Candidate& c : cs)
        if (c.best_ms * 1e3f < 0.98f * r.us_default && c.best_ms * 1e3f < r.us_best) {
            r.variant = c.variant;
            r.us_best = c.best_ms * 1e3f;
        }
    return r;
}

std::string format_entry(const std::string& arch, const Result& r)
{
    char buf[256];
    snprintf(buf, sizeof buf,
             "{\"arch\":\"%s\",\"kind\":\"%s\",\"n\":%d,\"prec\":%d,\"variant\":%d,"
             "\"us_default\":%.2f,\"us_best\":%.2f}",
             arch.c_str(), KIND_NAME[r.key.kind], r.key.n, r.key.prec, r.variant, r.us_default,
             r.us_best);
    return buf;
}

sar_status write_cache(const char* path, const std::string& arch, const std::vector<Result>& rs)
{
    bool found = false;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        found = (bool)f;
        std::string line;
        while (std::getline(f, line)) {
            Entry e;
            if (!parse_line(line, e)) continue;
            bool replaced = false;
            for (const Result& r : rs)
                if (e.arch == arch && !(e.key < r.key) && !(r.key < e.key)) replaced = true;
            if (!replaced) keep.push_back(line);
        }
    }
    (void)found;
    for (const Result& r : rs) keep.push_back(format_entry(arch, r));
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return sar::set_error(SAR_ERR_BAD_PARAM, "cannot write %s", tmp.c_str());
        for (const std::string& l : keep) o << l << "\n";
        if (!o) return sar::set_error(SAR_ERR_BAD_PARAM, "write to %s failed", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return sar::set_error(SAR_ERR_BAD_PARAM, "cannot rename %s to %s", tmp.c_str(), path);
    return SAR_OK;
}

}  // namespace

namespace sar {

int tuned_variant(int kind, int n, int prec)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_table.find(Key{kind, n, prec});
    return it == g_table.end() ? 0 : it->second;
}

void load_tune_cache_once()
{
    std::call_once(g_env_once, [] {
        const char* path = std::getenv("SAR_AUTOTUNE_CACHE");
        if (!path || !*path) return;
        std::string arch;
        if (device_arch(arch) != SAR_OK) return;
        bool found = false;
        (void)load_into_table(path, arch, found);
    });
}

}  // namespace sar

extern "C" {

sar_status sar_tune_load(const char* path, const char* arch)
{
    sar::clear_error();
    // the environment cache must not later overwrite what is loaded here
    std::call_once(g_env_once, [] {});
    if (!path) {
        std::lock_guard<std::mutex> g(g_mu);
        g_table.clear();
        return SAR_OK;
    }
    std::string a;
    if (arch) {
        a = arch;
    } else {
        sar_status st = device_arch(a);
        if (st != SAR_OK) return st;
    }
    bool found = false;
    (void)load_into_table(path, a, found);
    if (!found) return sar::set_error(SAR_ERR_BAD_PARAM, "cannot read %s", path);
    return SAR_OK;
}

int32_t sar_tune_variant(int32_t kind, int32_t n, int32_t precision)
{
    if (kind < 0 || kind >= NKIND) return -1;
    return sar::tuned_variant(kind, n, precision);
}

sar_status sar_autotune(const sar_params* p, const char* cache_path)
{
    sar::clear_error();
    sar_plan_t P = nullptr;
    sar_status st = sar_plan(p, nullptr, &P);
    if (st != SAR_OK) return st;
    std::string arch;
    if ((st = device_arch(arch)) != SAR_OK) {
        sar_plan_destroy(P);
        return st;
    }
    // half storage computes in FP32: its line kernels are tuned as FP32
    const int Nr = p->Nr, Na = p->Na,
              prec = p->precision == SAR_FP32_HALF_STORAGE ? SAR_FP32 : p->precision;
    const bool fp32 = prec == SAR_FP32;
    const bool hyper = p->az_model == SAR_AZ_HYPERBOLIC;
    const bool fused = p->schedule != SAR_UNFUSED;   // turn-free runs the fused kernels
    const size_t bytes = (size_t)Na * (size_t)Nr * 8;
    void *in = nullptr, *out = nullptr, *task = nullptr;
    hipStream_t s = nullptr;
    auto done = [&](sar_status code) {
        if (s) (void)hipStreamSynchronize(s);
        if (in) (void)hipFree(in);
        if (out) (void)hipFree(out);
        if (task) (void)hipFree(task);
        if (s) (void)hipStreamDestroy(s);
        sar_plan_destroy(P);
        return code;
    };
    if (hipMalloc(&in, bytes) != hipSuccess || hipMalloc(&out, bytes) != hipSuccess ||
        hipMalloc(&task, sizeof(sar::LineTask)) != hipSuccess)
        return done(sar::set_error(SAR_ERR_NO_MEMORY, "autotune buffers (2 x %zu bytes)", bytes));
    if (hipStreamCreate(&s) != hipSuccess) return done(sar::set_error(SAR_ERR_HIP, "hipStreamCreate"));
    // finite data: the kernels' timing does not depend on the values
    if (hipMemsetAsync(in, 0, bytes, s) != hipSuccess)
        return done(sar::set_error(SAR_ERR_HIP, "hipMemsetAsync"));

    const sar::PlanTables tb = sar::plan_tables(P);
    std::vector<Result> results;
    auto tune_line = [&](int kind, int n, int lines, const void* H, const void* tw) -> sar_status {
        for (const Result& r : results)
            if (r.key.kind == kind && r.key.n == n) return SAR_OK;
        std::vector<Candidate> cs{{0, 0.f}};
        if (fp32) cs.push_back({1, 0.f});
        if (fp32 && kind != sar::TK_FUSED) {          // split real/imaginary exchange layout
            cs.push_back({2, 0.f});
            cs.push_back({3, 0.f});
        }
        if (fp32 && n <= 8192) {                      // twice the lines per workgroup
            const size_t base = cs.size();
            for (size_t i = 0; i < base; ++i) cs.push_back({cs[i].variant | 4, 0.f});
        }
        const sar::LineOp op = kind == sar::TK_FUSED ? sar::LineOp::Fused
                               : kind == sar::TK_FWD ? sar::LineOp::Forward
                                                     : sar::LineOp::Inverse;
        sar_status r = time_candidates(
            cs, [&](int v) { return sar::launch_line(op, n, in, out, lines, H, tw, 1.f, nullptr, prec, v, s); },
            s);
        if (r == SAR_OK) results.push_back(pick(Key{kind, n, prec}, cs));
        return r;
    };
    auto tune_batch = [&](int n, int lines, const void* H, const void* tw) -> sar_status {
        for (const Result& r : results)
            if (r.key.kind == sar::TK_BATCH_FUSED && r.key.n == n) return SAR_OK;
        sar::LineTask t{};
        t.in = (const float2*)in;
        t.out = (float2*)out;
        t.H = (const float2*)H;
        t.tw = (const float2*)tw;
        t.lines = lines;
        t.group_begin = 0;
        if (hipMemcpy(task, &t, sizeof t, hipMemcpyHostToDevice) != hipSuccess)
            return sar::set_error(SAR_ERR_HIP, "task upload");
        const int groups = sar::line_groups(n, lines);
        std::vector<Candidate> cs;
        for (int g = 0; g < (fp32 ? 4 : 1); ++g)
            for (int tw_tab = 0; tw_tab < (fp32 ? 2 : 1); ++tw_tab) cs.push_back({tw_tab | (g << 2), 0.f});
        sar_status r = time_candidates(
            cs,
            [&](int v) { return sar::launch_line_batch(0, n, task, 1, groups, 1.f, prec, v, s); }, s);
        if (r == SAR_OK) results.push_back(pick(Key{sar::TK_BATCH_FUSED, n, prec}, cs));
        return r;
    };

    // range pass
    if (fused) st = tune_line(sar::TK_FUSED, Nr, Na, tb.Hr, tb.tw_r);
    else if ((st = tune_line(sar::TK_FWD, Nr, Na, nullptr, tb.tw_r)) == SAR_OK)
        st = tune_line(sar::TK_INV, Nr, Na, nullptr, tb.tw_r);
    if (st != SAR_OK) return done(st);
    // azimuth pass
    if (!hyper) {
        if (fused) st = tune_line(sar::TK_FUSED, Na, Nr, tb.Ha, tb.tw_a);
        else if ((st = tune_line(sar::TK_FWD, Na, Nr, nullptr, tb.tw_a)) == SAR_OK)
            st = tune_line(sar::TK_INV, Na, Nr, nullptr, tb.tw_a);
    } else {
        st = tune_line(sar::TK_FWD, Na, Nr, nullptr, tb.tw_a);
        if (st == SAR_OK && !fused) st = tune_line(sar::TK_INV, Na, Nr, nullptr, tb.tw_a);
        if (st == SAR_OK && fused) {
            const sar::RcmcHost rh = sar::plan_rcmc(P);
            std::vector<Candidate> cs;
            for (int v = 0; v < 8; ++v) {
                if (!fp32 && (v & 5)) continue;           // table twiddles / wide: FP32 only
                if ((v & 4) && ((v & 2) || (Na != 4096 && Na != 8192))) continue;   // no effect
                cs.push_back({v, 0.f});
            }
            st = time_candidates(
                cs,
                [&](int v) {
                    return sar::launch_line(sar::LineOp::RcmcAz, Na, in, out, Nr, nullptr, tb.tw_a, 1.f,
                                            &rh, prec, v, s);
                },
                s);
            if (st == SAR_OK) results.push_back(pick(Key{sar::TK_RCMC, Na, prec}, cs));
        }
    }
    if (st != SAR_OK) return done(st);
    // the corner turn(s) of the turned schedules (the half-storage turn moves
    // FP16 pairs and has no variants)
    auto tune_turn = [&](int rows, int cols) -> sar_status {
        for (const Result& r : results)
            if (r.key.kind == sar::TK_TURN && r.key.n == cols) return SAR_OK;
        std::vector<Candidate> cs{{0, 0.f}, {1, 0.f}, {2, 0.f}};
        sar_status r = time_candidates(
            cs, [&](int v) { return sar::launch_corner_turn(in, out, rows, cols, v, s); }, s);
        if (r == SAR_OK) results.push_back(pick(Key{sar::TK_TURN, cols, SAR_FP32}, cs));
        return r;
    };
    if (p->precision != SAR_FP32_HALF_STORAGE) {
        if (p->schedule != SAR_TURN_FREE) st = tune_turn(Na, Nr);
        if (st == SAR_OK && p->transpose_back) st = tune_turn(Nr, Na);
        if (st != SAR_OK) return done(st);
    }
    // the turn-free azimuth strips
    if (p->schedule == SAR_TURN_FREE && fp32 && Na <= 4096) {
        std::vector<Candidate> cs{{0, 0.f}, {1, 0.f}};
        st = time_candidates(
            cs,
            [&](int v) {
                return sar::launch_line_strip(!hyper, Na, in, out, Nr, Nr, hyper ? nullptr : tb.Ha,
                                              tb.tw_a, 1.f, v, s);
            },
            s);
        if (st != SAR_OK) return done(st);
        results.push_back(pick(Key{sar::TK_STRIP, Na, SAR_FP32}, cs));
    }
    // the batched fused line kernel (LFM fused scenes are batched)
    if (!hyper && fused) {
        if ((st = tune_batch(Nr, Na, tb.Hr, tb.tw_r)) == SAR_OK) st = tune_batch(Na, Nr, tb.Ha, tb.tw_a);
        if (st != SAR_OK) return done(st);
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (const Result& r : results) g_table[r.key] = r.variant;
    }
    const char* path = cache_path ? cache_path : std::getenv("SAR_AUTOTUNE_CACHE");
    if (path && *path) st = write_cache(path, arch, results);
    return done(st);
}

}  // extern "C"

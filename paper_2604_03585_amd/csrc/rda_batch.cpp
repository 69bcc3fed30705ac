// rda_batch.cpp -- batched execution of scenes of uneven size.
//
// All scenes of a batch share launches: one batched line launch per
// (stage, line length) covering every scene with that length, one batched
// corner turn for all scenes, so 64 scenes of 5 x 5 sizes take about a dozen
// launches instead of ~200, and small scenes fill the GPU together.  Each
// launch is a grid over the scenes' line groups (task lists in device memory,
// see LineTask / TurnTask).  On a non-null stream the whole sequence is
// captured once into a hipGraph per set of buffers and replayed; a new set of
// buffer pointers rebuilds the tasks and the graph.
//
// Scenes whose processing the batched launches do not cover (hyperbolic
// azimuth, the unfused schedule, half storage) and scenes large enough to
// fill the chip alone (see kShareBelowPx) run through sar_rda_execute inside
// the same stream (and graph); the large fused FP32 ones that the turn-free
// kernels cover run those (bit-identical, without the corner turn).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "rda_internal.h"
#include "sar_rda.h"

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct Launch {
    int type;          // 0 line batch, 1 corner-turn batch
    int kind;          // line kind (0 fused)
    int n;             // line length
    int prec;
    int variant;       // tuned line-kernel variant (line batches)
    size_t task_off;   // byte offset of the task array in the device task buffer
    int ntasks;
    int total;         // groups or tiles
};

bool same_params(const sar_params& a, const sar_params& b) { return std::memcmp(&a, &b, sizeof a) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    auto pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

struct sar_batch_s {
    std::vector<sar_params> params;        // per scene
    std::vector<sar_plan_t> plans;         // distinct parameter sets
    std::vector<int> plan_of;              // per scene: index into plans
    std::vector<size_t> work_off;          // per scene: workspace byte offset
    size_t work_bytes = 0;
    int device = 0;
    // execution state for the last buffer set
    std::vector<const void*> raw_key;
    std::vector<void*> img_key;
    void* work_key = nullptr;
    void* stream_key = nullptr;
    bool built = false;
    void* dev_tasks = nullptr;
    size_t dev_tasks_cap = 0;
    std::vector<Launch> launches;
    std::vector<int> fallback;             // scenes run through sar_rda_execute
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(sar_batch_s* B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

// A scene of 4 Mpx or more fills the chip with its own launches (at least
// 1024 line groups per pass), and run pass after pass it re-reads the
// previous pass's output from the 256 MiB MALL when it is no larger than
// that; sharing launches with other scenes would only separate its passes.
// Such scenes run as sar_rda_execute, in scene order, inside the same
// stream (and graph); the smaller ones share launches.
constexpr long long kShareBelowPx = 1LL << 22;

bool batched(const sar_params& p)
{
    return p.az_model == SAR_AZ_LFM && p.schedule == SAR_FUSED && p.precision != SAR_FP32_HALF_STORAGE &&
           (long long)p.Na * p.Nr < kShareBelowPx;
}

// The parameters a scene's own plan is built with.  A fused FP32 scene that
// runs alone (4 Mpx or more) and that the turn-free kernels cover (Na <=
// 4096, no back-turn) runs them: the same image bit for bit, without its
// corner turn (32 instead of 48 B/px for LFM, 48 instead of 64 hyperbolic).
sar_params own_plan_params(const sar_params& p)
{
    sar_params q = p;
    if (p.schedule == SAR_FUSED && p.precision == SAR_FP32 && p.transpose_back == 0 &&
        p.Na <= 4096 && (long long)p.Na * p.Nr >= kShareBelowPx)
        q.schedule = SAR_TURN_FREE;
    return q;
}

// Build task arrays for this buffer set and upload them (synchronous).
sar_status build(sar_batch_s* B, const void* const* raw, void* const* img, void* work)
{
    const int n = (int)B->params.size();
    std::vector<char> host;
    std::vector<Launch> launches;
    B->fallback.clear();
    // per scene: range output A, turned B (as in sar_rda_execute)
    std::vector<void*> A(n), Bt(n);
    for (int i = 0; i < n; ++i) {
        void* w = (char*)work + B->work_off[i];
        const bool back = B->params[i].transpose_back != 0;
        A[i] = back ? img[i] : w;
        Bt[i] = back ? w : img[i];
        if (!batched(B->params[i])) B->fallback.push_back(i);
    }
    auto add_line_stage = [&](bool range_stage, const std::vector<int>& scenes) {
        // group the scenes by (line length, precision)
        std::map<std::pair<int, int>, std::vector<int>> groups;
        for (int i : scenes) {
            const int len = range_stage ? B->params[i].Nr : B->params[i].Na;
            groups[{len, B->params[i].precision}].push_back(i);
        }
        for (auto& kv : groups) {
            Launch L{0, 0, kv.first.first, kv.first.second,
                     sar::tuned_variant(sar::TK_BATCH_FUSED, kv.first.first, kv.first.second),
                     host.size(), 0, 0};
            for (int i : kv.second) {
                sar_plan_t P = B->plans[B->plan_of[i]];
                sar::LineTask t{};
                const sar::PlanTables tb = sar::plan_tables(P);
                if (range_stage) {
                    t.in = (const float2*)raw[i];
                    t.out = (float2*)A[i];
                    t.H = (const float2*)tb.Hr;
                    t.tw = (const float2*)tb.tw_r;
                    t.lines = B->params[i].Na;
                } else {
                    t.in = (const float2*)Bt[i];
                    t.out = (float2*)Bt[i];
                    t.H = (const float2*)tb.Ha;
                    t.tw = (const float2*)tb.tw_a;
                    t.lines = B->params[i].Nr;
                }
                t.group_begin = L.total;
                L.total += sar::line_groups(L.n, t.lines);
                const char* b = (const char*)&t;
                host.insert(host.end(), b, b + sizeof t);
                ++L.ntasks;
            }
            launches.push_back(L);
            host.resize(align256(host.size()));
        }
    };
    auto add_turn_stage = [&](bool back_turn, const std::vector<int>& scenes) -> sar_status {
        Launch L{1, 0, 0, 0, 0, host.size(), 0, 0};
        for (int i : scenes) {
            const sar_params& p = B->params[i];
            if (back_turn && !p.transpose_back) continue;
            sar::TurnTask t{};
            if (!back_turn) {
                t.in = (const float2*)A[i];
                t.out = (float2*)Bt[i];
                t.rows = p.Na;
                t.cols = p.Nr;
            } else {                                   // [Nr][Na] in work -> img
                t.in = (const float2*)Bt[i];
                t.out = (float2*)img[i];
                t.rows = p.Nr;
                t.cols = p.Na;
            }
            if (t.rows % 64 != 0 || t.cols % 64 != 0 || (((uintptr_t)t.in | (uintptr_t)t.out) & 15u))
                return sar::set_error(SAR_ERR_BAD_PARAM, "scene %d: batched turn needs whole 64 x 64 tiles "
                                      "and 16-byte aligned buffers", i);
            t.tile_begin = L.total;
            L.total += sar::turn_tiles(t.rows, t.cols);
            const char* b = (const char*)&t;
            host.insert(host.end(), b, b + sizeof t);
            ++L.ntasks;
        }
        if (L.ntasks) launches.push_back(L);
        host.resize(align256(host.size()));
        return SAR_OK;
    };
    std::vector<int> scenes;
    for (int i = 0; i < n; ++i)
        if (batched(B->params[i])) scenes.push_back(i);
    add_line_stage(true, scenes);
    sar_status st = add_turn_stage(false, scenes);
    if (st != SAR_OK) return st;
    add_line_stage(false, scenes);
    if ((st = add_turn_stage(true, scenes)) != SAR_OK) return st;

    if (host.size() > B->dev_tasks_cap) {
        if (B->dev_tasks) (void)hipFree(B->dev_tasks);
        B->dev_tasks = nullptr;
        B->dev_tasks_cap = 0;
        if (hipMalloc(&B->dev_tasks, host.size()) != hipSuccess)
            return sar::set_error(SAR_ERR_NO_MEMORY, "batch task buffer (%zu bytes)", host.size());
        B->dev_tasks_cap = host.size();
    }
    if (!host.empty()) {
        const hipError_t e = hipMemcpy(B->dev_tasks, host.data(), host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return sar::set_error(SAR_ERR_HIP, "task upload: %s", hipGetErrorString(e));
    }
    B->launches = launches;
    return SAR_OK;
}

sar_status enqueue(sar_batch_s* B, const void* const* raw, void* const* img, void* work,
                   hipStream_t s)
{
    for (const Launch& L : B->launches) {
        const char* tasks = (const char*)B->dev_tasks + L.task_off;
        hipError_t e = L.type == 0
                           ? sar::launch_line_batch(L.kind, L.n, tasks, L.ntasks, L.total, 1.0f, L.prec,
                                                    L.variant, s)
                           : sar::launch_corner_turn_batch(tasks, L.ntasks, L.total, s);
        if (e != hipSuccess) return sar::set_error(SAR_ERR_HIP, "batched launch: %s", hipGetErrorString(e));
    }
    for (int i : B->fallback) {
        sar_status st = sar_rda_execute(B->plans[B->plan_of[i]], raw[i], img[i],
                                        (char*)work + B->work_off[i], s);
        if (st != SAR_OK) return st;
    }
    return SAR_OK;
}

}  // namespace

extern "C" {

sar_status sar_batch_plan(const sar_params* ps, int32_t n, void* stream, sar_batch_t* out)
{
    sar::clear_error();
    if (!out) return sar::set_error(SAR_ERR_NULL, "out is NULL");
    *out = nullptr;
    if (!ps) return sar::set_error(SAR_ERR_NULL, "params array is NULL");
    if (n < 1) return sar::set_error(SAR_ERR_BAD_SIZE, "batch of %d scenes", n);
    sar_batch_s* B = new (std::nothrow) sar_batch_s;
    if (!B) return sar::set_error(SAR_ERR_NO_MEMORY, "host allocation of the batch failed");
    (void)hipGetDevice(&B->device);
    std::vector<sar_params> distinct;
    for (int i = 0; i < n; ++i) {
        int idx = -1;
        for (size_t j = 0; j < distinct.size(); ++j)
            if (same_params(distinct[j], ps[i])) idx = (int)j;
        if (idx < 0) {
            sar_plan_t P = nullptr;
            const sar_params q = own_plan_params(ps[i]);
            sar_status st = sar_plan(&q, stream, &P);
            if (st != SAR_OK) {
                for (auto q : B->plans) sar_plan_destroy(q);
                delete B;
                return st;
            }
            distinct.push_back(ps[i]);
            B->plans.push_back(P);
            idx = (int)B->plans.size() - 1;
        }
        B->params.push_back(ps[i]);
        B->plan_of.push_back(idx);
        B->work_off.push_back(B->work_bytes);
        B->work_bytes += align256(sar_workspace_bytes(B->plans[idx]));
    }
    *out = B;
    return SAR_OK;
}

size_t sar_batch_workspace_bytes(sar_batch_t B) { return B ? B->work_bytes : 0; }

sar_status sar_batch_execute(sar_batch_t B, const void* const* raw, void* const* img, void* work,
                             void* stream)
{
    sar::clear_error();
    if (!B) return sar::set_error(SAR_ERR_NULL, "batch is NULL");
    if (!raw || !img || !work) return sar::set_error(SAR_ERR_NULL, "raw, img or work is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != B->device)
        return sar::set_error(SAR_ERR_BAD_PARAM, "batch was planned on device %d", B->device);
    const int n = (int)B->params.size();
    for (int i = 0; i < n; ++i) {
        const size_t bytes = (size_t)B->params[i].Na * B->params[i].Nr * 8;
        if (!raw[i] || !img[i]) return sar::set_error(SAR_ERR_NULL, "scene %d: raw or img is NULL", i);
        if (((uintptr_t)raw[i] | (uintptr_t)img[i]) & 15u)
            return sar::set_error(SAR_ERR_BAD_PARAM, "scene %d: buffers not 16-byte aligned", i);
        if (overlap(raw[i], bytes, img[i], bytes) ||
            overlap(raw[i], bytes, work, B->work_bytes) || overlap(img[i], bytes, work, B->work_bytes))
            return sar::set_error(SAR_ERR_ALIAS, "scene %d: raw, img and work must be disjoint", i);
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const size_t bj = (size_t)B->params[j].Na * B->params[j].Nr * 8;
            if (j < i && overlap(img[i], bytes, img[j], bj))
                return sar::set_error(SAR_ERR_ALIAS, "scenes %d and %d share an image buffer", j, i);
            if (!raw[j]) return sar::set_error(SAR_ERR_NULL, "scene %d: raw is NULL", j);
            if (overlap(img[i], bytes, raw[j], bj))
                return sar::set_error(SAR_ERR_ALIAS, "image %d overlaps raw input %d", i, j);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const bool same = B->built && B->work_key == work && B->stream_key == stream &&
                      std::equal(B->raw_key.begin(), B->raw_key.end(), raw) &&
                      std::equal(B->img_key.begin(), B->img_key.end(), img);
    if (!same) {
        // a previous replay may still read the task buffer
        if (B->built) {
            const hipError_t e = hipStreamSynchronize((hipStream_t)B->stream_key);
            if (e != hipSuccess) return sar::set_error(SAR_ERR_HIP, "sync: %s", hipGetErrorString(e));
        }
        drop_graph(B);
        B->built = false;
        sar_status st = build(B, raw, img, work);
        if (st != SAR_OK) return st;
        B->raw_key.assign(raw, raw + n);
        B->img_key.assign(img, img + n);
        B->work_key = work;
        B->stream_key = stream;
        B->built = true;
        if (s != nullptr) {
            // capture the whole batch once; replays reuse it
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                sar_status est = enqueue(B, raw, img, work, s);
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(s, &g);
                if (est != SAR_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    B->built = false;
                    return est;
                }
                if (e == hipSuccess) {
                    B->graph = g;
                    e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
                }
                if (e != hipSuccess) drop_graph(B);   // fall back to direct launches
            }
            (void)hipGetLastError();
        }
    }
    if (B->exec) {
        const hipError_t e = hipGraphLaunch(B->exec, s);
        if (e != hipSuccess) return sar::set_error(SAR_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
        return SAR_OK;
    }
    return enqueue(B, raw, img, work, s);
}

void sar_batch_destroy(sar_batch_t B)
{
    if (!B) return;
    drop_graph(B);
    if (B->dev_tasks) (void)hipFree(B->dev_tasks);
    for (auto q : B->plans) sar_plan_destroy(q);
    delete B;
}

}  // extern "C"

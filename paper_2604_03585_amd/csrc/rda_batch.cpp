// rda_batch.cpp -- batched execution of scenes of uneven size.
//
// A batch is a list of per-scene plans and workspace offsets.  Execution
// enqueues every scene's steps on the caller's stream in scene order.
#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "rda_internal.h"
#include "sar_rda.h"

struct sar_batch_s {
    std::vector<sar_plan_t> plans;
    std::vector<size_t> work_off;     // byte offset of each scene's workspace
    size_t work_bytes = 0;
};

namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
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
    for (int i = 0; i < n; ++i) {
        sar_plan_t P = nullptr;
        sar_status st = sar_plan(&ps[i], stream, &P);
        if (st != SAR_OK) {
            for (auto q : B->plans) sar_plan_destroy(q);
            delete B;
            return st;
        }
        B->plans.push_back(P);
        B->work_off.push_back(B->work_bytes);
        B->work_bytes += align256(sar_workspace_bytes(P));
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
    for (size_t i = 0; i < B->plans.size(); ++i) {
        sar_status st = sar_rda_execute(B->plans[i], raw[i], img[i], (char*)work + B->work_off[i], stream);
        if (st != SAR_OK) return st;
    }
    return SAR_OK;
}

void sar_batch_destroy(sar_batch_t B)
{
    if (!B) return;
    for (auto q : B->plans) sar_plan_destroy(q);
    delete B;
}

sar_status sar_autotune(const sar_params* p, const char* cache_path)
{
    (void)cache_path;
    sar_plan_t P = nullptr;
    sar_status st = sar_plan(p, nullptr, &P);
    if (st != SAR_OK) return st;
    sar_plan_destroy(P);
    return sar::set_error(SAR_ERR_UNSUPPORTED, "autotuning is not built in this library");
}

}  // extern "C"

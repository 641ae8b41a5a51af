// fmm_evaluate_batch_noalloc (include/fmm.h): the batched evaluation for
// callers that cannot allocate device memory.  fmm_evaluate_batch stages the
// per-plan views in memory it allocates on every call; this entry point
// stages them in `scratch`, a fixed device array of the library (each device
// holds its own copy until the process ends).  In host code the array's name
// is not a device address: its address on each device is looked up once, with
// that device current, and only that address is used.
#include <mutex>
#include <string>

#include "batch.h"

namespace fmm {
namespace {
constexpr int kScratchPlans = FMM_NOALLOC_MAX_PLANS;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[sizeof(PlanView) * kScratchPlans];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// address of `scratch` on device dev (the current device), looked up on the
// first call on that device
int scratch_address(int dev, PlanView **out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error(FMM_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(FMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = (PlanView *)g_scratch_ptr[dev];
    return 0;
}
} // namespace
} // namespace fmm

using namespace fmm;

extern "C" int fmm_evaluate_batch_noalloc(fmm_plan_t const *plans, const double *const *q_dev,
                                          double *const *phi_dev, double *const *field_dev, int32_t count,
                                          hipStream_t stream)
{
    set_error(FMM_OK, "");
    if (count < 0 || count > kScratchPlans)
        return set_error(FMM_EINVAL, "fmm_evaluate_batch_noalloc takes 0.." + std::to_string(kScratchPlans) + " plans");
    if (count == 0) return FMM_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(FMM_EDEVICE, "hipGetDevice failed");
    PlanView *base = nullptr;
    if (int rc = scratch_address(dev, &base)) return rc;
    int idx[kScratchPlans];
    if (int rc = batch_prepare(plans, q_dev, phi_dev, count, stream, idx)) return rc;
    for (int i = 0; i < count; ++i)
        if (plan_device(plans[i]) != dev) return set_error(FMM_EINVAL, "plan built on another device");
    for (int c0 = 0; c0 < count; c0 += kMaxBatch) {
        const int c1 = count < c0 + kMaxBatch ? count : c0 + kMaxBatch;
        if (int rc = batch_chunk(plans, idx, c0, c1, q_dev, phi_dev, field_dev, stream, base + c0)) return rc;
    }
    return batch_note_use(plans, count, stream);
}

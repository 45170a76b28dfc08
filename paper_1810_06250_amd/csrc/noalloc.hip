// rmsynth_search_noalloc: the peaks-only search with its workspace in a
// fixed device array of this library instead of a caller's buffer, for
// callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable; in host code its name is a
// host-side stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to the kernels.  Every call on a device shares the one array: calls
// that overlap on a device race.  Nothing in it has to start at zero (each
// batch's kernels write every byte they later read).
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];

int scratch_ptr(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return rms_fail(RMSYNTH_EUNSUPPORTED, "rmsynth_search_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return rms_hip_fail(e, "rmsynth_search_noalloc: hipGetSymbolAddress");
        if (!ptr) return rms_fail(RMSYNTH_EHIP, "rmsynth_search_noalloc: no device address for the scratch array");
        g_ptr[dev] = ptr;
    }
    *out = g_ptr[dev];
    return RMSYNTH_OK;
}

}  // namespace

extern "C" {

size_t rmsynth_search_noalloc_scratch_bytes(void) { return kScratchBytes; }

int rmsynth_search_noalloc(rmsynth_plan_t p, const float* Q, const float* U, int64_t nlos,
                           int32_t layout, int32_t precision, int32_t* idx, float* phi_pk,
                           float* amp, float* q_pk, float* u_pk, float* phi_fit, float* amp_fit,
                           void* stream)
{
    const char* who = "rmsynth_search_noalloc";
    if (!p) return rms_fail(RMSYNTH_EINVAL, "%s: plan is NULL", who);
    if (nlos < 0) return rms_fail(RMSYNTH_EINVAL, "%s: nlos=%lld", who, (long long)nlos);
    if (precision < RMSYNTH_FP32 || precision > RMSYNTH_SPLIT_FP16)
        return rms_fail(RMSYNTH_EINVAL, "%s: precision=%d", who, precision);
    if (nlos == 0) return rms_ok();
    // One batch of 128 LOS must fit, whatever nlos is, so that the limit does
    // not depend on the call's size (only the unfused paths, which hold F of
    // a batch, can exceed it: above 65536 phi).
    const size_t least = search_workspace_bytes(p, 128, precision);
    if (least > kScratchBytes)
        return rms_fail(RMSYNTH_EINVAL,
                        "%s: a batch of 128 LOS needs %zu bytes of scratch, more than its %zu "
                        "(nphi = %d is too large for this entry point; use rmsynth_search)",
                        who, least, kScratchBytes, p->nphi);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rms_hip_fail(e, "hipGetDevice");
    void* ws = nullptr;
    if (int rc = scratch_ptr(dev, &ws)) return rc;
    return search_impl(p, Q, U, nlos, layout, precision, idx, phi_pk, amp, q_pk, u_pk, phi_fit,
                       amp_fit, ws, kScratchBytes, stream, who);
}

}  // extern "C"

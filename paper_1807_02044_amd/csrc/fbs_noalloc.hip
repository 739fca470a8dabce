// fbs_noalloc.hip - fbs_run_lr_noalloc: the fused left-right path with its
// workspace in a static device array instead of a caller's buffer, for
// callers that cannot allocate device memory.
//
// The array `scratch` exists once per GPU (each device that loads the library
// holds its own copy until the process ends).  Its name is a host-side
// stand-in in host code, so host code never hands it to a kernel: the device
// address is looked up with hipGetSymbolAddress on the first call on each
// device, with that device current, and the kernels receive that address.
// Every call on one GPU shares the array; overlapping calls on one GPU race.
#include <mutex>

#include "fbs_internal.h"

namespace fbs {
size_t api_lr_workspace_bytes(const fbs_params* p);
fbs_status api_run_lr(const fbs_params* p, const uint8_t* left, const uint8_t* right,
                      int max_diff, int32_t* disp_left, int32_t* disp_right, uint8_t* valid,
                      float* disp_sub, unsigned char* ws, hipStream_t s, const char* what);
fbs_status api_check_params(const fbs_params* p);
fbs_status api_fail(fbs_status st, const char* fmt, ...);
fbs_status api_hip_status(hipError_t e, const char* what);
bool api_aligned4(const void* q);
}  // namespace fbs

namespace {

__device__ __align__(256) unsigned char scratch[FBS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_addr[kMaxDevices];  // device address of `scratch`, per device

fbs_status scratch_of_current_device(unsigned char** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fbs::api_hip_status(e, "fbs_run_lr_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fbs::api_fail(FBS_E_UNSUPPORTED, "fbs_run_lr_noalloc: device %d above %d", dev,
                             kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* addr = nullptr;
        e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return fbs::api_hip_status(e, "fbs_run_lr_noalloc: hipGetSymbolAddress(scratch)");
        if (!addr) return fbs::api_fail(FBS_E_HIP, "fbs_run_lr_noalloc: scratch has no address");
        g_scratch_addr[dev] = static_cast<unsigned char*>(addr);
    }
    *out = g_scratch_addr[dev];
    return FBS_OK;
}

}  // namespace

extern "C" fbs_status fbs_run_lr_noalloc(const fbs_params* p, const uint8_t* left,
                                         const uint8_t* right, int32_t max_diff,
                                         int32_t* disp_left, int32_t* disp_right, uint8_t* valid,
                                         float* disp_sub, void* stream)
{
    fbs_status st = fbs::api_check_params(p);
    if (st != FBS_OK) return st;
    if (!left || !right) return fbs::api_fail(FBS_E_INVALID, "left and right are required");
    if (max_diff < 0) return fbs::api_fail(FBS_E_INVALID, "max_diff must be >= 0");
    if (!fbs::api_aligned4(disp_left) || !fbs::api_aligned4(disp_right) ||
        !fbs::api_aligned4(disp_sub))
        return fbs::api_fail(FBS_E_INVALID, "outputs must be 4-byte aligned");
    const size_t need = fbs::api_lr_workspace_bytes(p);
    if (need > (size_t)FBS_NOALLOC_SCRATCH_BYTES)
        return fbs::api_fail(FBS_E_UNSUPPORTED,
                             "fbs_run_lr_noalloc: needs %zu bytes of scratch, the static scratch "
                             "holds %zu (use fbs_run_lr with a workspace)",
                             need, (size_t)FBS_NOALLOC_SCRATCH_BYTES);
    if (!disp_left && !disp_right && !valid && !disp_sub) return FBS_OK;
    unsigned char* ws = nullptr;
    st = scratch_of_current_device(&ws);
    if (st != FBS_OK) return st;
    (void)hipGetLastError();
    return fbs::api_run_lr(p, left, right, max_diff, disp_left, disp_right, valid, disp_sub, ws,
                           (hipStream_t)stream, "fbs_run_lr_noalloc");
}

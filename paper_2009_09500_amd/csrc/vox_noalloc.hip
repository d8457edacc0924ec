// vox_segments_to_list_noalloc: the int16 voxel lists of
// vox_segments_to_list with the workspace in a library-owned device array
// instead of a caller-provided one, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  The call
// itself allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vox.h"
#include "vox_internal.h"

namespace {

// The workspace every call on a device shares (each device holds its own
// copy of the array, from module load to the end of the process).
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's array: looked up once per device, with that
// device current (the array's name in host code is only a host-side
// stand-in, never passed to a kernel).
vox_status device_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return (vox_status)vox::report_error(VOX_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return (vox_status)vox::report_error(VOX_ERR_DEVICE, "device %d beyond the library's %d", dev,
                                             kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return (vox_status)vox::report_error(VOX_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s",
                                                 hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VOX_OK;
}

}  // namespace

extern "C" vox_status vox_segments_to_list_noalloc(const vox_segment* d_segs, int64_t n, int64_t* d_offsets,
                                                   int16_t* d_voxels, int64_t capacity, int64_t* h_total,
                                                   void* stream) {
    if (n < 0 || capacity < 0)
        return (vox_status)vox::report_error(VOX_ERR_INVALID_ARGUMENT, "n and capacity must be >= 0");
    const int64_t cap = (d_voxels != nullptr && capacity > 0) ? capacity : 0;
    const size_t need = vox::list_workspace_bytes(n, cap);
    if (need > kScratchBytes)
        return (vox_status)vox::report_error(VOX_ERR_WORKSPACE,
                                             "%lld segments and capacity %lld need %zu bytes of workspace; the "
                                             "library's array holds %zu (use vox_segments_to_list)",
                                             (long long)n, (long long)capacity, need, kScratchBytes);
    void* ptr = nullptr;
    const vox_status st = device_scratch(&ptr);
    if (st != VOX_OK) return st;
    return vox_segments_to_list(d_segs, n, d_offsets, d_voxels, capacity, h_total, ptr, kScratchBytes, stream);
}

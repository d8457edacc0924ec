// C ABI entry points (include/vox.h): host-side argument checks, workspace
// carving and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "vox.h"
#include "vox_internal.h"

namespace {

thread_local char g_last_error[512] = "";

std::mutex g_tuning_mu;
vox_tuning g_tuning = {{0, 0, 0}};

vox_status fail(vox_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

vox_status ok() {
    g_last_error[0] = '\0';
    return VOX_OK;
}

vox_status device_fail(hipError_t e, const char* where) {
    return fail(VOX_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

constexpr int64_t kMaxDim = int64_t(1) << 20;
constexpr int64_t kMaxBits = int64_t(1) << 38;

vox_status check_dims(int32_t dx, int32_t dy, int32_t dz) {
    if (dx < 1 || dy < 1 || dz < 1 || dx > kMaxDim || dy > kMaxDim || dz > kMaxDim)
        return fail(VOX_ERR_INVALID_ARGUMENT, "volume dims must lie in [1, 2^20], got %d x %d x %d",
                    dx, dy, dz);
    if ((int64_t)dx * dy * dz > kMaxBits)
        return fail(VOX_ERR_INVALID_ARGUMENT, "volume larger than 2^38 voxels");
    return VOX_OK;
}

}  // namespace

namespace vox {
void tuned_brick_lg(int lg[3]) {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    for (int a = 0; a < 3; ++a) lg[a] = g_tuning.brick_lg[a];
}
}  // namespace vox

extern "C" {

vox_status vox_set_tuning(const vox_tuning* tuning) {
    vox_tuning t = {{0, 0, 0}};
    if (tuning) {
        t = *tuning;
        const bool zero = t.brick_lg[0] == 0 && t.brick_lg[1] == 0 && t.brick_lg[2] == 0;
        if (!zero && !vox::brick_shape_supported(t.brick_lg))
            return fail(VOX_ERR_INVALID_ARGUMENT, "brick shape 2^%d x 2^%d x 2^%d has no compiled kernel",
                        t.brick_lg[0], t.brick_lg[1], t.brick_lg[2]);
    }
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning = t;
    return ok();
}

vox_status vox_get_tuning(vox_tuning* tuning) {
    if (!tuning) return fail(VOX_ERR_INVALID_ARGUMENT, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    *tuning = g_tuning;
    return ok();
}


int vox_abi_version(void) { return VOX_ABI_VERSION; }

const char* vox_last_error(void) { return g_last_error; }

const char* vox_status_string(vox_status status) {
    switch (status) {
        case VOX_OK: return "ok";
        case VOX_ERR_INVALID_ARGUMENT: return "invalid argument";
        case VOX_ERR_OUT_OF_RANGE: return "end point out of range";
        case VOX_ERR_CAPACITY: return "voxel list exceeds capacity";
        case VOX_ERR_DEVICE: return "HIP runtime error";
        case VOX_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

size_t vox_list_workspace_bytes(int64_t n, int64_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return vox::list_workspace_bytes(n, capacity);
}

vox_status vox_segments_to_list(const vox_segment* d_segs, int64_t n, int64_t* d_offsets,
                                int16_t* d_voxels, int64_t capacity, int64_t* h_total,
                                void* d_work, size_t work_bytes, void* stream) {
    if (n < 0) return fail(VOX_ERR_INVALID_ARGUMENT, "n must be >= 0");
    if (n > (int64_t(1) << 31) - 2) return fail(VOX_ERR_INVALID_ARGUMENT, "n must be < 2^31 - 1");
    if (n > 0 && d_segs == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "d_segs is NULL");
    if (d_segs && !aligned(d_segs, 4)) return fail(VOX_ERR_INVALID_ARGUMENT, "d_segs not 4-byte aligned");
    if (d_offsets == nullptr || !aligned(d_offsets, 8))
        return fail(VOX_ERR_INVALID_ARGUMENT, "d_offsets NULL or not 8-byte aligned");
    if (capacity < 0) return fail(VOX_ERR_INVALID_ARGUMENT, "capacity must be >= 0");
    if (d_voxels && !aligned(d_voxels, 16))
        return fail(VOX_ERR_INVALID_ARGUMENT, "d_voxels not 16-byte aligned");
    const bool want = d_voxels != nullptr && capacity > 0;
    const int64_t cap = want ? capacity : 0;
    if (d_work == nullptr || !aligned(d_work, vox::kAlign))
        return fail(VOX_ERR_WORKSPACE, "d_work NULL or not 256-byte aligned");
    const size_t need = vox::list_workspace_bytes(n, cap);
    if (work_bytes < need)
        return fail(VOX_ERR_WORKSPACE, "workspace %zu bytes, need %zu", work_bytes, need);

    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t* segs = reinterpret_cast<const int32_t*>(d_segs);
    const bool a8 = aligned(d_segs, 8);
    vox::ListWork w = vox::list_workspace(d_work, n, cap);
    hipError_t e;
    if ((e = vox::launch_list_count(segs, n, a8, w, s)) != hipSuccess) return device_fail(e, "count");
    if ((e = vox::launch_list_scan(w, n, d_offsets, cap, want, s)) != hipSuccess)
        return device_fail(e, "scan");
    if ((e = vox::launch_list_offsets(n, d_offsets, w, cap, want, s)) != hipSuccess)
        return device_fail(e, "offsets");

    int64_t tiles = want ? (cap + vox::kListTile - 1) / vox::kListTile : 0;
    vox_status result = VOX_OK;
    if (h_total) {
        // One synchronisation: learn the total (and the status) before the
        // voxel launch so it can be sized exactly.
        int64_t hdr[2];
        if ((e = hipMemcpyAsync(hdr, d_work, sizeof(hdr), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return device_fail(e, "read total");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return device_fail(e, "synchronize");
        const int32_t st = (int32_t)(hdr[0] & 0xFFFFFFFF);
        *h_total = hdr[1];
        if (st & vox::kStatusOutOfRange) {
            result = fail(VOX_ERR_OUT_OF_RANGE, "a segment end point lies outside the int16 range");
            tiles = 0;
        } else if (st & vox::kStatusCapacity) {
            result = fail(VOX_ERR_CAPACITY, "total %lld voxels exceeds capacity %lld",
                          (long long)hdr[1], (long long)capacity);
            tiles = 0;
        } else {
            tiles = want ? (hdr[1] + vox::kListTile - 1) / vox::kListTile : 0;
        }
    }
    if (tiles > 0) {
        if ((e = vox::launch_list_voxels(segs, n, a8, d_offsets, w, d_voxels, cap, tiles, s)) !=
            hipSuccess)
            return device_fail(e, "voxels");
    }
    return result == VOX_OK ? ok() : result;
}

size_t vox_grid_workspace_bytes(int64_t n, int32_t dim_x, int32_t dim_y, int32_t dim_z) {
    if (n < 0 || check_dims(dim_x, dim_y, dim_z) != VOX_OK) return 0;
    return vox::grid_workspace_bytes(n, dim_x, dim_y, dim_z);
}

vox_status vox_segments_to_grid(const vox_segment* d_segs, int64_t n, int32_t dim_x, int32_t dim_y,
                                int32_t dim_z, uint32_t* d_grid, int32_t* d_counts, uint32_t flags,
                                void* d_work, size_t work_bytes, void* stream) {
    if (n < 0) return fail(VOX_ERR_INVALID_ARGUMENT, "n must be >= 0");
    if (n > (int64_t(1) << 31) - 2) return fail(VOX_ERR_INVALID_ARGUMENT, "n must be < 2^31 - 1");
    if (n > 0 && d_segs == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "d_segs is NULL");
    if (d_segs && !aligned(d_segs, 4)) return fail(VOX_ERR_INVALID_ARGUMENT, "d_segs not 4-byte aligned");
    vox_status st = check_dims(dim_x, dim_y, dim_z);
    if (st != VOX_OK) return st;
    if (d_grid == nullptr || !aligned(d_grid, 16))
        return fail(VOX_ERR_INVALID_ARGUMENT, "d_grid NULL or not 16-byte aligned");
    if (d_counts && !aligned(d_counts, 4))
        return fail(VOX_ERR_INVALID_ARGUMENT, "d_counts not 4-byte aligned");
    if (flags & ~VOX_GRID_CLEAR) return fail(VOX_ERR_INVALID_ARGUMENT, "unknown flag bits");
    if (d_work == nullptr || !aligned(d_work, vox::kAlign))
        return fail(VOX_ERR_WORKSPACE, "d_work NULL or not 256-byte aligned");
    const size_t need = vox::grid_workspace_bytes(n, dim_x, dim_y, dim_z);
    if (work_bytes < need) return fail(VOX_ERR_WORKSPACE, "workspace %zu bytes, need %zu", work_bytes, need);

    hipStream_t s = static_cast<hipStream_t>(stream);
    vox::GridWork w = vox::grid_workspace(d_work, n, dim_x, dim_y, dim_z);
    hipError_t e = vox::launch_grid(reinterpret_cast<const int32_t*>(d_segs), n, aligned(d_segs, 8),
                                    dim_x, dim_y, dim_z, d_grid, d_counts, flags, w, s);
    if (e != hipSuccess) return device_fail(e, "grid");
    return ok();
}

vox_status vox_batch_plan(const vox_scene* h_scenes, int32_t n_scenes, void* h_table,
                          size_t h_table_bytes, size_t* table_bytes, size_t* work_bytes) {
    (void)h_scenes; (void)n_scenes; (void)h_table; (void)h_table_bytes; (void)table_bytes;
    (void)work_bytes;
    return fail(VOX_ERR_INVALID_ARGUMENT, "vox_batch_plan: not available in this build");
}

vox_status vox_batch_scenes(const void* d_table, int32_t max_scenes, int64_t max_segments,
                            int64_t max_bricks, void* d_work, size_t work_bytes, void* stream) {
    (void)d_table; (void)max_scenes; (void)max_segments; (void)max_bricks; (void)d_work;
    (void)work_bytes; (void)stream;
    return fail(VOX_ERR_INVALID_ARGUMENT, "vox_batch_scenes: not available in this build");
}

vox_status vox_read_status(const void* d_work, int32_t* h_status, void* stream) {
    if (d_work == nullptr || h_status == nullptr)
        return fail(VOX_ERR_INVALID_ARGUMENT, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t raw = 0;
    hipError_t e = hipMemcpyAsync(&raw, d_work, sizeof(raw), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "read status");
    if (raw & vox::kStatusOutOfRange) *h_status = VOX_ERR_OUT_OF_RANGE;
    else if (raw & vox::kStatusCapacity) *h_status = VOX_ERR_CAPACITY;
    else *h_status = VOX_OK;
    return ok();
}

}  // extern "C"

// C ABI entry points (include/vox.h): host-side argument checks, workspace
// carving and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

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
        case VOX_ERR_BATCH_MISMATCH: return "batch table does not fit its launch or workspace";
    }
    return "unknown status";
}

size_t vox_list_workspace_bytes(int64_t n, int64_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return vox::list_workspace_bytes(n, capacity);
}

static vox_status segments_to_list(const vox_segment* d_segs, int64_t n, int64_t* d_offsets,
                                   void* d_voxels, int64_t capacity, int64_t* h_total,
                                   void* d_work, size_t work_bytes, void* stream, vox::ListKind kind) {
    const bool euclid = kind == vox::kListEuclid;
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
    if (n >= 1 && n <= vox::kSegsPerCountBlock) {
        // One block counts, scans and places.
        if ((e = vox::launch_list_one_block(segs, n, a8, w, d_offsets, cap, want, s, kind)) != hipSuccess)
            return device_fail(e, "count");
    } else {
        if ((e = vox::launch_list_count(segs, n, a8, w, s, kind)) != hipSuccess) return device_fail(e, "count");
        if ((e = vox::launch_list_scan(w, n, d_offsets, cap, want, s)) != hipSuccess)
            return device_fail(e, "scan");
        // (The Euclidean lists are written per segment: no output tiles.)
        if ((e = vox::launch_list_offsets(n, d_offsets, w, cap, want && !euclid, s)) != hipSuccess)
            return device_fail(e, "offsets");
    }

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
            result = kind == vox::kListI32
                         ? fail(VOX_ERR_OUT_OF_RANGE, "a segment spans 2^30 or more voxels along an axis")
                         : fail(VOX_ERR_OUT_OF_RANGE, "a segment end point lies outside the int16 range");
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
        if (euclid)
            e = vox::launch_list_voxels_euclid(segs, n, a8, d_offsets, w, static_cast<int16_t*>(d_voxels), s);
        else if (kind == vox::kListI32)
            e = vox::launch_list_voxels32(segs, n, a8, d_offsets, w, static_cast<int32_t*>(d_voxels), tiles, s);
        else
            e = vox::launch_list_voxels(segs, n, a8, d_offsets, w, static_cast<int16_t*>(d_voxels), cap, tiles,
                                        s);
        if (e != hipSuccess) return device_fail(e, "voxels");
    }
    return result == VOX_OK ? ok() : result;
}

vox_status vox_segments_to_list(const vox_segment* d_segs, int64_t n, int64_t* d_offsets,
                                int16_t* d_voxels, int64_t capacity, int64_t* h_total,
                                void* d_work, size_t work_bytes, void* stream) {
    return segments_to_list(d_segs, n, d_offsets, d_voxels, capacity, h_total, d_work, work_bytes, stream,
                            vox::kListI16);
}

vox_status vox_segments_to_list32(const vox_segment* d_segs, int64_t n, int64_t* d_offsets,
                                  int32_t* d_voxels, int64_t capacity, int64_t* h_total,
                                  void* d_work, size_t work_bytes, void* stream) {
    return segments_to_list(d_segs, n, d_offsets, d_voxels, capacity, h_total, d_work, work_bytes, stream,
                            vox::kListI32);
}

vox_status vox_segments_to_list_euclid(const vox_segment* d_segs, int64_t n, int64_t* d_offsets,
                                       int16_t* d_voxels, int64_t capacity, int64_t* h_total,
                                       void* d_work, size_t work_bytes, void* stream) {
    return segments_to_list(d_segs, n, d_offsets, d_voxels, capacity, h_total, d_work, work_bytes, stream,
                            vox::kListEuclid);
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
    if (flags & ~(VOX_GRID_CLEAR | VOX_GRID_EUCLID)) return fail(VOX_ERR_INVALID_ARGUMENT, "unknown flag bits");
    if (d_work == nullptr || !aligned(d_work, vox::kAlign))
        return fail(VOX_ERR_WORKSPACE, "d_work NULL or not 256-byte aligned");
    const size_t need = vox::grid_workspace_bytes(n, dim_x, dim_y, dim_z);
    if (work_bytes < need) return fail(VOX_ERR_WORKSPACE, "workspace %zu bytes, need %zu", work_bytes, need);

    hipStream_t s = static_cast<hipStream_t>(stream);
    vox::GridWork w = vox::grid_workspace(d_work, work_bytes, n, dim_x, dim_y, dim_z);
    hipError_t e = vox::launch_grid(reinterpret_cast<const int32_t*>(d_segs), n, aligned(d_segs, 8),
                                    dim_x, dim_y, dim_z, d_grid, d_counts, flags, w, s);
    if (e != hipSuccess) return device_fail(e, "grid");
    return ok();
}

vox_status vox_batch_plan(const vox_scene* h_scenes, int32_t n_scenes, void* h_table, size_t h_table_bytes,
                          vox_batch_launch* launch) {
    if (launch == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "launch is NULL");
    if (n_scenes < 1 || h_scenes == nullptr)
        return fail(VOX_ERR_INVALID_ARGUMENT, "need h_scenes with n_scenes >= 1");
    // Brick shape: the tuning if set, else the default of the largest volume.
    int lg[3];
    vox::tuned_brick_lg(lg);
    if (lg[0] == 0) {
        int64_t best = -1;
        for (int32_t i = 0; i < n_scenes; ++i) {
            const vox_scene& sc = h_scenes[i];
            const int64_t v = (int64_t)sc.dim_x * sc.dim_y * sc.dim_z;
            if (v > best) {
                best = v;
                vox::default_brick_lg(sc.dim_x, sc.dim_y, sc.dim_z, lg);
            }
        }
    }
    std::vector<vox::BrickScene> scenes((size_t)n_scenes);
    for (int32_t i = 0; i < n_scenes; ++i) {
        const vox_scene& in = h_scenes[i];
        if (in.n < 0 || in.n > (int64_t(1) << 31) - 2)
            return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: n must lie in [0, 2^31 - 2]", i);
        if (in.n > 0 && in.segs == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: segs is NULL", i);
        if (in.segs && !aligned(in.segs, 8))
            return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: segs not 8-byte aligned", i);
        if (check_dims(in.dim_x, in.dim_y, in.dim_z) != VOX_OK)
            return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: %s", i, g_last_error);
        if (in.grid == nullptr || !aligned(in.grid, 16))
            return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: grid NULL or not 16-byte aligned", i);
        if (in.counts && !aligned(in.counts, 4))
            return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: counts not 4-byte aligned", i);
        if (in.flags & ~VOX_GRID_CLEAR) return fail(VOX_ERR_INVALID_ARGUMENT, "scene %d: unknown flag bits", i);
        vox::BrickScene& sc = scenes[(size_t)i];
        if (!vox::brick_geometry_for(in.dim_x, in.dim_y, in.dim_z, lg, sc.bg))
            return fail(VOX_ERR_INVALID_ARGUMENT,
                        "scene %d: volume %d x %d x %d cannot take bricks of 2^%d x 2^%d x 2^%d (dim_x a multiple "
                        "of 32, sides <= 16384, <= 16384 bricks)",
                        i, in.dim_x, in.dim_y, in.dim_z, lg[0], lg[1], lg[2]);
        sc.segs = reinterpret_cast<const int32_t*>(in.segs);
        sc.counts = in.counts;
        sc.grid = in.grid;
        sc.n = in.n;
        sc.flags = (in.flags & VOX_GRID_CLEAR) ? vox::kSceneClear : 0u;
    }
    vox::BrickTable t{};
    for (int a = 0; a < 3; ++a) t.lg[a] = lg[a];
    if (!vox::brick_table_layout(t, scenes.data(), (uint32_t)n_scenes))
        return fail(VOX_ERR_INVALID_ARGUMENT, "batch too large: more than 2^32 - 1 bricks or pieces");
    launch->rows = t.rows;
    launch->bricks = t.bricks;
    for (int a = 0; a < 3; ++a) launch->brick_lg[a] = lg[a];
    launch->max_scene_bricks = (int32_t)t.max_nb;
    launch->work_bytes = t.work_bytes;
    launch->table_bytes = t.table_bytes;
    if (h_table == nullptr) return ok();
    if (h_table_bytes < t.table_bytes)
        return fail(VOX_ERR_INVALID_ARGUMENT, "h_table holds %zu bytes, the table needs %llu", h_table_bytes,
                    (unsigned long long)t.table_bytes);
    uint8_t* out = static_cast<uint8_t*>(h_table);
    std::memset(out, 0, (size_t)t.table_bytes);
    std::memcpy(out, &t, sizeof(t));
    std::memcpy(out + vox::kTableScenes, scenes.data(), scenes.size() * sizeof(vox::BrickScene));
    if (n_scenes > 1) {
        uint32_t* row_scene = reinterpret_cast<uint32_t*>(out + vox::kTableScenes +
                                                          scenes.size() * sizeof(vox::BrickScene));
        uint32_t* brick_scene = row_scene + t.rows;
        for (int32_t i = 0; i < n_scenes; ++i) {
            const vox::BrickScene& sc = scenes[(size_t)i];
            for (uint32_t r = 0; r < sc.rows; ++r) row_scene[sc.row_base + r] = (uint32_t)i;
            for (uint32_t b = 0; b < sc.bg.nbricks; ++b) brick_scene[sc.brick_base + b] = (uint32_t)i;
        }
    }
    return ok();
}

vox_status vox_batch_launch_cover(vox_batch_launch* bound, const vox_batch_launch* launch) {
    if (bound == nullptr || launch == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "NULL argument");
    const bool empty = bound->brick_lg[0] == 0 && bound->brick_lg[1] == 0 && bound->brick_lg[2] == 0;
    if (!empty && (bound->brick_lg[0] != launch->brick_lg[0] || bound->brick_lg[1] != launch->brick_lg[1] ||
                   bound->brick_lg[2] != launch->brick_lg[2]))
        return fail(VOX_ERR_INVALID_ARGUMENT, "brick shapes differ");
    for (int a = 0; a < 3; ++a) bound->brick_lg[a] = launch->brick_lg[a];
    if (launch->rows > bound->rows) bound->rows = launch->rows;
    if (launch->bricks > bound->bricks) bound->bricks = launch->bricks;
    if (launch->max_scene_bricks > bound->max_scene_bricks) bound->max_scene_bricks = launch->max_scene_bricks;
    if (launch->work_bytes > bound->work_bytes) bound->work_bytes = launch->work_bytes;
    if (launch->table_bytes > bound->table_bytes) bound->table_bytes = launch->table_bytes;
    return ok();
}

vox_status vox_batch_scenes(const void* d_table, const vox_batch_launch* launch, void* d_work, size_t work_bytes,
                            void* stream) {
    if (d_table == nullptr || !aligned(d_table, 16))
        return fail(VOX_ERR_INVALID_ARGUMENT, "d_table NULL or not 16-byte aligned");
    if (launch == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "launch is NULL");
    if (launch->rows < 1 || launch->rows >= (int64_t(1) << 31) || launch->bricks < 1 ||
        launch->bricks >= 0xFFFFFFFFll || launch->max_scene_bricks < 1 ||
        launch->max_scene_bricks > (int32_t)vox::kMaxBricks)
        return fail(VOX_ERR_INVALID_ARGUMENT, "launch sizes out of range (use vox_batch_plan)");
    if (!vox::brick_shape_supported(launch->brick_lg))
        return fail(VOX_ERR_INVALID_ARGUMENT, "brick shape 2^%d x 2^%d x 2^%d has no compiled kernel",
                    launch->brick_lg[0], launch->brick_lg[1], launch->brick_lg[2]);
    if (d_work == nullptr || !aligned(d_work, vox::kAlign))
        return fail(VOX_ERR_WORKSPACE, "d_work NULL or not 256-byte aligned");
    if (work_bytes < launch->work_bytes)
        return fail(VOX_ERR_WORKSPACE, "workspace %zu bytes, the launch needs %llu", work_bytes,
                    (unsigned long long)launch->work_bytes);
    vox::BrickLaunch L;
    L.rows = (uint32_t)launch->rows;
    L.bricks = (uint32_t)launch->bricks;
    for (int a = 0; a < 3; ++a) L.lg[a] = launch->brick_lg[a];
    L.max_nb = (uint32_t)launch->max_scene_bricks;
    hipError_t e = vox::launch_bricks(d_table, L, nullptr, nullptr, d_work, work_bytes,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(e, "batch");
    return ok();
}

vox_status vox_read_status(const void* d_work, int32_t* h_status, void* stream) {
    if (d_work == nullptr || h_status == nullptr)
        return fail(VOX_ERR_INVALID_ARGUMENT, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t raw = 0;
    hipError_t e = hipMemcpyAsync(&raw, d_work, sizeof(raw), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "read status");
    if (raw & vox::kStatusLaunch) *h_status = VOX_ERR_BATCH_MISMATCH;
    else if (raw & vox::kStatusOutOfRange) *h_status = VOX_ERR_OUT_OF_RANGE;
    else if (raw & vox::kStatusCapacity) *h_status = VOX_ERR_CAPACITY;
    else *h_status = VOX_OK;
    return ok();
}

}  // extern "C"

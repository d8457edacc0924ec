// C ABI entry points (include/vox.h): host-side argument checks, workspace
// carving and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "vox.h"
#include "vox_internal.h"

namespace {

thread_local char g_last_error[512] = "";

// Autotune cache: tuning per (volume, floor(log2 n)); dims 0 x 0 x 0 for
// batches keyed by their total segment count.
struct CacheKey {
    int32_t dim[3];
    int32_t lgn;
    bool operator==(const CacheKey& o) const {
        return dim[0] == o.dim[0] && dim[1] == o.dim[1] && dim[2] == o.dim[2] && lgn == o.lgn;
    }
};
std::mutex g_cache_mu;
std::vector<std::pair<CacheKey, vox::Tuning>> g_cache;

CacheKey cache_key(int32_t dx, int32_t dy, int32_t dz, int64_t n) {
    int32_t lgn = 0;
    for (uint64_t v = n > 1 ? (uint64_t)n : 1u; v > 1; v >>= 1) ++lgn;
    return CacheKey{{dx, dy, dz}, lgn};
}

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
constexpr int32_t kMaxBatchScenes = 65536;
constexpr int64_t kMaxBatchSegments = int64_t(1) << 40;
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

int report_error(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return status;
}

// A vox_tuning from the ABI: a supported shape (or all zero = the default of
// the call), fill_wgs_per_cu 0, 1 or 2 (2 only for 64 KiB bricks), zero
// reserved words.
bool tuning_from_abi(const void* p, Tuning& t, char* why, size_t why_len) {
    const vox_tuning& in = *static_cast<const vox_tuning*>(p);
    for (int a = 0; a < 3; ++a) t.lg[a] = in.brick_lg[a];
    t.fill_wgs_per_cu = in.fill_wgs_per_cu;
    const bool zero = t.lg[0] == 0 && t.lg[1] == 0 && t.lg[2] == 0;
    if (!zero && !brick_shape_supported(t.lg)) {
        snprintf(why, why_len, "brick shape 2^%d x 2^%d x 2^%d has no compiled kernel", t.lg[0], t.lg[1], t.lg[2]);
        return false;
    }
    const int bits = t.lg[0] + t.lg[1] + t.lg[2];
    if (t.fill_wgs_per_cu < 0 || t.fill_wgs_per_cu > 2 || (t.fill_wgs_per_cu == 2 && !zero && bits >= 20)) {
        snprintf(why, why_len, "fill_wgs_per_cu %d not available for this brick shape", t.fill_wgs_per_cu);
        return false;
    }
    for (int i = 0; i < 4; ++i)
        if (in.reserved[i] != 0) {
            snprintf(why, why_len, "reserved tuning fields must be zero");
            return false;
        }
    return true;
}

bool tuning_cache_lookup(int32_t dx, int32_t dy, int32_t dz, int64_t n, Tuning& t) {
    const CacheKey k = cache_key(dx, dy, dz, n);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (const auto& e : g_cache)
        if (e.first == k) {
            t = e.second;
            return t.lg[0] != 0;
        }
    return false;
}

}  // namespace vox

extern "C" {

vox_status vox_tuning_cache_set(int32_t dim_x, int32_t dim_y, int32_t dim_z, int64_t n_segments,
                                const vox_tuning* tuning) {
    if (n_segments < 0 || dim_x < 0 || dim_y < 0 || dim_z < 0)
        return fail(VOX_ERR_INVALID_ARGUMENT, "negative key");
    const CacheKey k = cache_key(dim_x, dim_y, dim_z, n_segments);
    vox::Tuning t{};
    if (tuning) {
        char why[160];
        if (!vox::tuning_from_abi(tuning, t, why, sizeof(why))) return fail(VOX_ERR_INVALID_ARGUMENT, "%s", why);
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_cache.size(); ++i)
        if (g_cache[i].first == k) {
            g_cache.erase(g_cache.begin() + (long)i);
            break;
        }
    if (tuning) g_cache.emplace_back(k, t);
    return ok();
}

vox_status vox_tuning_cache_get(int32_t dim_x, int32_t dim_y, int32_t dim_z, int64_t n_segments,
                                vox_tuning* tuning, int32_t* found) {
    if (tuning == nullptr || found == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "NULL argument");
    const CacheKey k = cache_key(dim_x, dim_y, dim_z, n_segments);
    std::memset(tuning, 0, sizeof(*tuning));
    *found = 0;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (const auto& e : g_cache)
        if (e.first == k) {
            for (int a = 0; a < 3; ++a) tuning->brick_lg[a] = e.second.lg[a];
            tuning->fill_wgs_per_cu = e.second.fill_wgs_per_cu;
            *found = 1;
            break;
        }
    return ok();
}

void vox_tuning_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.clear();
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
        case VOX_ERR_BATCH_MISMATCH: return "batch scenes exceed the call's n_scenes or total_segments";
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
    // The full workspace, or a compact one (vox_workspace_bytes(VOX_OP_GRID)):
    // at least its table and histogram part, the records as far as they fit.
    const size_t need = vox::grid_workspace_bytes(n, dim_x, dim_y, dim_z);
    const size_t need_compact = vox::grid_compact_fixed_bytes(n, dim_x, dim_y, dim_z);
    if (work_bytes < need && work_bytes < need_compact)
        return fail(VOX_ERR_WORKSPACE, "workspace %zu bytes, need %zu (compact: at least %zu)", work_bytes, need,
                    need_compact);

    hipStream_t s = static_cast<hipStream_t>(stream);
    vox::GridWork w = vox::grid_workspace(d_work, work_bytes, n, dim_x, dim_y, dim_z);
    hipError_t e = vox::launch_grid(reinterpret_cast<const int32_t*>(d_segs), n, aligned(d_segs, 8),
                                    dim_x, dim_y, dim_z, d_grid, d_counts, flags, w, s);
    if (e != hipSuccess) return device_fail(e, "grid");
    return ok();
}

size_t vox_workspace_bytes(int op, int64_t n_segments, int32_t n_scenes) {
    if (n_segments < 0 || n_scenes < 1) return 0;
    if (op == VOX_OP_GRID && n_scenes != 1) return 0;
    if (op == VOX_OP_BATCH || op == VOX_OP_GRID) {
        if (n_scenes > kMaxBatchScenes || n_segments > kMaxBatchSegments) return 0;
        const int lg[3] = {8, 6, 6};  // (the fixed part does not depend on the shape)
        const vox::BrickLaunch L = vox::batch_launch((uint32_t)n_scenes, (uint64_t)n_segments, lg);
        return vox::batch_fixed_bytes(L) +
               (size_t)((uint64_t)n_segments * vox::kDefaultPiecesPerSegment * vox::kRecordBytes);
    }
    return 0;
}

vox_status vox_batch_scenes(const vox_scene* d_scenes, int32_t n_scenes, int64_t total_segments,
                            const vox_tuning* tuning, void* d_work, size_t work_bytes, void* stream) {
    if (d_scenes == nullptr || !aligned(d_scenes, 8))
        return fail(VOX_ERR_INVALID_ARGUMENT, "d_scenes NULL or not 8-byte aligned");
    if (n_scenes < 1 || n_scenes > kMaxBatchScenes)
        return fail(VOX_ERR_INVALID_ARGUMENT, "n_scenes must lie in [1, %d]", kMaxBatchScenes);
    if (total_segments < 0 || total_segments > kMaxBatchSegments)
        return fail(VOX_ERR_INVALID_ARGUMENT, "total_segments must lie in [0, 2^40]");
    vox::Tuning t{};
    if (tuning) {
        char why[160];
        if (!vox::tuning_from_abi(tuning, t, why, sizeof(why))) return fail(VOX_ERR_INVALID_ARGUMENT, "%s", why);
    } else if (!vox::tuning_cache_lookup(0, 0, 0, total_segments, t)) {
        t = vox::Tuning{};
    }
    if (t.lg[0] == 0) {
        // Default: 256 x 64 x 64 bricks, the fastest shape on the 256-scene
        // workload (64^3 ... 512^3 volumes: 2.11 ms against 2.28 ms for
        // 256 x 64 x 32 with two workgroups per CU), with one workgroup of
        // 1024 threads per CU.
        t.lg[0] = 8;
        t.lg[1] = 6;
        t.lg[2] = 6;
    }
    if (d_work == nullptr || !aligned(d_work, vox::kAlign))
        return fail(VOX_ERR_WORKSPACE, "d_work NULL or not 256-byte aligned");
    const vox::BrickLaunch L = vox::batch_launch((uint32_t)n_scenes, (uint64_t)total_segments, t.lg);
    const size_t need = vox::batch_fixed_bytes(L);
    if (work_bytes < need)
        return fail(VOX_ERR_WORKSPACE, "workspace %zu bytes, the table and histograms need %zu", work_bytes, need);
    hipError_t e = vox::launch_bricks(d_scenes, nullptr, L, t.fill_wgs_per_cu, d_work, work_bytes,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(e, "batch");
    return ok();
}

int32_t* vox_device_status(void* d_work) { return static_cast<int32_t*>(d_work); }

vox_status vox_read_batch_info(const void* d_work, uint64_t* h_pieces, int32_t* h_direct_all, void* stream) {
    if (d_work == nullptr) return fail(VOX_ERR_INVALID_ARGUMENT, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t hdr[vox::kWPieces + 2];
    hipError_t e = hipMemcpyAsync(hdr, d_work, sizeof(hdr), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(e, "read batch info");
    if (h_pieces) *h_pieces = (uint64_t)hdr[vox::kWPieces] | ((uint64_t)hdr[vox::kWPieces + 1] << 32);
    if (h_direct_all) *h_direct_all = hdr[vox::kWDirectAll] ? 1 : 0;
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
    else if (raw & vox::kStatusInvalid) *h_status = VOX_ERR_INVALID_ARGUMENT;
    else if (raw & vox::kStatusOutOfRange) *h_status = VOX_ERR_OUT_OF_RANGE;
    else if (raw & vox::kStatusCapacity) *h_status = VOX_ERR_CAPACITY;
    else *h_status = VOX_OK;
    return ok();
}

}  // extern "C"

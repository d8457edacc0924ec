// Bit-volume output, direct form: every voxel is ORed into its grid word
// with a device-scope atomic.  Correct for any volume shape; used for
// volumes the brick path does not cover.
#include "vox.h"
#include "vox_device.h"
#include "vox_direct.h"
#include "vox_exact.h"
#include "vox_internal.h"

namespace vox {

constexpr int kGridBlock = 256;

__global__ void k_grid_init(int32_t* status) {
    if (threadIdx.x == 0) *status = 0;
}

// Zeroes the volume and the status word (a cleared direct call is then two
// launches).
__global__ __launch_bounds__(kGridBlock) void k_grid_clear(uint32_t* __restrict__ grid, int64_t nwords,
                                                           int32_t* __restrict__ status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
    clear_words(grid, nwords, (int64_t)blockIdx.x * kGridBlock + threadIdx.x, (int64_t)gridDim.x * kGridBlock);
}

// All segments of one volume (direct_segments, vox_direct.h).
template <bool kAligned8, bool kEuclid>
__global__ __launch_bounds__(kGridBlock) void k_grid_direct(const int32_t* __restrict__ segs, int64_t n,
                                                            int32_t dx, int32_t dy, int32_t dz,
                                                            uint32_t* __restrict__ grid,
                                                            int32_t* __restrict__ counts,
                                                            int32_t* __restrict__ status) {
    direct_segments<kAligned8, kEuclid>(segs, n, dx, dy, dz, grid, counts, status,
                                        (int64_t)blockIdx.x * (kGridBlock / kWave) + threadIdx.x / kWave,
                                        (int64_t)gridDim.x * (kGridBlock / kWave));
}

// Plain calls with at most this many segments take the direct path: its
// three launches beat the brick pipeline's six there (measured on one
// MI355X: 1 000 segments in 256^3, 11 vs 38 us a call; one segment, 10 vs
// 30 us; 16 384 segments in 512^3, 44 vs 77 us).
constexpr int64_t kDirectMaxSegments = 16384;

// The brick path serves calls with more segments than that, on volumes whose
// rows are whole words and whose piece ids fit 32 bits; everything else takes
// the direct path.
static bool use_bricks(int64_t n, int32_t dx, int32_t dy, int32_t dz, bool euclid, BrickGeom& bg, Tuning& t) {
    if (n <= kDirectMaxSegments) return false;
    if (euclid && !euclid_bricks_ok(dx, dy, dz)) return false;
    if (!tuning_cache_lookup(dx, dy, dz, n, t)) {
        default_brick_lg(dx, dy, dz, t.lg);
        t.fill_wgs_per_cu = 0;
    }
    if (!brick_geometry(dx, dy, dz, t.lg, bg)) return false;
    if (!brick_shape_supported(bg.lg)) return false;
    if (n >= (int64_t(1) << 31) - 1) return false;
    return max_pieces(n, bg) < (uint64_t(1) << 32) - 1;
}

size_t grid_workspace_bytes(int64_t n, int32_t dx, int32_t dy, int32_t dz) {
    BrickGeom bg;
    Tuning t;
    // (The Euclidean N takes the brick path under the same rules, but for the
    // volume's diagonal; the workspace bound covers both.)
    if (use_bricks(n, dx, dy, dz, false, bg, t)) return brick_workspace_bytes(n, bg);
    return kAlign;
}

size_t grid_compact_fixed_bytes(int64_t n, int32_t dx, int32_t dy, int32_t dz) {
    BrickGeom bg;
    Tuning t;
    if (!use_bricks(n, dx, dy, dz, false, bg, t)) return kAlign;
    return batch_fixed_bytes(batch_launch(1u, (uint64_t)n, bg.lg));
}

GridWork grid_workspace(void* d_work, size_t work_bytes, int64_t n, int32_t dx, int32_t dy, int32_t dz) {
    (void)n; (void)dx; (void)dy; (void)dz;
    GridWork w;
    w.status = static_cast<int32_t*>(d_work);
    w.bytes = work_bytes;
    return w;
}

hipError_t launch_grid(const int32_t* segs, int64_t n, bool aligned8, int32_t dx, int32_t dy,
                       int32_t dz, uint32_t* grid, int32_t* counts, uint32_t flags,
                       const GridWork& w, hipStream_t stream) {
    BrickGeom bg;
    Tuning t;
    // The brick path reads segments with 8-byte loads; arrays that are only
    // 4-byte aligned take the direct path.
    const bool euclid = (flags & 2u) != 0;  // VOX_GRID_EUCLID
    if (aligned8 && use_bricks(n, dx, dy, dz, euclid, bg, t)) {
        vox_scene one{};
        one.segs = reinterpret_cast<const vox_segment*>(segs);
        one.n = n;
        one.dim_x = dx;
        one.dim_y = dy;
        one.dim_z = dz;
        one.flags = flags & 3u;
        one.grid = grid;
        one.counts = counts;
        // A workspace below the worst case of records: the call runs as a
        // one-scene batch, whose direct kernels serve it when its records do
        // not fit.
        const BrickLaunch L = w.bytes >= brick_workspace_bytes(n, bg) ? plain_launch(n, bg)
                                                                       : batch_launch(1u, (uint64_t)n, bg.lg);
        return launch_bricks(nullptr, &one, L, t.fill_wgs_per_cu, w.status, w.bytes, stream);
    }
    hipError_t e = hipSuccess;
    const int64_t nwords = ((int64_t)dx * dy * dz + 31) / 32;
    if (flags & 1u) {
        int64_t blocks = (nwords / 4 + kGridBlock - 1) / kGridBlock;
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        KernelTimer timer("grid_clear", stream);
        k_grid_clear<<<dim3((unsigned)blocks), kGridBlock, 0, stream>>>(grid, nwords, w.status);
    } else {
        KernelTimer timer("grid_init", stream);
        k_grid_init<<<1, 64, 0, stream>>>(w.status);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    constexpr int kSegsPerBlock = kGridBlock / kSampleLanes;
    int64_t blocks = (n + kSegsPerBlock - 1) / kSegsPerBlock;
    if (blocks > 16384) blocks = 16384;
    dim3 gridDim((unsigned)blocks);
    KernelTimer timer(euclid ? "grid_direct_euclid" : "grid_direct", stream);
    if (euclid) {
        if (aligned8)
            k_grid_direct<true, true><<<gridDim, kGridBlock, 0, stream>>>(segs, n, dx, dy, dz, grid, counts,
                                                                          w.status);
        else
            k_grid_direct<false, true><<<gridDim, kGridBlock, 0, stream>>>(segs, n, dx, dy, dz, grid, counts,
                                                                           w.status);
    } else {
        if (aligned8)
            k_grid_direct<true, false><<<gridDim, kGridBlock, 0, stream>>>(segs, n, dx, dy, dz, grid, counts,
                                                                           w.status);
        else
            k_grid_direct<false, false><<<gridDim, kGridBlock, 0, stream>>>(segs, n, dx, dy, dz, grid, counts,
                                                                            w.status);
    }
    return hipGetLastError();
}

}  // namespace vox

// Bit-volume output, direct form: every voxel is ORed into its grid word
// with a device-scope atomic.  Correct for any volume shape; used for
// volumes the brick path does not cover.
#include "vox_device.h"
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
    const int64_t stride = (int64_t)gridDim.x * kGridBlock;
    const int64_t n4 = nwords / 4;
    uint4* g4 = reinterpret_cast<uint4*>(grid);
    for (int64_t i = (int64_t)blockIdx.x * kGridBlock + threadIdx.x; i < n4; i += stride)
        g4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = n4 * 4 + (int64_t)blockIdx.x * kGridBlock + threadIdx.x; i < nwords; i += stride)
        grid[i] = 0u;
}

// Four segments per wave, 16 lanes each; a segment's lanes take its samples
// 16 at a time (SampleAt), and each lane whose sample starts a new voxel ORs
// that voxel's bit into the grid.  Range check first: a segment with an end
// point outside the volume sets the status and writes nothing.  Counts:
// N + 1 for the Chebyshev N (also for a segment outside the volume), the
// number of voxels after duplicate removal for the Euclidean N of eq. (1)
// (0 outside the volume).
template <bool kAligned8, bool kEuclid>
__global__ __launch_bounds__(kGridBlock) void k_grid_direct(const int32_t* __restrict__ segs, int64_t n,
                                                            int32_t dx, int32_t dy, int32_t dz,
                                                            uint32_t* __restrict__ grid,
                                                            int32_t* __restrict__ counts,
                                                            int32_t* __restrict__ status) {
    constexpr int kSlots = kWave / kSampleLanes;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t sub = lane % kSampleLanes;
    const uint32_t slot = lane / kSampleLanes;
    const uint64_t slot_bits = ((1ull << kSampleLanes) - 1) << (kSampleLanes * slot);
    const int32_t dim[3] = {dx, dy, dz};
    const int64_t step = (int64_t)gridDim.x * (kGridBlock / kWave) * kSlots;
    for (int64_t i0 = ((int64_t)blockIdx.x * (kGridBlock / kWave) + threadIdx.x / kWave) * kSlots; i0 < n;
         i0 += step) {
        const int64_t i = i0 + slot;
        const bool valid = i < n;
        Seg g = {};
        if (valid) g = load_seg<kAligned8>(segs, i);
        bool ok = valid;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            ok &= (g.p0[a] >= 0) & (g.p0[a] < dim[a]) & (g.p1[a] >= 0) & (g.p1[a] < dim[a]);
        if (valid && sub == 0) {
            if (!kEuclid && counts) {
                const int64_t N64 = seg_length(g);
                counts[i] = (int32_t)(N64 + 1 > 0x7FFFFFFFll ? 0x7FFFFFFFll : N64 + 1);
            }
            if (!ok) {
                if (kEuclid && counts) counts[i] = 0;
                atomicOr(status, kStatusOutOfRange);
            }
        }
        if (!ok) g = Seg{};
        // Inside the volume every side is below 2^20: N < 2^21.
        SampleAt s;
        s.init(g, kEuclid ? euclid_length(g) : (uint32_t)seg_length(g));
        bool moved = s.start(sub);
        uint32_t kept = 0;
        for (uint32_t c0 = 0; __ballot(ok && c0 <= s.N) != 0; c0 += kSampleLanes) {
            if (c0 != 0) moved = s.next();
            const bool keep = moved && ok && c0 + sub <= s.N;
            if (keep) {
                const uint64_t b = ((uint64_t)s.coord(g, 2) * (uint64_t)dy + (uint64_t)s.coord(g, 1)) *
                                       (uint64_t)dx +
                                   (uint64_t)s.coord(g, 0);
                atomicOr(grid + (b >> 5), 1u << (uint32_t)(b & 31u));
            }
            if (kEuclid) kept += (uint32_t)__popcll(__ballot(keep) & slot_bits);
        }
        if (kEuclid && ok && sub == 0 && counts) counts[i] = (int32_t)kept;
    }
}

// Plain calls with at most this many segments take the direct path: its
// three launches beat the brick pipeline's six there (measured on one
// MI355X: 1 000 segments in 256^3, 11 vs 38 us a call; one segment, 10 vs
// 30 us; 16 384 segments in 512^3, 44 vs 77 us).
constexpr int64_t kDirectMaxSegments = 16384;

// The brick path serves calls with more segments than that, on volumes whose
// rows are whole words and whose piece ids fit 32 bits; everything else takes
// the direct path.
static bool use_bricks(int64_t n, int32_t dx, int32_t dy, int32_t dz, BrickGeom& bg) {
    if (n <= kDirectMaxSegments) return false;
    int lg[3];
    default_brick_lg(dx, dy, dz, lg);
    int tl[3];
    tuned_brick_lg(tl);
    if (tl[0] > 0) {
        lg[0] = tl[0];
        lg[1] = tl[1];
        lg[2] = tl[2];
    }
    if (!brick_geometry(dx, dy, dz, lg, bg)) return false;
    if (!brick_shape_supported(bg.lg)) return false;
    if (n >= (int64_t(1) << 32) - 1) return false;
    return max_pieces(n, bg) < (uint64_t(1) << 32) - 1;
}

size_t grid_workspace_bytes(int64_t n, int32_t dx, int32_t dy, int32_t dz) {
    BrickGeom bg;
    if (use_bricks(n, dx, dy, dz, bg)) return brick_workspace_bytes(n, bg);
    return kAlign;
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
    // The brick path reads segments with 8-byte loads; arrays that are only
    // 4-byte aligned take the direct path.
    const bool euclid = (flags & 2u) != 0;  // VOX_GRID_EUCLID: the direct path only
    if (!euclid && aligned8 && use_bricks(n, dx, dy, dz, bg))
        return launch_brick_grid(segs, n, bg, grid, counts, flags, w.status, w.bytes, stream);
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

// The direct form of the bit-volume output: every voxel ORed into its grid
// word with a device-scope atomic.  Correct for any volume shape; shared by
// the plain direct path (vox_grid.hip) and the scenes of a batch that the
// brick path does not serve (vox_brick.hip).
#pragma once

#include "vox_device.h"
#include "vox_internal.h"

namespace vox {

// Segments [0, n) of one volume, four per wave, 16 lanes each; the waves of
// the launch take segment groups wave0, wave0 + wave_stride, ...  A
// segment's lanes take its samples 16 at a time (SampleAt), and each lane
// whose sample starts a new voxel ORs that voxel's bit into the grid.  Range
// check first: a segment with an end point outside the volume sets the
// status and writes nothing.  Counts: N + 1 for the Chebyshev N (also for a
// segment outside the volume), the number of voxels after duplicate removal
// for the Euclidean N of eq. (1) (0 outside the volume).
template <bool kAligned8, bool kEuclid>
__device__ __forceinline__ void direct_segments(const int32_t* __restrict__ segs, int64_t n, int32_t dx,
                                                int32_t dy, int32_t dz, uint32_t* __restrict__ grid,
                                                int32_t* __restrict__ counts, int32_t* __restrict__ status,
                                                int64_t wave0, int64_t wave_stride) {
    constexpr int kSlots = kWave / kSampleLanes;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t sub = lane % kSampleLanes;
    const uint32_t slot = lane / kSampleLanes;
    const uint64_t slot_bits = ((1ull << kSampleLanes) - 1) << (kSampleLanes * slot);
    const int32_t dim[3] = {dx, dy, dz};
    for (int64_t i0 = wave0 * kSlots; i0 < n; i0 += wave_stride * kSlots) {
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

// Zeroes words [0, nwords) of a 16-byte-aligned volume; the threads of the
// launch take 16-byte units t0, t0 + t_stride, ...
__device__ __forceinline__ void clear_words(uint32_t* __restrict__ grid, int64_t nwords, int64_t t0,
                                            int64_t t_stride) {
    const int64_t n4 = nwords / 4;
    uint4* g4 = reinterpret_cast<uint4*>(grid);
    for (int64_t i = t0; i < n4; i += t_stride) g4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = n4 * 4 + t0; i < nwords; i += t_stride) grid[i] = 0u;
}

}  // namespace vox

// Voxel lists: count -> scan -> offsets + tile map -> lane-per-voxel tiles.
//
// Steps of the path (arXiv 2009.09500, Section 4 lists them as host
// preprocessing followed by one kernel; here all of them run on the GPU):
//   1. count   N_i + 1 per segment ("the voxels number in the segment",
//              host step 1 of Section 4), int16 range check;
//   2. scan    exclusive prefix sum of the counts -> d_offsets (replaces the
//              paper's padding of every segment to N_max, Section 5);
//   3. tiles   each tile of kListTile consecutive output voxels learns the
//              segment holding its first voxel;
//   4. voxels  every lane computes kListPerThread consecutive voxels of the
//              flat output with the exact stepping of eq. (3), stages them
//              in LDS and the block writes the tile with 16-byte stores.
#include <type_traits>

#include "vox_device.h"
#include "vox_internal.h"

namespace vox {

// ------------------------------------------------------------------ count

// The Euclidean length N = floor(|P1 - P0|) of eq. (1) for int16 lists:
// |d|^2 < 3 * 2^32 is rounded to float and its square root, within about
// 2^-23 relative, is within one of N; the integer corrections make it exact.
// (A float root here instead of the double one of the grid kernels: the
// Euclidean list kernels measured 3-10 % faster.)
__device__ __forceinline__ uint32_t list_euclid_length(const Seg& s) {
    uint64_t ss = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t d = (int64_t)s.p1[a] - (int64_t)s.p0[a];
        ss += (uint64_t)(d * d);
    }
    uint64_t r = (uint64_t)__builtin_sqrtf((float)ss);
    while (r * r > ss) --r;
    while ((r + 1) * (r + 1) <= ss) ++r;
    return (uint32_t)r;
}

// Samples of [k0, k1) (k0 < k1 <= N + 1, N >= 1) of an int16-range
// segment that start a new voxel under the Euclidean N: sample k0 from its
// remainders (one division unless k0 = 0), then one step a sample.
template <bool kFromStart>
__device__ __forceinline__ uint32_t euclid_walk(const Seg& g, uint32_t N, uint32_t k0, uint32_t k1) {
    const uint32_t two_n = 2u * N;
    uint32_t ta[3], f[3];
    bool moved = k0 == 0u;
    const float rcpd = rcp_down(two_n);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int32_t d = g.p1[ax] - g.p0[ax];
        const uint32_t neg = d < 0 ? 1u : 0u;
        ta[ax] = 2u * (uint32_t)(d < 0 ? -d : d);
        uint32_t r;
        if (kFromStart || k0 == 0u) {
            r = N - neg;
        } else if (N <= 32767u) {
            // 2 k0 a + N < 2^31, 2N < 2^16, quotient <= a < 2^15.
            uint32_t q;
            divmod_down(2u * k0 * (ta[ax] >> 1) + N - neg, two_n, rcpd, q, r);
        } else {
            r = (uint32_t)(((uint64_t)k0 * ta[ax] + N - neg) % two_n);
        }
        moved |= r < ta[ax];
        f[ax] = r - two_n;
    }
    uint32_t c = moved ? 1u : 0u;
    for (uint32_t k = k0 + 1u; k < k1; ++k) {
        bool mv = false;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const uint32_t t = f[ax] + ta[ax];
            const bool carry = t < ta[ax];
            f[ax] = carry ? t - two_n : t;
            mv |= carry;
        }
        c += mv ? 1u : 0u;
    }
    return c;
}

// Voxels of each segment under the Euclidean N of eq. (1) (consecutive
// duplicates removed): 1 + the steps k - 1 -> k, k = 1..N, that carry on
// some axis (a carry of r_a + 2a past 2N is exactly a move of that axis,
// since a <= N); 1 for a segment outside int16, which writes nothing.
// kLanes lanes share a segment, lane l walking samples [l S, (l + 1) S),
// S = ceil((N + 1) / kLanes), from one division at its first sample, and the
// lanes' counts are summed; the host takes more lanes a segment when there
// are fewer segments, so that a few long segments still spread over the
// chip.  Per axis the walk keeps f = r - 2N, whose add of 2a carries out of
// 32 bits exactly when r + 2a >= 2N.
template <bool kAligned8, int kLanes>
__global__ __launch_bounds__(kCountBlock) void k_euclid_counts(const int32_t* __restrict__ segs, int64_t n,
                                                              uint32_t* __restrict__ counts) {
    static_assert(kLanes >= 1 && kLanes <= kWave && (kWave % kLanes) == 0, "lanes a segment");
    const uint32_t sub = threadIdx.x % kLanes;
    const int64_t groups = (int64_t)gridDim.x * (kCountBlock / kLanes);
    // (Every lane of a group takes the same segments, so a group's lanes are
    // active together at the sum below.)
    for (int64_t i = ((int64_t)blockIdx.x * kCountBlock + threadIdx.x) / kLanes; i < n; i += groups) {
        const Seg g = load_seg<kAligned8>(segs, i);
        uint32_t c = 0;
        if (!in_int16(g)) {
            c = sub == 0 ? 1u : 0u;
        } else {
            const uint32_t N = list_euclid_length(g);
            const uint32_t S = (N + (uint32_t)kLanes) / (uint32_t)kLanes;
            const uint32_t k0 = sub * S;
            const uint32_t k1 = k0 + S < N + 1u ? k0 + S : N + 1u;
            if (N == 0u) {
                c = sub == 0 ? 1u : 0u;
            } else if (k0 < k1) {
                c = euclid_walk<kLanes == 1>(g, N, k0, k1);
            }
        }
#pragma unroll
        for (int o = kLanes / 2; o >= 1; o >>= 1) c += __shfl_xor(c, o, kLanes);
        if (sub == 0) counts[i] = c;
    }
}

// Voxel counts per segment (N + 1, or with the Euclidean N of eq. (1) the
// samples that start a new voxel) and their block sums; out-of-range flags
// (int16 lists: a coordinate outside int16; int32 lists: an axis spanning
// 2^30 or more).
template <bool kAligned8, int kKind>
__global__ __launch_bounds__(kCountBlock) void k_list_count(const int32_t* __restrict__ segs,
                                                            int64_t n, uint32_t* __restrict__ counts,
                                                            int64_t* __restrict__ block_sums,
                                                            int32_t* __restrict__ block_flags, int walk) {
    __shared__ int64_t red[kCountBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSegsPerCountBlock;
    int64_t sum = 0;
    int32_t flag = 0;
#pragma unroll
    for (int s = 0; s < kCountPerThread; ++s) {
        int64_t i = base + (int64_t)s * kCountBlock + threadIdx.x;
        if (i < n) {
            Seg g = load_seg<kAligned8>(segs, i);
            const bool inr = kKind == kListI32 ? span_below_2p30(g) : in_int16(g);
            int64_t c;
            if constexpr (kKind == kListEuclid) {
                // A thread walks its segment (walk), else from k_euclid_counts.
                if (walk) {
                    const uint32_t N = inr ? list_euclid_length(g) : 0u;
                    c = !inr || N == 0u ? 1 : (int64_t)euclid_walk<true>(g, N, 0u, N + 1u);
                } else {
                    c = counts[i];
                }
            } else {
                c = seg_length(g) + 1;
            }
            flag |= inr ? 0 : kStatusOutOfRange;
            // Counts above 2^32 - 1 only arise from out-of-range input.
            counts[i] = c > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)c;
            sum += c > 0xFFFFFFFFll ? 0xFFFFFFFFll : c;
        }
    }
    sum = block_sum<kCountBlock>(sum, red);
    int32_t f = (int32_t)block_sum<kCountBlock>((int64_t)flag, red);
    if (threadIdx.x == 0) {
        block_sums[blockIdx.x] = sum;
        block_flags[blockIdx.x] = f ? kStatusOutOfRange : 0;
    }
}

// ------------------------------------------------------- scan of partials

constexpr int kScanBlock = 1024;

// One block: exclusive scan of the per-block sums in place, the total into
// offsets[n] and *total, and the status word (out-of-range flags of the
// count blocks, capacity).
__global__ __launch_bounds__(kScanBlock) void k_list_scan(int64_t* __restrict__ block_sums,
                                                          const int32_t* __restrict__ block_flags,
                                                          int64_t nb, int64_t* __restrict__ offsets,
                                                          int64_t n, int64_t* __restrict__ total,
                                                          int32_t* __restrict__ status,
                                                          int64_t capacity, int want_voxels) {
    __shared__ int64_t lds[kScanBlock / kWave];
    int64_t carry = 0;
    int64_t flags = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanBlock) {
        int64_t i = c0 + threadIdx.x;
        int64_t v = i < nb ? block_sums[i] : 0;
        flags |= i < nb ? block_flags[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_sum<kScanBlock>(v, lds, tot);
        if (i < nb) block_sums[i] = carry + ex;
        carry += tot;
    }
    int32_t f = (int32_t)block_sum<kScanBlock>(flags, lds);
    if (threadIdx.x == 0) {
        offsets[n] = carry;
        *total = carry;
        int32_t st = f ? kStatusOutOfRange : 0;
        if (want_voxels && carry > capacity) st |= kStatusCapacity;
        *status = st;
    }
}

// --------------------------------------------------- offsets and tile map

// Count blocks up to this many: the offsets kernel sums the count blocks'
// partials itself (every block reads all of them, at most 3 KiB) and the
// scan kernel is not launched.  Measured per call: 100 000 segments 0.0255
// -> 0.0225 ms, 5 000 segments 0.016 -> 0.0135 ms; at 1 024 blocks (10^6
// segments) no gain for the Chebyshev lists and 4-6 % slower for the
// Euclidean ones, so larger calls keep the scan kernel.
constexpr int64_t kFusedScanMaxBlocks = 256;

// Same segment blocks as the count kernel.  Each sub-tile of kCountBlock
// consecutive segments is scanned by the block; every segment then records
// itself as the first segment of each output tile whose first voxel it
// holds.  kFused: the block's prefix, the total and the status come from the
// count blocks' raw sums and flags (what k_list_scan would write; block 0
// writes offsets[n], the total and the status word), else from k_list_scan.
template <bool kFused>
__global__ __launch_bounds__(kCountBlock) void k_list_offsets(
    int64_t n, const uint32_t* __restrict__ counts, const int64_t* __restrict__ block_prefix,
    const int32_t* __restrict__ block_flags, int64_t nb, int64_t capacity,
    int64_t* __restrict__ offsets, int32_t* __restrict__ tile_seg, int64_t tile_limit,
    int64_t* __restrict__ total, int32_t* __restrict__ status) {
    __shared__ int64_t lds[kCountBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kSegsPerCountBlock;
    int64_t carry, tot;
    bool tiles;  // only needed when voxels will be written
    if constexpr (kFused) {
        int64_t pre = 0, all = 0, fl = 0;
        for (int64_t b = threadIdx.x; b < nb; b += kCountBlock) {
            const int64_t v = block_prefix[b];
            all += v;
            pre += b < (int64_t)blockIdx.x ? v : 0;
            fl |= block_flags[b];
        }
        carry = block_sum<kCountBlock>(pre, lds);
        tot = block_sum<kCountBlock>(all, lds);
        int32_t st = block_sum<kCountBlock>(fl, lds) ? kStatusOutOfRange : 0;
        // (capacity > 0 exactly when voxels are wanted.)
        if (capacity > 0 && tot > capacity) st |= kStatusCapacity;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            offsets[n] = tot;
            *total = tot;
            *status = st;
        }
        tiles = tile_limit > 0 && st == 0;
    } else {
        carry = block_prefix[blockIdx.x];
        tiles = tile_limit > 0 && *status == 0;
        tot = *total;
    }
    const int64_t ntiles = tot < tile_limit * kListTile ? (tot + kListTile - 1) / kListTile : tile_limit;
    for (int s = 0; s < kCountPerThread; ++s) {
        int64_t i = base + (int64_t)s * kCountBlock + threadIdx.x;
        int64_t c = i < n ? (int64_t)counts[i] : 0;
        int64_t sub;
        int64_t ex = block_exclusive_sum<kCountBlock>(c, lds, sub);
        int64_t off = carry + ex;
        if (i < n) {
            offsets[i] = off;
            if (tiles) {
                int64_t t0 = (off + kListTile - 1) / kListTile;
                int64_t t1 = (off + c - 1) / kListTile;  // inclusive
                if (t1 >= ntiles) t1 = ntiles - 1;
                for (int64_t t = t0; t <= t1; ++t) tile_seg[t] = (int32_t)i;
            }
        }
        carry += sub;
    }
}

// ---------------------------------------------------- one-block lists

// Lists of at most kSegsPerCountBlock segments: the count, scan and offsets
// kernels in one block (a call is then two launches with the voxel kernel).
// Writes what those three write: counts, offsets[0..n], the total, the
// status word (range flags, capacity) and the tile map (here tile-parallel).
template <bool kAligned8, int kKind>
__global__ __launch_bounds__(kCountBlock) void k_list_one_block(
    const int32_t* __restrict__ segs, int64_t n, uint32_t* __restrict__ counts, int64_t* __restrict__ offsets,
    int32_t* __restrict__ tile_seg, int64_t tile_limit, int64_t* __restrict__ total_p,
    int32_t* __restrict__ status, int64_t capacity, int want_voxels) {
    __shared__ int64_t lds[kCountBlock / kWave];
    __shared__ int64_t soff[kSegsPerCountBlock + 1];
    int64_t c[kCountPerThread];
    int64_t flag = 0;
#pragma unroll
    for (int s = 0; s < kCountPerThread; ++s) {
        const int64_t i = (int64_t)s * kCountBlock + threadIdx.x;
        c[s] = 0;
        if (i < n) {
            Seg g = load_seg<kAligned8>(segs, i);
            const bool inr = kKind == kListI32 ? span_below_2p30(g) : in_int16(g);
            int64_t v;
            if constexpr (kKind == kListEuclid) {
                v = counts[i];  // from k_euclid_counts
            } else {
                v = seg_length(g) + 1;
            }
            flag |= inr ? 0 : kStatusOutOfRange;
            c[s] = v > 0xFFFFFFFFll ? 0xFFFFFFFFll : v;
            counts[i] = (uint32_t)c[s];
        }
    }
    const int64_t flags = block_sum<kCountBlock>(flag, lds);
    // Offsets, as the scan and offsets kernels would write them.
    int64_t carry = 0;
    int64_t off[kCountPerThread];
#pragma unroll
    for (int s = 0; s < kCountPerThread; ++s) {
        int64_t sub;
        off[s] = carry + block_exclusive_sum<kCountBlock>(c[s], lds, sub);
        const int64_t i = (int64_t)s * kCountBlock + threadIdx.x;
        if (i < n) {
            offsets[i] = off[s];
            soff[i] = off[s];
        }
        carry += sub;
    }
    const int64_t tot = carry;
    int32_t st = flags ? kStatusOutOfRange : 0;
    if (want_voxels && tot > capacity) st |= kStatusCapacity;
    if (threadIdx.x == 0) {
        offsets[n] = tot;
        *total_p = tot;
        *status = st;
    }
    __syncthreads();  // soff complete
    if (tile_limit > 0 && st == 0) {
        // Tile t starts in the segment holding voxel t * kListTile: the
        // largest i with offsets[i] <= t * kListTile (every segment has at
        // least one voxel, so the offsets increase strictly).  One tile per
        // thread at a time, so one long segment spreads over the block.
        const int64_t ntiles = tot < tile_limit * kListTile ? (tot + kListTile - 1) / kListTile : tile_limit;
        for (int64_t t = threadIdx.x; t < ntiles; t += kCountBlock) {
            const int64_t j = t * kListTile;
            int lo = 0, hi = (int)n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (soff[mid] <= j) lo = mid; else hi = mid - 1;
            }
            tile_seg[t] = lo;
        }
    }
}

// Tile map for many tiles, one thread per tile: tile t starts in the
// segment holding voxel t * kListTile, the largest i with offsets[i] <=
// t * kListTile (found by binary search over the n offsets).
__global__ __launch_bounds__(kCountBlock) void k_list_tiles(const int64_t* __restrict__ offsets, int64_t n,
                                                            int32_t* __restrict__ tile_seg, int64_t tile_limit,
                                                            const int64_t* __restrict__ total_p,
                                                            const int32_t* __restrict__ status) {
    if (*status != 0) return;
    const int64_t tot = *total_p;
    const int64_t ntiles = tot < tile_limit * kListTile ? (tot + kListTile - 1) / kListTile : tile_limit;
    const int64_t t = (int64_t)blockIdx.x * kCountBlock + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t j = t * kListTile;
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= j) lo = mid; else hi = mid - 1;
    }
    tile_seg[t] = (int32_t)lo;
}

// ------------------------------------------------------------ voxel tiles

// One tile = kListTile consecutive output voxels [j0, j1).  Its segments
// s0..s1 are staged in LDS, at most kWinSegs at a time, each as its
// stepping state at k = 0 (SegStart) with its offset relative to j0; lane t
// computes voxels j0 + t*P .. j0 + t*P + P - 1 (P = kListPerThread),
// stepping exactly from one voxel to the next and loading the following
// segment's state when the voxel index reaches its offset.  A tile with
// more segments than a window holds (segments shorter than kListTile /
// kWinSegs voxels on average) is done in several windows, each lane
// computing the voxels of its P that fall in the window; LDS sized for the
// usual case keeps many blocks on a CU.
//
// The stepping of eq. (3) per axis, for direction sign m (0 or all ones)
// and r = (2 k a + N - neg) mod 2N: the coordinate is kept as c' = c ^ m,
// which grows by one on every carry whichever the sign (for m = all ones,
// c' = -c - 1), and the remainder as f = r - 2N (mod 2^32), so that
// f + 2a carries out of 32 bits exactly when r + 2a >= 2N: one add with
// carry, one add of the carry to c', one conditional subtract of 2N.
struct SegStart {
    uint32_t c[3];     // p0 ^ m per axis
    uint32_t f[3];     // r(0) - 2N = N - neg - 2N (0 for a point)
    uint32_t ta[3];    // 2 |d_a|
    uint32_t two_n;    // 2N
    uint32_t neg;      // sign bits of d, axis a at bit a
    uint32_t pad;
};
constexpr int kWinSegs = 256;

// T = int16_t: coordinates in int16 (differences below 2^16); T = int32_t:
// every axis difference below 2^30 (checked by the count kernel).  The int16
// kernel is held to 64 VGPRs (eight waves a SIMD, which its 13 KiB of LDS
// allows); the int32 kernel's 25 KiB of LDS allows six blocks a CU anyway.
template <bool kAligned8, typename T>
__global__ __launch_bounds__(kListBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 2 ? 8 : 1)))
void k_list_voxels(
    const int32_t* __restrict__ segs, int64_t n, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ tile_seg, T* __restrict__ voxels,
    const int64_t* __restrict__ total_p, const int32_t* __restrict__ status) {
    constexpr int kSegWords = (int)(kWinSegs * sizeof(SegStart) / 4);
    constexpr int kVoxBytes = 3 * (int)sizeof(T);
    constexpr int kLaneWords = kListPerThread * kVoxBytes / 4;  // a lane's staged voxels
    constexpr int kStageWords = (int)kListTile * kVoxBytes / 4;
    // The staged segments and the output stage share LDS (the segments are
    // dead once every lane has its voxels): 13 KiB a block for int16 lists,
    // 25 KiB for int32 lists.
    __shared__ __align__(16) uint32_t lds_raw[kSegWords > kStageWords ? kSegWords : kStageWords];
    __shared__ int32_t srel[kWinSegs + 1];
    SegStart* sseg = reinterpret_cast<SegStart*>(lds_raw);
    uint32_t* stage = lds_raw;
    static_assert(sizeof(SegStart) % 16 == 0 && (kListPerThread * kVoxBytes) % 4 == 0, "packing");

    if (*status != 0) return;
    const int64_t total = *total_p;
    const int64_t tile = blockIdx.x;
    const int64_t j0 = tile * kListTile;
    if (j0 >= total) return;
    const int64_t j1 = j0 + kListTile < total ? j0 + kListTile : total;
    const int64_t ntiles = (total + kListTile - 1) / kListTile;
    const int32_t s0 = tile_seg[tile];
    int32_t s1 = tile + 1 < ntiles ? tile_seg[tile + 1] : (int32_t)(n - 1);
    const int nseg = s1 - s0 + 1;  // <= kListTile + 1

    const int first = threadIdx.x * kListPerThread;  // tile-relative voxel
    const int count = (int)(j1 - j0);
    T out[kListPerThread * 3];
    // Window w: the tile's segments [w, w + m); srel[i] is the offset of
    // segment w + i relative to j0 (srel[m]: of the segment after the window,
    // or the total), so the window's voxels are [srel[0], srel[m]).  Almost
    // every tile is one window (kOne: every voxel of the lane's P lies in it).
    auto run_window = [&](int w, int m, auto one, auto full) {
        constexpr bool kOne = decltype(one)::value;
        constexpr bool kFull = decltype(full)::value;  // a tile of kListTile voxels, one window
        for (int i = threadIdx.x; i < m; i += kListBlock) {
            const Seg g = load_seg<kAligned8>(segs, (int64_t)s0 + w + i);
            SegStart st;
            uint32_t N = 0, neg[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                // (int32 end points: the difference is formed without
                // overflow and is below 2^30 in magnitude.)
                const uint32_t d = (uint32_t)g.p1[ax] - (uint32_t)g.p0[ax];
                neg[ax] = (int32_t)d < 0 ? 1u : 0u;
                const uint32_t a = (int32_t)d < 0 ? 0u - d : d;
                st.ta[ax] = 2u * a;
                N = a > N ? a : N;
            }
            st.two_n = 2u * N;
            st.neg = neg[0] | (neg[1] << 1) | (neg[2] << 2);
            st.pad = 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                st.c[ax] = (uint32_t)g.p0[ax] ^ (0u - neg[ax]);
                st.f[ax] = N ? (N - neg[ax]) - 2u * N : 0u;
            }
            sseg[i] = st;
        }
        for (int i = threadIdx.x; i <= m; i += kListBlock) {
            const int64_t si = (int64_t)s0 + w + i;
            int64_t o = si <= n ? offsets[si] : total;
            int64_t rel = o - j0;
            // A tile's own segments start within [-(2^30 - 1), kListTile].
            rel = rel < -(1ll << 30) ? -(1ll << 30) : (rel > (1ll << 30) ? (1ll << 30) : rel);
            srel[i] = (int32_t)rel;
        }
        __syncthreads();

        // This lane's voxels inside the window: [lo, hi).
        int lo = first, hi = kFull ? first + kListPerThread : (first + kListPerThread < count ? first + kListPerThread : count);
        if constexpr (!kOne) {
            const int wlo = srel[0], whi = srel[m];
            lo = first > wlo ? first : wlo;
            hi = hi < whi ? hi : whi;
        }
        if (lo >= hi) return;
        // Segment of voxel lo: largest s with srel[s] <= lo.
        int a_ = 0, b_ = m - 1;
        while (a_ < b_) {
            int mid = (a_ + b_ + 1) >> 1;
            if (srel[mid] <= lo) a_ = mid; else b_ = mid - 1;
        }
        int s = a_;
        int next = srel[s + 1];
        SegStart st = sseg[s];
        uint32_t mk[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) mk[ax] = 0u - ((st.neg >> ax) & 1u);
        const uint32_t k = (uint32_t)(lo - srel[s]);
        if (k != 0u) {
            // Voxel k of the segment (k <= N, so N >= 1): c' = c'(0) + q.
            uint32_t a[3], neg[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                a[ax] = st.ta[ax] >> 1;
                neg[ax] = (st.neg >> ax) & 1u;
            }
            AxisStep as[3];
            axis_init3(a, neg, st.two_n >> 1, k, as);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                st.c[ax] += as[ax].q;
                st.f[ax] = as[ax].r - st.two_n;
            }
        }
#pragma unroll
        for (int v = 0; v < kListPerThread; ++v) {
            const int j = first + v;
            if (j >= hi || (!kOne && j < lo)) continue;
            // (Never at j = lo: the search found the segment holding voxel
            // lo, and every segment has at least one voxel.)
            if (j > lo && j >= next) {
                // First voxel of the following segment (inside the window, as
                // j < hi <= srel[m]): its state at k = 0.
                ++s;
                next = srel[s + 1];
                st = sseg[s];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) mk[ax] = 0u - ((st.neg >> ax) & 1u);
            }
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                out[v * 3 + ax] = (T)(int32_t)(st.c[ax] ^ mk[ax]);
                const uint32_t t = st.f[ax] + st.ta[ax];
                const bool carry = t < st.ta[ax];
                st.f[ax] = carry ? t - st.two_n : t;
                st.c[ax] += carry ? 1u : 0u;
            }
        }
    };
    if (nseg <= kWinSegs && count == (int)kListTile) {
        run_window(0, nseg, std::integral_constant<bool, true>{}, std::integral_constant<bool, true>{});
    } else if (nseg <= kWinSegs) {
        run_window(0, nseg, std::integral_constant<bool, true>{}, std::integral_constant<bool, false>{});
    } else {
        for (int w = 0; w < nseg; w += kWinSegs) {
            if (w > 0) __syncthreads();  // the previous window is read
            run_window(w, nseg - w < kWinSegs ? nseg - w : kWinSegs, std::integral_constant<bool, false>{},
                       std::integral_constant<bool, false>{});
        }
    }
    __syncthreads();  // the staged segments are dead from here
    if (first < count) {
        // Stage: lane t owns its 3*P coordinates, kLaneWords words at word
        // kLaneWords*t.
        uint32_t* dst = stage + kLaneWords * threadIdx.x;
        if constexpr (sizeof(T) == 2) {
#pragma unroll
            for (int w = 0; w < kLaneWords; ++w)
                dst[w] = (uint32_t)(uint16_t)out[2 * w] | ((uint32_t)(uint16_t)out[2 * w + 1] << 16);
        } else {
#pragma unroll
            for (int w = 0; w < kLaneWords; ++w) dst[w] = (uint32_t)out[w];
        }
    }
    __syncthreads();

    // Write the tile: bytes [B*j0, B*j1), B = 3*sizeof(T).  j0 is a multiple
    // of kListTile, so the start is 16-byte aligned whenever `voxels` is.
    const int64_t bytes = kVoxBytes * (j1 - j0);
    uint8_t* gbase = reinterpret_cast<uint8_t*>(voxels) + kVoxBytes * j0;
    const int64_t n16 = bytes / 16;
    const uint4* src = reinterpret_cast<const uint4*>(stage);
    uint4* gdst = reinterpret_cast<uint4*>(gbase);
    for (int64_t c = threadIdx.x; c < n16; c += kListBlock) gdst[c] = src[c];
    // Tail (only in the last tile): 2-byte pieces.
    const int64_t tail0 = n16 * 16;
    const uint16_t* src16 = reinterpret_cast<const uint16_t*>(stage);
    uint16_t* dst16 = reinterpret_cast<uint16_t*>(gbase);
    for (int64_t c = tail0 / 2 + threadIdx.x; c < bytes / 2; c += kListBlock) dst16[c] = src16[c];
}

// The samples k, k + L, k + 2L, ... of one segment under the Euclidean N as
// taken by one of its L = kLanes lanes, stepped as the tile kernel steps (per axis:
// c' = coordinate ^ sign mask grows by dq + carry, f = r - 2N carries out of
// 32 bits exactly when r + dr >= 2N).  A sample k >= 1 starts a new voxel
// when some axis moved from k - 1 to k, that is when r_a(k) < 2a_a for some
// a, i.e. f_a < 2a_a - 2N as signed values (|2N| < 2^31).
template <int kLanes>
struct ListSamples {
    uint32_t c[3], f[3], h[3], dq[3], dr[3], mk[3];
    uint32_t N, two_n;

    // Sample k of segment g (length n); returns whether it starts a voxel.
    __device__ __forceinline__ bool start(const Seg& g, uint32_t n, uint32_t k) {
        N = n;
        two_n = 2u * n;
        uint32_t two_a[3], num0[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int32_t d = g.p1[ax] - g.p0[ax];
            mk[ax] = d < 0 ? ~0u : 0u;
            two_a[ax] = 2u * (uint32_t)(d < 0 ? -d : d);
            num0[ax] = n - (d < 0 ? 1u : 0u);
            h[ax] = two_a[ax] - two_n;
        }
        uint32_t q[3], r[3];
        if (n == 0) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) q[ax] = r[ax] = dq[ax] = dr[ax] = 0;
        } else if (n <= 32767u) {
            const float rcpd = rcp_down(two_n);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                divmod_down(__umul24(k, two_a[ax]) + num0[ax], two_n, rcpd, q[ax], r[ax]);
                divmod_down(kLanes * two_a[ax], two_n, rcpd, dq[ax], dr[ax]);
            }
        } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const uint64_t num = (uint64_t)k * two_a[ax] + num0[ax];
                q[ax] = (uint32_t)(num / two_n);
                r[ax] = (uint32_t)(num - (uint64_t)q[ax] * two_n);
                const uint32_t s = kLanes * two_a[ax];
                dq[ax] = s / two_n;
                dr[ax] = s - dq[ax] * two_n;
            }
        }
        bool moved = k == 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            c[ax] = ((uint32_t)g.p0[ax] ^ mk[ax]) + q[ax];
            f[ax] = r[ax] - two_n;
            moved |= (int32_t)f[ax] < (int32_t)h[ax];
        }
        return moved;
    }

    // Moves on by kLanes samples; returns whether the sample starts a voxel.
    __device__ __forceinline__ bool next() {
        bool moved = false;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const uint32_t t = f[ax] + dr[ax];
            const bool carry = t < dr[ax];
            f[ax] = carry ? t - two_n : t;
            c[ax] += dq[ax] + (carry ? 1u : 0u);
            moved |= (int32_t)f[ax] < (int32_t)h[ax];
        }
        return moved;
    }

    __device__ __forceinline__ int32_t coord(int ax) const { return (int32_t)(c[ax] ^ mk[ax]); }
};

// Lists with the Euclidean N of eq. (1).  A wave takes 64 / kLanes segments,
// kLanes lanes each; a segment's lanes take its samples k = 0..N kLanes at a
// time, each stepping its own samples and deciding alone whether its sample
// starts a new voxel (ListSamples); a ballot of those decisions places the
// kept voxels, and consecutive lanes write consecutive voxels.
template <bool kAligned8, int kLanes>
__global__ __launch_bounds__(kCountBlock) void k_list_voxels_euclid(
    const int32_t* __restrict__ segs, int64_t n, const int64_t* __restrict__ offsets,
    int16_t* __restrict__ voxels, const int32_t* __restrict__ status) {
    if (*status != 0) return;
    static_assert(kLanes >= 2 && kLanes <= kWave && (kWave % kLanes) == 0, "lanes a segment");
    constexpr int kSlots = kWave / kLanes;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t sub = lane % kLanes;
    const uint32_t slot = lane / kLanes;
    const uint64_t slot_bits = (kLanes == kWave ? ~0ull : ((1ull << kLanes) - 1)) << (kLanes * slot);
    const int64_t step = (int64_t)gridDim.x * (kCountBlock / kWave) * kSlots;
    for (int64_t i0 = ((int64_t)blockIdx.x * (kCountBlock / kWave) + threadIdx.x / kWave) * kSlots; i0 < n;
         i0 += step) {
        const int64_t i = i0 + slot;
        const bool valid = i < n;
        Seg g = {};
        if (valid) g = load_seg<kAligned8>(segs, i);
        ListSamples<kLanes> s;
        bool moved = s.start(g, list_euclid_length(g), sub);
        int16_t* out = voxels + 3 * (valid ? offsets[i] : 0);
        for (uint32_t c0 = 0; __ballot(valid && c0 <= s.N) != 0; c0 += kLanes) {
            if (c0 != 0) moved = s.next();
            const bool keep = moved && valid && c0 + sub <= s.N;
            const uint64_t m = __ballot(keep) & slot_bits;
            if (keep) {
                const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                int16_t* o = out + 3 * before;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) o[ax] = (int16_t)s.coord(ax);
            }
            out += 3 * __popcll(m);
        }
    }
}

// ---------------------------------------------------------------- host side

size_t list_workspace_bytes(int64_t n, int64_t capacity) {
    int64_t nb = (n + kSegsPerCountBlock - 1) / kSegsPerCountBlock;
    if (nb < 1) nb = 1;
    int64_t ntiles = (capacity + kListTile - 1) / kListTile;
    size_t b = kAlign;                                  // status, total
    b += align_up((size_t)nb * sizeof(int64_t));         // block sums
    b += align_up((size_t)nb * sizeof(int32_t));         // block flags
    b += align_up((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));  // counts
    b += align_up((size_t)(ntiles + 1) * sizeof(int32_t));      // tile map
    return b;
}

ListWork list_workspace(void* d_work, int64_t n, int64_t capacity) {
    ListWork w;
    int64_t nb = (n + kSegsPerCountBlock - 1) / kSegsPerCountBlock;
    if (nb < 1) nb = 1;
    uint8_t* p = static_cast<uint8_t*>(d_work);
    w.status = reinterpret_cast<int32_t*>(p);
    w.total = reinterpret_cast<int64_t*>(p + 8);
    p += kAlign;
    w.block_sums = reinterpret_cast<int64_t*>(p);
    p += align_up((size_t)nb * sizeof(int64_t));
    w.block_flags = reinterpret_cast<int32_t*>(p);
    p += align_up((size_t)nb * sizeof(int32_t));
    w.counts = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    w.tile_seg = reinterpret_cast<int32_t*>(p);
    w.nb = nb;
    w.ntiles = (capacity + kListTile - 1) / kListTile;
    return w;
}

template <int kLanes>
static void euclid_counts(const int32_t* segs, int64_t n, bool aligned8, uint32_t* counts, hipStream_t stream) {
    int64_t blocks = (n * kLanes + kCountBlock - 1) / kCountBlock;
    if (blocks > 16384) blocks = 16384;
    if (aligned8)
        k_euclid_counts<true, kLanes><<<dim3((unsigned)blocks), kCountBlock, 0, stream>>>(segs, n, counts);
    else
        k_euclid_counts<false, kLanes><<<dim3((unsigned)blocks), kCountBlock, 0, stream>>>(segs, n, counts);
}

// Euclidean counts into w.counts (n >= 1): one lane a segment from 65 536
// segments on (a thread per segment already fills the chip), more lanes a
// segment below that, and more again while a lane would walk more than
// about 256 samples (voxels a segment taken from the caller's capacity, the
// workspace's tile count; none when only the total is asked for).
static int euclid_count_lanes(int64_t n, const ListWork& w) {
    int lanes = n >= 65536 ? 1 : (n >= 16384 ? 4 : (n >= 4096 ? 16 : 64));
    const int64_t avg = w.ntiles * kListTile / n;
    while (lanes < kWave && (int64_t)lanes * 256 < avg) lanes *= 4;
    return lanes;
}

static void launch_euclid_counts(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w,
                                 hipStream_t stream) {
    const int lanes = euclid_count_lanes(n, w);
    if (lanes == 1)
        euclid_counts<1>(segs, n, aligned8, w.counts, stream);
    else if (lanes == 4)
        euclid_counts<4>(segs, n, aligned8, w.counts, stream);
    else if (lanes == 16)
        euclid_counts<16>(segs, n, aligned8, w.counts, stream);
    else
        euclid_counts<64>(segs, n, aligned8, w.counts, stream);
}

template <int kKind>
static void list_count(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w, hipStream_t stream) {
    // One lane a segment and short segments (at most 32 voxels on average by
    // the capacity, or none given): the count kernel walks the segments
    // itself, one launch fewer (1 M segments of 9-14 samples 0.018 -> 0.014
    // ms).  Longer ones keep k_euclid_counts, a thread per segment rather
    // than per four (1 M segments of 64-110 samples: 0.041 against 0.044 ms).
    const int walk = kKind == kListEuclid && n > 0 && euclid_count_lanes(n, w) == 1 &&
                             w.ntiles * kListTile / n <= 32
                         ? 1
                         : 0;
    if (kKind == kListEuclid && n > 0 && !walk) launch_euclid_counts(segs, n, aligned8, w, stream);
    // n == 0: one block that writes a zero sum and no flag.
    dim3 grid(n == 0 ? 1u : (unsigned)w.nb);
    if (aligned8)
        k_list_count<true, kKind><<<grid, kCountBlock, 0, stream>>>(segs, n, w.counts, w.block_sums,
                                                                     w.block_flags, walk);
    else
        k_list_count<false, kKind><<<grid, kCountBlock, 0, stream>>>(segs, n, w.counts, w.block_sums,
                                                                      w.block_flags, walk);
}

hipError_t launch_list_count(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w,
                             hipStream_t stream, ListKind kind) {
    KernelTimer timer(kind == kListEuclid ? "list_count_euclid" : (kind == kListI32 ? "list_count32" : "list_count"),
                      stream);
    if (kind == kListEuclid)
        list_count<kListEuclid>(segs, n, aligned8, w, stream);
    else if (kind == kListI32)
        list_count<kListI32>(segs, n, aligned8, w, stream);
    else
        list_count<kListI16>(segs, n, aligned8, w, stream);
    return hipGetLastError();
}

// Tile maps up to this many tiles are written by the one-block kernel
// itself; larger ones by k_list_tiles, one thread per tile.
constexpr int64_t kOneBlockMaxTiles = 4096;

template <int kKind>
static void list_one_block(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w, int64_t* offsets,
                           int64_t capacity, bool want_voxels, hipStream_t stream) {
    // (The Euclidean lists are written per segment: no output tiles.)
    const int64_t tiles = want_voxels && kKind != kListEuclid ? (capacity + kListTile - 1) / kListTile : 0;
    const int64_t tile_limit = tiles <= kOneBlockMaxTiles ? tiles : 0;
    if (kKind == kListEuclid && n > 0) launch_euclid_counts(segs, n, aligned8, w, stream);
    if (aligned8)
        k_list_one_block<true, kKind><<<1, kCountBlock, 0, stream>>>(segs, n, w.counts, offsets, w.tile_seg,
                                                                      tile_limit, w.total, w.status, capacity,
                                                                      want_voxels ? 1 : 0);
    else
        k_list_one_block<false, kKind><<<1, kCountBlock, 0, stream>>>(segs, n, w.counts, offsets, w.tile_seg,
                                                                       tile_limit, w.total, w.status, capacity,
                                                                       want_voxels ? 1 : 0);
    if (tiles > kOneBlockMaxTiles)
        k_list_tiles<<<dim3((unsigned)((tiles + kCountBlock - 1) / kCountBlock)), kCountBlock, 0, stream>>>(
            offsets, n, w.tile_seg, tiles, w.total, w.status);
}

hipError_t launch_list_one_block(const int32_t* segs, int64_t n, bool aligned8, const ListWork& w,
                                 int64_t* offsets, int64_t capacity, bool want_voxels, hipStream_t stream,
                                 ListKind kind) {
    KernelTimer timer("list_one_block", stream);
    if (kind == kListEuclid)
        list_one_block<kListEuclid>(segs, n, aligned8, w, offsets, capacity, want_voxels, stream);
    else if (kind == kListI32)
        list_one_block<kListI32>(segs, n, aligned8, w, offsets, capacity, want_voxels, stream);
    else
        list_one_block<kListI16>(segs, n, aligned8, w, offsets, capacity, want_voxels, stream);
    return hipGetLastError();
}

hipError_t launch_list_scan(const ListWork& w, int64_t n, int64_t* offsets, int64_t capacity,
                            bool want_voxels, hipStream_t stream) {
    if (n >= 1 && w.nb <= kFusedScanMaxBlocks) return hipSuccess;  // done by the offsets kernel
    KernelTimer timer("list_scan", stream);
    k_list_scan<<<1, kScanBlock, 0, stream>>>(w.block_sums, w.block_flags, w.nb, offsets, n, w.total,
                                              w.status, capacity, want_voxels ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_list_offsets(int64_t n, int64_t* offsets, const ListWork& w, int64_t capacity,
                               bool want_voxels, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int64_t tiles = want_voxels ? (capacity + kListTile - 1) / kListTile : 0;
    // Segments of more than four tiles on average: the tile map from
    // k_list_tiles (one thread per tile) rather than one thread per segment.
    const bool per_tile = tiles > 4 * n;
    KernelTimer timer("list_offsets", stream);
    if (w.nb <= kFusedScanMaxBlocks)
        k_list_offsets<true><<<dim3((unsigned)w.nb), kCountBlock, 0, stream>>>(
            n, w.counts, w.block_sums, w.block_flags, w.nb, capacity, offsets, w.tile_seg, per_tile ? 0 : tiles,
            w.total, w.status);
    else
        k_list_offsets<false><<<dim3((unsigned)w.nb), kCountBlock, 0, stream>>>(
            n, w.counts, w.block_sums, w.block_flags, w.nb, capacity, offsets, w.tile_seg, per_tile ? 0 : tiles,
            w.total, w.status);
    if (per_tile)
        k_list_tiles<<<dim3((unsigned)((tiles + kCountBlock - 1) / kCountBlock)), kCountBlock, 0, stream>>>(
            offsets, n, w.tile_seg, tiles, w.total, w.status);
    return hipGetLastError();
}

hipError_t launch_list_voxels(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                              const ListWork& w, int16_t* voxels, int64_t capacity,
                              int64_t tiles_to_launch, hipStream_t stream) {
    (void)capacity;
    if (n == 0 || tiles_to_launch <= 0) return hipSuccess;
    dim3 grid((unsigned)tiles_to_launch);
    KernelTimer timer("list_voxels", stream);
    if (aligned8)
        k_list_voxels<true, int16_t><<<grid, kListBlock, 0, stream>>>(segs, n, offsets, w.tile_seg, voxels,
                                                                      w.total, w.status);
    else
        k_list_voxels<false, int16_t><<<grid, kListBlock, 0, stream>>>(segs, n, offsets, w.tile_seg, voxels,
                                                                       w.total, w.status);
    return hipGetLastError();
}

hipError_t launch_list_voxels32(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                                const ListWork& w, int32_t* voxels, int64_t tiles_to_launch, hipStream_t stream) {
    if (n == 0 || tiles_to_launch <= 0) return hipSuccess;
    dim3 grid((unsigned)tiles_to_launch);
    KernelTimer timer("list_voxels32", stream);
    if (aligned8)
        k_list_voxels<true, int32_t><<<grid, kListBlock, 0, stream>>>(segs, n, offsets, w.tile_seg, voxels,
                                                                      w.total, w.status);
    else
        k_list_voxels<false, int32_t><<<grid, kListBlock, 0, stream>>>(segs, n, offsets, w.tile_seg, voxels,
                                                                       w.total, w.status);
    return hipGetLastError();
}

template <int kLanes>
static void list_voxels_euclid(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                               const ListWork& w, int16_t* voxels, hipStream_t stream) {
    constexpr int kSegsPerBlock = kCountBlock / kLanes;
    int64_t blocks = (n + kSegsPerBlock - 1) / kSegsPerBlock;
    if (blocks > 16384) blocks = 16384;
    if (aligned8)
        k_list_voxels_euclid<true, kLanes><<<dim3((unsigned)blocks), kCountBlock, 0, stream>>>(segs, n, offsets,
                                                                                               voxels, w.status);
    else
        k_list_voxels_euclid<false, kLanes><<<dim3((unsigned)blocks), kCountBlock, 0, stream>>>(segs, n, offsets,
                                                                                                voxels, w.status);
}

// Lanes a segment for the Euclidean list kernel: about one pass of the
// lanes per segment (at least 4 lanes, a pass covering up to 8 voxels a
// lane), and at least 65 536 lanes in all so that a few long segments still
// spread over the chip.  The voxels per segment are taken from the caller's
// capacity (the workspace's tile count), so an oversized buffer only costs
// speed.
static int euclid_list_lanes(int64_t n, int64_t capacity) {
    const int64_t avg = capacity / n;
    int lanes = 4;
    while (lanes < kWave && ((int64_t)lanes * 8 < avg || n * lanes < 65536)) lanes *= 2;
    return lanes;
}

hipError_t launch_list_voxels_euclid(const int32_t* segs, int64_t n, bool aligned8, const int64_t* offsets,
                                     const ListWork& w, int16_t* voxels, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    KernelTimer timer("list_voxels_euclid", stream);
    switch (euclid_list_lanes(n, w.ntiles * kListTile)) {
        case 4: list_voxels_euclid<4>(segs, n, aligned8, offsets, w, voxels, stream); break;
        case 8: list_voxels_euclid<8>(segs, n, aligned8, offsets, w, voxels, stream); break;
        case 16: list_voxels_euclid<16>(segs, n, aligned8, offsets, w, voxels, stream); break;
        case 32: list_voxels_euclid<32>(segs, n, aligned8, offsets, w, voxels, stream); break;
        default: list_voxels_euclid<64>(segs, n, aligned8, offsets, w, voxels, stream); break;
    }
    return hipGetLastError();
}

}  // namespace vox

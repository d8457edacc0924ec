// Bit-volume output through LDS bricks.
//
// The volume is cut into bricks of BX x BY x BZ voxels (powers of two, BX a
// multiple of 32 so brick rows are whole 32-bit words).  A brick's bits fit in
// one workgroup's LDS; the workgroup that owns a brick sets all of its voxels
// there and then writes the brick to HBM once with plain stores, which also
// clears it (no separate clear pass, no global atomics).
//
// Each segment is cut into pieces, one per brick it passes through.  As every
// coordinate of eq. (3) is monotone in k, the voxels of a segment inside one
// brick form a single k-interval, and the brick changes exactly when one
// coordinate crosses a brick boundary (exact helpers in vox_exact.h).
//
// Pipeline (one stream, no host synchronisation):
//   init      status word and work counter to zero
//   hist      per segment: count N+1, range check, walk its bricks and count
//             pieces per brick in an LDS histogram; one histogram row per
//             workgroup
//   colscan   per brick, exclusive prefix of the rows over workgroups, and
//             the brick's piece total
//   base      exclusive scan of the brick totals -> bin offsets
//   scatter   the same walk again, writing one 16-byte piece record (start
//             point, direction, k-window in the brick) into the brick's bin
//   fill      persistent workgroups take bricks from an atomic counter, set
//             the bits of every piece with LDS atomic OR and flush the brick
//             to the volume
#include "vox_device.h"
#include "vox_exact.h"
#include "vox_internal.h"

namespace vox {

// Barrier that waits for this wave's LDS traffic only, so global loads
// issued before it (prefetches) stay in flight.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Block-wide exclusive sum like block_exclusive_sum, synchronised with
// lds_barrier so that outstanding global loads are not waited for.
template <int kBlock>
__device__ __forceinline__ uint32_t block_exclusive_sum_lds(uint32_t v, uint32_t* lds, uint32_t& total) {
    constexpr int kWaves = kBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const uint32_t incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) lds[w] = incl;
    lds_barrier();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        const uint32_t x = lds[i];
        pre += (i < w) ? x : 0u;
        tot += x;
    }
    lds_barrier();
    total = tot;
    return pre + incl - v;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

typedef int16_t i16x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ kernels

__global__ void k_brick_init(int32_t* status, uint32_t* work_counter) {
    if (threadIdx.x == 0) {
        *status = 0;
        *work_counter = 0;
    }
}

// Segment range of histogram/scatter workgroup g.
__device__ __forceinline__ void seg_range(int64_t n, int g, int G, int64_t& lo, int64_t& hi) {
    int64_t per = (n + G - 1) / G;
    lo = (int64_t)g * per;
    hi = lo + per < n ? lo + per : n;
}

// A segment staged in LDS for the walk: end points as uint16 (every brick
// volume side is <= 16384).
struct StagedSeg {
    uint16_t p0[3];
    uint16_t p1[3];
};

constexpr int kStage = 4096;      // segments staged per round
constexpr int kOrderBins = 64;

// Staged segments ordered by their number of bricks, longest walks first, so
// the lanes of a wave walk segments of (nearly) equal piece counts: they all
// start together and finish together.  The count used is
// 1 + sum_a |brick_a(P1) - brick_a(P0)| (exact unless two axes cross at the
// same k), clamped to the last bucket.
struct Stage {
    StagedSeg seg[kStage];
    uint16_t order[kStage];
    uint32_t bins[kOrderBins];  // bucket sizes, then bucket cursors
    uint32_t nvalid;
};

__device__ __forceinline__ uint32_t order_bin(const StagedSeg& g, const BrickGeom& bg) {
    uint32_t est = 1;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int32_t db = ((int32_t)g.p1[ax] >> bg.lg[ax]) - ((int32_t)g.p0[ax] >> bg.lg[ax]);
        est += (uint32_t)(db < 0 ? -db : db);
    }
    return kOrderBins - 1 - (est < kOrderBins - 1 ? est : kOrderBins - 1);
}

// Loads segments [base, base + cnt) into the stage (all threads of the
// block), writes counts, flags out-of-volume segments, and builds the order
// of the in-volume ones.
template <bool kAligned8>
__device__ __forceinline__ void stage_segments(const int32_t* __restrict__ segs, int64_t base, uint32_t cnt,
                                               const BrickGeom& bg, Stage& st, int32_t* __restrict__ counts,
                                               bool& bad) {
    if (threadIdx.x < kOrderBins) st.bins[threadIdx.x] = 0;
    lds_barrier();
    // Bit t of `mine` marks this thread's t-th segment as in the volume.
    uint32_t mine = 0;
    int slot = 0;
    for (uint32_t t = threadIdx.x; t < cnt; t += kHistBlock, ++slot) {
        const Seg g = load_seg<kAligned8>(segs, base + t);
        if (counts) {
            const int64_t c = seg_length(g) + 1;
            counts[base + t] = (int32_t)(c > 0x7FFFFFFFll ? 0x7FFFFFFFll : c);
        }
        StagedSeg s;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            s.p0[ax] = (uint16_t)g.p0[ax];
            s.p1[ax] = (uint16_t)g.p1[ax];
        }
        st.seg[t] = s;
        if (in_volume(g, bg)) {
            mine |= 1u << slot;
            atomicAdd(&st.bins[order_bin(s, bg)], 1u);
        } else {
            bad = true;
        }
    }
    lds_barrier();
    if (threadIdx.x < kWave) {  // bucket offsets: one wave, one bucket per lane
        const uint32_t c = st.bins[threadIdx.x];
        const uint32_t incl = wave_inclusive_sum(c);
        st.bins[threadIdx.x] = incl - c;
        if (threadIdx.x == kWave - 1) st.nvalid = incl;
    }
    lds_barrier();
    slot = 0;
    for (uint32_t t = threadIdx.x; t < cnt; t += kHistBlock, ++slot) {
        if (mine & (1u << slot)) {
            const uint32_t pos = atomicAdd(&st.bins[order_bin(st.seg[t], bg)], 1u);
            st.order[pos] = (uint16_t)t;
        }
    }
    lds_barrier();
}
static_assert(kStage / kHistBlock <= 32, "one validity bit per staged segment and thread");

struct WalkState {
    AxisCross c[3];
    uint32_t N, klo;  // Chebyshev length, first k inside the current brick
};

__device__ __forceinline__ void walk_init(WalkState& w, const StagedSeg& g, const BrickGeom& bg) {
    int32_t p0[3], p1[3];
    uint32_t a[3], neg[3], N = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        p0[ax] = g.p0[ax];
        p1[ax] = g.p1[ax];
        const int32_t d = p1[ax] - p0[ax];
        neg[ax] = d < 0;
        a[ax] = (uint32_t)(d < 0 ? -d : d);
        N = a[ax] > N ? a[ax] : N;
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) cross_init(w.c[ax], p0[ax], p1[ax], a[ax], neg[ax], N, bg.lg[ax]);
    w.N = N;
    w.klo = 0;
}

// Walks the ordered staged segments: each wave takes the next 64 in order
// and steps all of them one brick at a time until the wave's last segment
// ends.  emit(brick id, klo, khi, staged index) per piece, [klo, khi] being
// the segment's k-window inside the brick.
template <typename Emit>
__device__ __forceinline__ void walk_ordered(const Stage& st, const BrickGeom& bg, Emit emit) {
    const uint32_t lane = __lane_id();
    const uint32_t nvalid = st.nvalid;
    for (uint32_t base = threadIdx.x - lane; base < nvalid; base += kHistBlock) {
        const uint32_t i = base + lane;
        bool active = i < nvalid;
        uint32_t j = 0;
        WalkState w;
        if (active) {
            j = st.order[i];
            walk_init(w, st.seg[j], bg);
        }
        while (__ballot(active)) {
            if (active) {
                uint32_t km = w.c[0].kn < w.c[1].kn ? w.c[0].kn : w.c[1].kn;
                km = km < w.c[2].kn ? km : w.c[2].kn;
                emit((uint32_t)((w.c[2].b * bg.nb[1] + w.c[1].b) * bg.nb[0] + w.c[0].b), w.klo,
                     km == kNever ? w.N : km - 1u, j);
                if (km == kNever) {
                    active = false;
                } else {
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax)
                        if (w.c[ax].kn == km) cross_step(w.c[ax]);
                    w.klo = km;
                }
            }
        }
    }
}

template <bool kAligned8>
__global__ __launch_bounds__(kHistBlock) void k_brick_hist(const int32_t* __restrict__ segs, int64_t n,
                                                           BrickGeom bg, uint32_t* __restrict__ hist,
                                                           int32_t* __restrict__ counts,
                                                           int32_t* __restrict__ status) {
    extern __shared__ uint32_t lh[];
    __shared__ Stage st;
    const uint32_t NB = bg.nbricks;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) lh[b] = 0;
    int64_t lo, hi;
    seg_range(n, blockIdx.x, gridDim.x, lo, hi);
    bool bad = false;
    for (int64_t base = lo; base < hi; base += kStage) {
        const uint32_t cnt = (uint32_t)(hi - base < kStage ? hi - base : kStage);
        stage_segments<kAligned8>(segs, base, cnt, bg, st, counts, bad);
        walk_ordered(st, bg, [&](uint32_t b, uint32_t, uint32_t, uint32_t) { atomicAdd(&lh[b], 1u); });
        lds_barrier();
    }
    if (bad) atomicOr(status, kStatusOutOfRange);
    lds_barrier();
    uint32_t* row = hist + (size_t)blockIdx.x * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) row[b] = lh[b];
}

constexpr int kColBins = 64;
constexpr int kColSplit = 4;  // row chunks per brick
constexpr int kColRows = (kHistRows + kColSplit - 1) / kColSplit;

// Block of 256 threads = 64 bricks x 4 row chunks: per brick, exclusive
// prefix of hist[g][b] over the G rows (in place) and the brick total.
__global__ __launch_bounds__(256) void k_brick_colscan(uint32_t* __restrict__ hist, int G, uint32_t NB,
                                                       uint32_t* __restrict__ totals) {
    __shared__ uint32_t part[kColSplit][kColBins];
    const int bl = threadIdx.x % kColBins;
    const int ch = threadIdx.x / kColBins;
    const uint32_t b = blockIdx.x * kColBins + bl;
    const int g0 = ch * kColRows;
    uint32_t v[kColRows];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
        const int g = g0 + r;
        v[r] = (b < NB && g < G) ? hist[(size_t)g * NB + b] : 0u;
        sum += v[r];
    }
    part[ch][bl] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (int c = 0; c < kColSplit; ++c) {
        run += c < ch ? part[c][bl] : 0u;
        tot += part[c][bl];
    }
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
        const int g = g0 + r;
        if (b < NB && g < G) hist[(size_t)g * NB + b] = run;
        run += v[r];
    }
    if (ch == 0 && b < NB) totals[b] = tot;
}

constexpr int kBaseBlock = 1024;

// One block: bin_base[b] = sum of totals before b; bin_base[NB] = total.
__global__ __launch_bounds__(kBaseBlock) void k_brick_base(const uint32_t* __restrict__ totals, uint32_t NB,
                                                           uint32_t* __restrict__ bin_base) {
    __shared__ uint32_t lds[kBaseBlock / kWave];
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < NB; c0 += kBaseBlock) {
        uint32_t i = c0 + threadIdx.x;
        uint32_t v = i < NB ? totals[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_sum<kBaseBlock>(v, lds, tot);
        if (i < NB) bin_base[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bin_base[NB] = carry;
}

// Piece record (16 bytes): start point, direction and the k-window inside
// its brick; everything the fill needs, so it reads records and never
// gathers segments.
struct Piece {
    uint16_t p0[3];
    int16_t d[3];
    uint16_t klo, khi;  // inclusive
};
static_assert(sizeof(Piece) == 16, "16-byte piece records");

template <bool kAligned8>
__global__ __launch_bounds__(kHistBlock) void k_brick_scatter(const int32_t* __restrict__ segs, int64_t n,
                                                              BrickGeom bg, const uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ bin_base,
                                                              Piece* __restrict__ recs) {
    extern __shared__ uint32_t cur[];
    __shared__ Stage st;
    const uint32_t NB = bg.nbricks;
    const uint32_t* row = hist + (size_t)blockIdx.x * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) cur[b] = bin_base[b] + row[b];
    int64_t lo, hi;
    seg_range(n, blockIdx.x, gridDim.x, lo, hi);
    bool bad = false;
    for (int64_t base = lo; base < hi; base += kStage) {
        const uint32_t cnt = (uint32_t)(hi - base < kStage ? hi - base : kStage);
        stage_segments<kAligned8>(segs, base, cnt, bg, st, nullptr, bad);
        walk_ordered(st, bg, [&](uint32_t b, uint32_t klo, uint32_t khi, uint32_t j) {
            const uint32_t pos = atomicAdd(&cur[b], 1u);
            const StagedSeg g = st.seg[j];
            Piece pc;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                pc.p0[ax] = g.p0[ax];
                pc.d[ax] = (int16_t)((int32_t)g.p1[ax] - (int32_t)g.p0[ax]);
            }
            pc.klo = (uint16_t)klo;
            pc.khi = (uint16_t)khi;
            recs[pos] = pc;
        });
        lds_barrier();
    }
}

// ------------------------------------------------------------------- fill

template <int LGX, int LGY, int LGZ>
struct BrickShape {
    static constexpr int kBXw = 1 << (LGX - 5);                       // words per row
    static constexpr uint32_t kWords = (uint32_t)kBXw << (LGY + LGZ);
    static constexpr size_t kBytes = (size_t)kWords * 4;
    static constexpr int kMaxLg = LGX > LGY ? (LGX > LGZ ? LGX : LGZ) : (LGY > LGZ ? LGY : LGZ);
};

// floor(x / y) and remainder for x < 2^32 and quotients below 2^15, from a
// hardware reciprocal estimate corrected in integers (exact).
__device__ __forceinline__ void divmod_rcp(uint32_t x, uint32_t y, float rcp, uint32_t& q, uint32_t& r) {
    uint32_t qq = (uint32_t)((float)x * rcp);
    int32_t rr = (int32_t)(x - qq * y);
    if (rr < 0) { --qq; rr += (int32_t)y; }
    if (rr < 0) { --qq; rr += (int32_t)y; }
    if (rr >= (int32_t)y) { ++qq; rr -= (int32_t)y; }
    if (rr >= (int32_t)y) { ++qq; rr -= (int32_t)y; }
    q = qq;
    r = (uint32_t)rr;
}

// Sets the bits of voxels k0 .. k0 + len - 1 (len <= kChunk; exactly kChunk
// when kFull) of one piece.
//
// The dominant axis moves by one voxel per step.  The two other axes keep
// their error terms as biased 16-bit halves u = r - 2N + 32768 of one
// register (r the remainder of eq. (3)'s division, so u in [32768-2N, 32768)):
// adding 2a sets bit 15 exactly when that coordinate advances, the carry
// bits then subtract 2N from their halves and add the axes' signed strides to
// the bit index with one packed dot product.  Needs 2N <= 32768.
template <bool kFull, int kChunk, int LGX, int LGY>
__device__ __forceinline__ void set_chunk(uint32_t* brick, const u32x4& rec, uint32_t k0, int len,
                                          const int32_t org[3]) {
    constexpr int32_t kSy = 1 << LGX, kSz = 1 << (LGX + LGY);
    // Record words: x0|y0<<16, z0|dx<<16, dy|dz<<16, klo|khi<<16.
    const int32_t p0[3] = {(int32_t)(rec.x & 0xFFFFu), (int32_t)(rec.x >> 16), (int32_t)(rec.y & 0xFFFFu)};
    const int32_t d[3] = {(int32_t)(int16_t)(rec.y >> 16), (int32_t)(int16_t)(rec.z & 0xFFFFu),
                          (int32_t)(int16_t)(rec.z >> 16)};
    const uint32_t a0 = (uint32_t)(d[0] < 0 ? -d[0] : d[0]);
    const uint32_t a1_ = (uint32_t)(d[1] < 0 ? -d[1] : d[1]);
    const uint32_t a2_ = (uint32_t)(d[2] < 0 ? -d[2] : d[2]);
    const uint32_t N = a0 > a1_ ? (a0 > a2_ ? a0 : a2_) : (a1_ > a2_ ? a1_ : a2_);
    // Dominant axis m (first of the maximal ones) and the two minor axes,
    // chosen with selects only.
    const bool m0 = a0 == N, m1 = !m0 && a1_ == N;
    const bool m2 = !m0 && !m1;
    const int32_t st0 = d[0] < 0 ? -1 : 1, st1 = d[1] < 0 ? -kSy : kSy, st2 = d[2] < 0 ? -kSz : kSz;
    const int32_t sm = m0 ? st0 : (m1 ? st1 : st2);
    // Minor axis 1: the lower-numbered of the two; minor axis 2: the other.
    const uint32_t aa = m0 ? a1_ : a0, ab = m2 ? a1_ : a2_;
    const int32_t sa = m0 ? st1 : st0, sb = m2 ? st1 : st2;
    const int32_t pa = m0 ? p0[1] : p0[0], pb = m2 ? p0[1] : p0[2];
    const int32_t oa = m0 ? org[1] : org[0], ob = m2 ? org[1] : org[2];
    const int32_t pm = m0 ? p0[0] : (m1 ? p0[1] : p0[2]);
    const int32_t om = m0 ? org[0] : (m1 ? org[1] : org[2]);
    const uint32_t nega = (uint32_t)(sa < 0), negb = (uint32_t)(sb < 0);
    const uint32_t two_n = 2u * N;
    uint32_t qa = 0, ra = 0, qb = 0, rb = 0;
    if (N > 0) {
        const float rcp = __builtin_amdgcn_rcpf((float)two_n);
        divmod_rcp(2u * k0 * aa + N - nega, two_n, rcp, qa, ra);
        divmod_rcp(2u * k0 * ab + N - negb, two_n, rcp, qb, rb);
    }
    // Bit index of voxel k0 inside the brick; each stride's sign is the
    // direction of its axis.
    const int32_t sgn_m = sm < 0 ? -1 : 1;
    int32_t idx = (pm + sgn_m * (int32_t)k0 - om) * (sm < 0 ? -sm : sm) +
                  (pa + (nega ? -(int32_t)qa : (int32_t)qa) - oa) * (sa < 0 ? -sa : sa) +
                  (pb + (negb ? -(int32_t)qb : (int32_t)qb) - ob) * (sb < 0 ? -sb : sb);
    u16x2 E = {(uint16_t)(ra + 32768u - two_n), (uint16_t)(rb + 32768u - two_n)};
    const u16x2 T = {(uint16_t)(2u * aa), (uint16_t)(2u * ab)};
    const u16x2 M = {(uint16_t)(0u - two_n), (uint16_t)(0u - two_n)};
    const i16x2 S = {(int16_t)sa, (int16_t)sb};
    const u16x2 k15 = {15, 15};
    if constexpr (kFull) {
#pragma unroll 8
        for (int k = 0; k < kChunk; ++k) {
            atomicOr(&brick[(uint32_t)idx >> 5], 1u << ((uint32_t)idx & 31u));
            E = E + T;
            const u16x2 C = E >> k15;
            E = E + C * M;
            idx = __builtin_amdgcn_sdot2(__builtin_bit_cast(i16x2, C), S, idx, false) + sm;
        }
    } else {
        for (int k = 0; k < len; ++k) {
            atomicOr(&brick[(uint32_t)idx >> 5], 1u << ((uint32_t)idx & 31u));
            E = E + T;
            const u16x2 C = E >> k15;
            E = E + C * M;
            idx = __builtin_amdgcn_sdot2(__builtin_bit_cast(i16x2, C), S, idx, false) + sm;
        }
    }
}

// Launch shape of the fill kernel per brick shape: threads, pieces per batch,
// voxels per chunk, chunk-table capacity.  One workgroup per CU; a batch
// holds (nearly) a whole brick so every wave gets many chunks between
// barriers and the longest chunk is short next to a wave's share.
template <int LGX, int LGY, int LGZ>
struct FillCfg {
    static constexpr int kBlock = 1024;
    static constexpr int kBatch = (LGX + LGY + LGZ) >= 20 ? 1024 : 2048;
    static constexpr int kChunk = 32;
    static constexpr int kCtab = 3 * kBatch;
};

template <int LGX, int LGY, int LGZ, bool kVec>
__global__ __launch_bounds__((FillCfg<LGX, LGY, LGZ>::kBlock))
void k_brick_fill(BrickGeom bg, const Piece* __restrict__ recs, const uint32_t* __restrict__ bin_base,
                  uint32_t* __restrict__ grid, uint32_t clear, uint32_t* __restrict__ work_counter) {
    using Shape = BrickShape<LGX, LGY, LGZ>;
    using Cfg = FillCfg<LGX, LGY, LGZ>;
    constexpr int kBlock = Cfg::kBlock, kBatch = Cfg::kBatch, kChunk = Cfg::kChunk, kCtab = Cfg::kCtab;
    constexpr int kPpt = kBatch / kBlock;                           // pieces per thread and batch
    constexpr int kMaxChunks = ((1 << Shape::kMaxLg) + kChunk - 1) / kChunk;  // per piece
    static_assert(kBatch % kBlock == 0, "whole pieces per thread");
    static_assert(kBatch * kMaxChunks <= 65536, "chunk table entries are 16-bit");
    static_assert(kChunk <= kWave, "chunk-length buckets are scanned by one wave");
    static_assert(kMaxChunks <= kCtab, "a batch always takes its first piece");
    // The brick first, so its addresses need no base offset.
    __shared__ __align__(16) uint32_t brick[Shape::kWords];
    __shared__ u32x4 pieces[kBatch];
    __shared__ uint16_t ctab[kCtab];
    // Chunks per length bucket (bucket 0: full chunks; bucket l: partial
    // chunks of kChunk - l voxels), then bucket offsets; two sets used by
    // alternate batches so clearing one needs no extra barrier.
    __shared__ uint32_t lenc[2][kChunk];
    __shared__ uint32_t red[kBlock / kWave];
    __shared__ uint32_t tot_s, round_s, cut_s;
    __shared__ uint32_t next_s[3];

    const uint32_t NB = bg.nbricks;
    const int64_t row_words = (int64_t)bg.dim[0] >> 5;
    const uint32_t lane = __lane_id();
    const u32x4* recv = reinterpret_cast<const u32x4*>(recs);
    if (threadIdx.x < kChunk) lenc[0][threadIdx.x] = lenc[1][threadIdx.x] = 0;
    uint32_t set = 0;

    // Bricks are taken from a global counter (work stealing: bricks differ
    // a lot in work).  The next brick and its bin range are claimed by
    // thread 0 at the start of the current one, so their memory latency
    // overlaps this brick's work, and the next brick's first records are
    // loaded before this brick is flushed.
    if (threadIdx.x == 0) {
        const uint32_t nb = atomicAdd(work_counter, 1u);
        next_s[0] = nb;
        next_s[1] = nb < NB ? bin_base[nb] : 0u;
        next_s[2] = nb < NB ? bin_base[nb + 1] : 0u;
    }
    lds_barrier();
    uint32_t b = next_s[0];
    uint32_t p_lo = next_s[1], p_hi = next_s[2];
    // Records of this thread's pieces in the next batch (consecutive), kept
    // as raw 16-byte vectors.
    u32x4 rec_n[kPpt];
#pragma unroll
    for (int j = 0; j < kPpt; ++j) {
        const uint32_t pos = p_lo + threadIdx.x * kPpt + j;
        rec_n[j] = (b < NB && pos < p_hi) ? recv[pos] : (u32x4){0u, 0u, 0u, 0u};
    }

    while (b < NB) {
        uint32_t nb = 0, nlo = 0, nhi = 0;
        if (threadIdx.x == 0) {
            nb = atomicAdd(work_counter, 1u);
            if (nb < NB) {
                nlo = bin_base[nb];
                nhi = bin_base[nb + 1];
            }
        }
        const int bx = (int)(b % (uint32_t)bg.nb[0]);
        const int by = (int)((b / (uint32_t)bg.nb[0]) % (uint32_t)bg.nb[1]);
        const int bz = (int)(b / ((uint32_t)bg.nb[0] * (uint32_t)bg.nb[1]));
        const int32_t org[3] = {bx << LGX, by << LGY, bz << LGZ};
        int32_t ext[3];
        {
            const int lgs[3] = {LGX, LGY, LGZ};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int32_t e = bg.dim[ax] - org[ax];
                ext[ax] = e < (1 << lgs[ax]) ? e : (1 << lgs[ax]);
            }
        }
        {
            u32x4* b4 = reinterpret_cast<u32x4*>(brick);
            for (uint32_t w = threadIdx.x; w < Shape::kWords / 4; w += kBlock) b4[w] = (u32x4){0, 0, 0, 0};
        }

        uint32_t p0 = p_lo;
        while (p0 < p_hi) {
            uint32_t* cnt = lenc[set];
            const uint32_t nbatch = p_hi - p0 < (uint32_t)kBatch ? p_hi - p0 : (uint32_t)kBatch;
            // Chunks of this thread's pieces.
            u32x4 rec[kPpt];
            uint32_t nch[kPpt], mysum = 0;
#pragma unroll
            for (int j = 0; j < kPpt; ++j) {
                rec[j] = rec_n[j];
                const uint32_t pos = threadIdx.x * kPpt + j;
                nch[j] = 0;
                if (pos < nbatch) {
                    const uint32_t len = (rec[j].w >> 16) - (rec[j].w & 0xFFFFu) + 1u;
                    nch[j] = (len + kChunk - 1) / kChunk;
                }
                mysum += nch[j];
            }
            if (threadIdx.x == 0) cut_s = nbatch;
            uint32_t total;
            uint32_t run = block_exclusive_sum_lds<kBlock>(mysum, red, total);
            // Batch cut: the first piece whose chunks overflow the table.
            if (total > (uint32_t)kCtab) {
#pragma unroll
                for (int j = 0; j < kPpt; ++j) {
                    if (run <= (uint32_t)kCtab && run + nch[j] > (uint32_t)kCtab)
                        atomicMin(&cut_s, threadIdx.x * kPpt + j);
                    run += nch[j];
                }
            }
            lds_barrier();
            const uint32_t cut = cut_s;
            // Bucket counts of the pieces inside the cut.
            uint32_t rf[kPpt], rp[kPpt];
#pragma unroll
            for (int j = 0; j < kPpt; ++j) {
                const uint32_t pos = threadIdx.x * kPpt + j;
                rf[j] = rp[j] = 0;
                if (pos < cut) {
                    pieces[pos] = rec[j];
                    const uint32_t len = (rec[j].w >> 16) - (rec[j].w & 0xFFFFu) + 1u;
                    const uint32_t nfull = len / kChunk, part = len % kChunk;
                    if (nfull) rf[j] = atomicAdd(&cnt[0], nfull);
                    if (part) rp[j] = atomicAdd(&cnt[kChunk - part], 1u);
                }
            }
            lds_barrier();
            if (threadIdx.x < kWave) {  // bucket offsets, one bucket per lane
                const uint32_t c = threadIdx.x < kChunk ? cnt[threadIdx.x] : 0u;
                const uint32_t incl = wave_inclusive_sum(c);
                if (threadIdx.x < kChunk) cnt[threadIdx.x] = incl - c;
                if (threadIdx.x == kWave - 1) {
                    tot_s = incl;
                    round_s = 0;
                }
            }
            lds_barrier();
#pragma unroll
            for (int j = 0; j < kPpt; ++j) {
                const uint32_t pos = threadIdx.x * kPpt + j;
                if (pos < cut) {
                    const uint32_t len = (rec[j].w >> 16) - (rec[j].w & 0xFFFFu) + 1u;
                    const uint32_t nfull = len / kChunk, part = len % kChunk;
                    for (uint32_t c = 0; c < nfull; ++c)
                        ctab[cnt[0] + rf[j] + c] = (uint16_t)(pos * kMaxChunks + c);
                    if (part) ctab[cnt[kChunk - part] + rp[j]] = (uint16_t)(pos * kMaxChunks + nfull);
                }
            }
            if (threadIdx.x < kChunk) lenc[set ^ 1][threadIdx.x] = 0;
            const uint32_t tot = tot_s;
            const uint32_t full = cnt[1];  // chunks before the first partial bucket
            // Next batch's records, in flight during this batch's rounds.
            p0 += cut;
#pragma unroll
            for (int j = 0; j < kPpt; ++j) {
                const uint32_t pos = p0 + threadIdx.x * kPpt + j;
                rec_n[j] = pos < p_hi ? recv[pos] : (u32x4){0u, 0u, 0u, 0u};
            }
            lds_barrier();

            // Rounds of kWave chunks, longest first, taken by whichever wave
            // is free: every wave runs chunks of (nearly) one length.
            const uint32_t rounds = (tot + kWave - 1) / kWave;
            while (true) {
                uint32_t r = 0;
                if (lane == 0) r = atomicAdd(&round_s, 1u);
                r = __builtin_amdgcn_readfirstlane(r);
                if (r >= rounds) break;
                const uint32_t c = r * kWave + lane;
                if (c >= tot) continue;
                const uint32_t e = ctab[c];
                const u32x4 q = pieces[e / kMaxChunks];
                const uint32_t k0 = (q.w & 0xFFFFu) + (e % kMaxChunks) * kChunk;
                if (c < full) {
                    set_chunk<true, kChunk, LGX, LGY>(brick, q, k0, kChunk, org);
                } else {
                    set_chunk<false, kChunk, LGX, LGY>(brick, q, k0, (int)((q.w >> 16) - k0 + 1u), org);
                }
            }
            set ^= 1;
            lds_barrier();
        }

        // Hand over the next brick; its first records load during the flush.
        if (threadIdx.x == 0) {
            next_s[0] = nb;
            next_s[1] = nlo;
            next_s[2] = nhi;
        }
        lds_barrier();
        b = next_s[0];
        p_lo = next_s[1];
        p_hi = next_s[2];
#pragma unroll
        for (int j = 0; j < kPpt; ++j) {
            const uint32_t pos = p_lo + threadIdx.x * kPpt + j;
            rec_n[j] = (b < NB && pos < p_hi) ? recv[pos] : (u32x4){0u, 0u, 0u, 0u};
        }

        // Flush: brick rows -> volume words.  The owner writes every word of
        // its brick, so a clearing call needs no other pass.
        const int rows = ext[1] * ext[2];
        if constexpr (kVec) {
            // 16-byte units, Shape::kBXw / 4 per row, rows full width.
            constexpr int kUpr = Shape::kBXw / 4;
            const int units = rows * kUpr;
            for (int t = threadIdx.x; t < units; t += kBlock) {
                const int part = t % kUpr, r = t / kUpr;
                const int y = r % ext[1], z = r / ext[1];
                const u32x4 v = *reinterpret_cast<const u32x4*>(
                    &brick[(((uint32_t)z << LGY) | (uint32_t)y) * (uint32_t)Shape::kBXw + 4u * part]);
                u32x4* dst = reinterpret_cast<u32x4*>(
                    grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words + (org[0] >> 5) +
                    4 * part);
                if (clear) {
                    __builtin_nontemporal_store(v, dst);
                } else {
                    *dst = *dst | v;
                }
            }
        } else {
            const int xws = ext[0] >> 5;
            const int total = rows * xws;
            for (int t = threadIdx.x; t < total; t += kBlock) {
                const int xw = t % xws, r = t / xws;
                const int y = r % ext[1], z = r / ext[1];
                const uint32_t v = brick[(((uint32_t)z << LGY) | (uint32_t)y) * (uint32_t)Shape::kBXw + xw];
                uint32_t* dst = grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words +
                                (org[0] >> 5) + xw;
                if (clear) *dst = v;
                else *dst |= v;
            }
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------- host side


// Brick shapes with a compiled fill kernel.
static const int kShapes[][3] = {{8, 6, 5}, {8, 6, 6}, {7, 6, 6}, {7, 7, 6}};

bool brick_shape_supported(const int lg[3]) {
    for (const auto& sh : kShapes)
        if (sh[0] == lg[0] && sh[1] == lg[1] && sh[2] == lg[2]) return true;
    return false;
}

void default_brick_lg(int32_t dx, int32_t dy, int32_t dz, int lg[3]) {
    (void)dx; (void)dy; (void)dz;
    lg[0] = 8;  // 256: 32-byte brick rows
    lg[1] = 6;  // 64
    lg[2] = 5;  // 32
}

uint64_t max_pieces(int64_t n, const BrickGeom& bg) {
    return (uint64_t)n * (uint64_t)(1 + (bg.nb[0] - 1) + (bg.nb[1] - 1) + (bg.nb[2] - 1));
}

int hist_blocks(int64_t n) {
    int64_t g = (n + 4095) / 4096;
    if (g > kHistRows) g = kHistRows;
    if (g < 1) g = 1;
    return (int)g;
}

size_t brick_workspace_bytes(int64_t n, const BrickGeom& bg) {
    const int G = hist_blocks(n);
    size_t b = kAlign;                                                  // status, counter
    b += align_up((size_t)G * bg.nbricks * sizeof(uint32_t));          // hist rows
    b += align_up((size_t)bg.nbricks * sizeof(uint32_t));              // totals
    b += align_up((size_t)(bg.nbricks + 1) * sizeof(uint32_t));        // bin base
    b += align_up((size_t)max_pieces(n, bg) * sizeof(Piece));          // piece records
    return b;
}

template <int LGX, int LGY, int LGZ>
static hipError_t launch_fill(const BrickGeom& bg, const Piece* recs, const uint32_t* bin_base, uint32_t* grid,
                              uint32_t clear, uint32_t* counter, hipStream_t stream) {
    using Shape = BrickShape<LGX, LGY, LGZ>;
    constexpr int kBlock = FillCfg<LGX, LGY, LGZ>::kBlock;
    const bool vec = (bg.dim[0] % (1 << LGX)) == 0 && Shape::kBXw % 4 == 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    int wgs = cus;
    if ((uint32_t)wgs > bg.nbricks) wgs = (int)bg.nbricks;
    if (vec)
        k_brick_fill<LGX, LGY, LGZ, true><<<wgs, kBlock, 0, stream>>>(bg, recs, bin_base, grid, clear, counter);
    else
        k_brick_fill<LGX, LGY, LGZ, false><<<wgs, kBlock, 0, stream>>>(bg, recs, bin_base, grid, clear, counter);
    return hipGetLastError();
}

hipError_t launch_brick_grid(const int32_t* segs, int64_t n, bool aligned8, const BrickGeom& bg,
                             uint32_t* grid, int32_t* counts, uint32_t flags, void* d_work,
                             hipStream_t stream) {
    const int G = hist_blocks(n);
    uint8_t* p = static_cast<uint8_t*>(d_work);
    int32_t* status = reinterpret_cast<int32_t*>(p);
    uint32_t* counter = reinterpret_cast<uint32_t*>(p + 4);
    p += kAlign;
    uint32_t* hist = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)G * bg.nbricks * sizeof(uint32_t));
    uint32_t* totals = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)bg.nbricks * sizeof(uint32_t));
    uint32_t* bin_base = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)(bg.nbricks + 1) * sizeof(uint32_t));
    Piece* recs = reinterpret_cast<Piece*>(p);
    const size_t hist_lds = (size_t)bg.nbricks * sizeof(uint32_t);
    hipError_t e;
    {
        KernelTimer t("brick_init", stream);
        k_brick_init<<<1, 64, 0, stream>>>(status, counter);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        // Dynamic LDS (the brick histogram) beyond the default limit.
        const void* ks[4] = {(const void*)k_brick_hist<true>, (const void*)k_brick_hist<false>,
                             (const void*)k_brick_scatter<true>, (const void*)k_brick_scatter<false>};
        for (const void* k : ks)
            if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hist_lds)) !=
                hipSuccess)
                return e;
    }
    {
        KernelTimer t("brick_hist", stream);
        if (aligned8)
            k_brick_hist<true><<<G, kHistBlock, hist_lds, stream>>>(segs, n, bg, hist, counts, status);
        else
            k_brick_hist<false><<<G, kHistBlock, hist_lds, stream>>>(segs, n, bg, hist, counts, status);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        KernelTimer t("brick_colscan", stream);
        k_brick_colscan<<<(bg.nbricks + kColBins - 1) / kColBins, 256, 0, stream>>>(hist, G, bg.nbricks,
                                                                                    totals);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        KernelTimer t("brick_base", stream);
        k_brick_base<<<1, kBaseBlock, 0, stream>>>(totals, bg.nbricks, bin_base);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        KernelTimer t("brick_scatter", stream);
        if (aligned8)
            k_brick_scatter<true><<<G, kHistBlock, hist_lds, stream>>>(segs, n, bg, hist, bin_base, recs);
        else
            k_brick_scatter<false><<<G, kHistBlock, hist_lds, stream>>>(segs, n, bg, hist, bin_base, recs);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;

    const uint32_t clear = (flags & 1u) ? 1u : 0u;
    KernelTimer t("brick_fill", stream);
    const int* lg = bg.lg;
    if (lg[0] == 8 && lg[1] == 6 && lg[2] == 5)
        return launch_fill<8, 6, 5>(bg, recs, bin_base, grid, clear, counter, stream);
    if (lg[0] == 8 && lg[1] == 6 && lg[2] == 6)
        return launch_fill<8, 6, 6>(bg, recs, bin_base, grid, clear, counter, stream);
    if (lg[0] == 7 && lg[1] == 6 && lg[2] == 6)
        return launch_fill<7, 6, 6>(bg, recs, bin_base, grid, clear, counter, stream);
    if (lg[0] == 7 && lg[1] == 7 && lg[2] == 6)
        return launch_fill<7, 7, 6>(bg, recs, bin_base, grid, clear, counter, stream);
    return hipErrorInvalidValue;
}

}  // namespace vox

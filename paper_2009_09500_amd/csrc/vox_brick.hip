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
// Every kernel reads its volumes from a scene table (BrickTable followed by
// BrickScene entries) that the plan kernel writes into the workspace from
// the caller's vox_scene entries: a plain call is a table of one scene, a
// batch a table of many, whose bricks and histogram rows are numbered
// globally so that each kernel below is still one launch for the whole batch.
//
// Pipeline (one stream, no host synchronisation, no allocation):
//   plan      checks every scene, decides brick or direct kernels per scene,
//             numbers rows and bricks (block scans), writes the table, the
//             status word and the fill's work queues
//   expand    scene of each histogram row and brick (several scenes only)
//   hist      per segment: count N+1, range check, walk its bricks and count
//             pieces per brick in an LDS histogram; one histogram row per
//             workgroup
//   colscan   per brick, exclusive prefix of the rows over workgroups, and
//             the brick's piece total
//   base      exclusive scan of the brick totals -> bin offsets; if the
//             records do not fit the workspace, the direct kernels take over;
//             the fill's work items: one per brick, several for a brick with
//             more than a fair share of the records
//   clear     (batches) zeroes the volumes of the cleared direct scenes
//   scatter   zeroes the bricks cut into several items in cleared volumes,
//             then the same walk again, writing one 16-byte piece record
//             (start point, direction, k-window in the brick) into the
//             brick's bin
//   fill      persistent workgroups take work items from work-stealing
//             queues, set the bits of every piece with LDS atomic OR and
//             flush the brick to the volume (an item that holds part of a
//             brick with device atomic OR)
//   direct    (batches) one device atomic per voxel, for the scenes the
//             bricks do not serve
#include "vox.h"
#include "vox_device.h"
#include "vox_direct.h"
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
// Global-memory views: volume pointers come from the scene table, so the
// compiler cannot infer their address space; without these casts it emits
// flat stores, which also count against the LDS wait counter.
typedef __attribute__((address_space(1))) u32x4 global_u32x4;
typedef __attribute__((address_space(1))) uint32_t global_u32;

typedef int16_t i16x2 __attribute__((ext_vector_type(2)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ kernels

__host__ __device__ constexpr uint64_t up256(uint64_t v) { return (v + 255u) & ~uint64_t(255); }

// Piece record (16 bytes): the stepping state of a piece at its first voxel
// (k = klo), made by the scatter, which has the segment at hand, so that the
// fill only unpacks it and never gathers segments.  Minor axes a < b in axis
// order, m the dominant axis (the first of the longest ones):
//   e  the minor axes' error terms as biased 16-bit halves u = r - 2N + 32768
//      (r the remainder of eq. (3)'s division at k = klo)
//   t  their increments, 2a | 2b << 16
//   v  m | nega << 2 | negb << 3 | negm << 4 | 2N << 16 (2N = 2 when N = 0)
//   w  the bit index of the voxel at klo inside the brick
//      | (voxels - 1) << (log2 of the brick's voxel count)
struct Piece {
    uint32_t e, t, v, w;
};
static_assert(sizeof(Piece) == 16, "16-byte piece records");

// Sections of the workspace: the header words, the table the plan kernel
// writes at kWorkTable, then at the table's data_off the histograms, the
// brick totals, the bin offsets, the fill's work items and the piece records
// (the rest of the workspace).
//
// Bytes from the table's data_off to the piece records.
__host__ __device__ inline uint64_t brick_data_bytes(uint64_t hist_words, uint64_t bricks) {
    return up256(hist_words * 4u) + up256(bricks * 4u) + 2u * up256((bricks + 1u) * 4u) +
           up256((bricks + kMaxExtraItems) * 4u) + up256((uint64_t)kMaxExtraItems * 4u);
}

struct WorkView {
    int32_t* status;
    uint32_t* counter;   // [kXcds] work queues of the fill, one per XCD
    uint32_t* ok;
    uint32_t* direct_all;
    uint64_t* pieces;
    uint32_t* hist;
    uint32_t* totals;
    uint32_t* bin_base;
    uint32_t* n_items;     // fill work items (header word)
    uint32_t* n_split;     // bricks cut into several items (header word)
    uint32_t* item_base;   // [bricks + 1] first work item of each brick
    uint32_t* item_brick;  // [bricks + kMaxExtraItems] brick of each work item
    uint32_t* split;       // [kMaxExtraItems] the bricks cut into several items
    Piece* recs;
    uint64_t rec_off;    // byte offset of the records
};

__host__ __device__ inline WorkView work_view(uint8_t* work, uint64_t data_off, uint64_t hist_words,
                                              uint32_t bricks) {
    WorkView v;
    uint32_t* w = reinterpret_cast<uint32_t*>(work);
    v.status = reinterpret_cast<int32_t*>(work) + kWStatus;
    v.counter = w + kWQueues;
    v.ok = w + kWOk;
    v.direct_all = w + kWDirectAll;
    v.pieces = reinterpret_cast<uint64_t*>(w + kWPieces);
    v.n_items = w + kWItems;
    v.n_split = w + kWSplit;
    uint64_t off = data_off;
    v.hist = reinterpret_cast<uint32_t*>(work + off);
    off += up256(hist_words * 4u);
    v.totals = reinterpret_cast<uint32_t*>(work + off);
    off += up256((uint64_t)bricks * 4u);
    v.bin_base = reinterpret_cast<uint32_t*>(work + off);
    off += up256(((uint64_t)bricks + 1u) * 4u);
    v.item_base = reinterpret_cast<uint32_t*>(work + off);
    off += up256(((uint64_t)bricks + 1u) * 4u);
    v.item_brick = reinterpret_cast<uint32_t*>(work + off);
    off += up256(((uint64_t)bricks + kMaxExtraItems) * 4u);
    v.split = reinterpret_cast<uint32_t*>(work + off);
    off += up256((uint64_t)kMaxExtraItems * 4u);
    v.recs = reinterpret_cast<Piece*>(work + off);
    v.rec_off = off;
    return v;
}

// The scene table as the kernels see it.
struct TableView {
    BrickTable h;
    const BrickScene* scenes;
    const uint32_t* direct;       // the direct scenes, in order
    const uint32_t* row_scene;    // null with one scene
    const uint32_t* brick_scene;  // null with one scene
};

__host__ __device__ __forceinline__ TableView table_view(const uint8_t* table) {
    TableView v;
    v.h = *reinterpret_cast<const BrickTable*>(table);
    v.scenes = reinterpret_cast<const BrickScene*>(table + kTableScenes);
    v.direct = reinterpret_cast<const uint32_t*>(v.scenes + v.h.n_scenes);
    if (v.h.n_scenes > 1) {
        v.row_scene = v.direct + v.h.n_scenes;
        v.brick_scene = v.row_scene + v.h.row_cap;
    } else {
        v.row_scene = v.brick_scene = nullptr;
    }
    return v;
}

__device__ __forceinline__ WorkView work_of(uint8_t* work, const TableView& tv) {
    return work_view(work, tv.h.data_off, tv.h.hist_words, tv.h.bricks);
}

// Work queues of the fill (over its work items: one per brick, more for a
// brick cut into several).  The 8 XCDs of the chip each have their own L2;
// workgroup w runs on XCD w % 8.  Groups of 8 consecutive items (bricks
// along x, the fastest brick axis) are dealt to the XCDs in turn, so
// neighbouring bricks, whose 32-byte row pieces share memory lines, are
// flushed through the same L2 at about the same time and reach HBM as whole
// lines.  A workgroup takes from its own XCD's queue first and then from
// the others.
constexpr int kXcds = 8;

// Item of the c-th claim on queue x.
__device__ __forceinline__ uint32_t queue_brick(uint32_t x, uint32_t c) {
    return (c >> 3) * (8u * kXcds) + x * 8u + (c & 7u);
}

// A device-scope atomic costs a full memory round trip, so once its own queue
// is empty a workgroup reads all the other counters at once (one round trip)
// and claims only from queues that still hold bricks, rather than trying
// each in turn; it stops when every queue is empty (counters only grow, so
// every pass either claims or finds fewer queues open).
__device__ __forceinline__ uint32_t claim_brick(uint32_t* queues, uint32_t xcd, uint32_t NB) {
    uint32_t g = queue_brick(xcd, atomicAdd(&queues[xcd], 1u));
    if (g < NB) return g;
    for (;;) {
        uint32_t c[kXcds];
#pragma unroll
        for (int x = 0; x < kXcds; ++x) c[x] = __hip_atomic_load(&queues[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool open = false;
#pragma unroll
        for (uint32_t x = 0; x < (uint32_t)kXcds; ++x) {
            if (x == xcd || queue_brick(x, c[x]) >= NB) continue;
            open = true;
            g = queue_brick(x, atomicAdd(&queues[x], 1u));
            if (g < NB) return g;
        }
        if (!open) return NB;
    }
}

// The next work item of a workgroup (claimed by one thread): its brick (NB
// when none is left), its part [lo, hi) of the brick's records and whether
// the brick is cut into several items.
struct ItemClaim {
    uint32_t brick, lo, hi, split;
};
__device__ __forceinline__ ItemClaim claim_item(const WorkView& wv, uint32_t xcd, uint32_t n_items, uint32_t n_split,
                                                uint32_t NB) {
    ItemClaim c = {NB, 0u, 0u, 0u};
    const uint32_t i = claim_brick(wv.counter, xcd, n_items);
    if (i >= n_items) return c;
    if (n_split == 0u) {  // the items are the bricks
        c.brick = i;
        c.lo = wv.bin_base[i];
        c.hi = wv.bin_base[i + 1];
        return c;
    }
    const uint32_t b = wv.item_brick[i];
    const uint32_t i0 = wv.item_base[b], k = wv.item_base[b + 1] - i0, j = i - i0;
    const uint32_t lo = wv.bin_base[b];
    c.brick = b;
    item_range(lo, wv.bin_base[b + 1] - lo, j, k, c.lo, c.hi);
    c.split = k > 1u ? 1u : 0u;
    return c;
}

// Histogram row of workgroup w out of G.  Each XCD takes a contiguous block
// of rows (workgroup w runs on XCD w % 8): a bin holds the records of row 0,
// then row 1, ..., so the scatter's short per-row runs of one bin that share
// memory lines are written through one L2 at about the same time.
__device__ __forceinline__ uint32_t xcd_row(uint32_t w, uint32_t G) {
    const uint32_t x = w % kXcds, a = w / kXcds;
    uint32_t start = 0;
    for (uint32_t i = 0; i < x; ++i) start += (G - i + kXcds - 1) / kXcds;  // rows of XCD i
    return start + a;
}

constexpr int kPlanBlock = 1024;

// The table header, status word, flags and work queues of a launch whose
// scenes have been numbered (one lane).
__device__ __forceinline__ void write_table(uint8_t* work, const BrickLaunch& L, uint64_t work_bytes, uint32_t rows_c,
                                            uint32_t bricks_c, uint32_t direct_c, uint32_t max_nb, uint64_t hist_c,
                                            uint64_t segs_c, uint64_t dsegs_c, bool bad) {
    uint8_t* tb = work + kWorkTable;
    BrickTable t{};
    t.magic = kTableMagic;
    t.n_scenes = L.n_scenes;
    t.rows = rows_c;
    t.bricks = bricks_c;
    for (int a = 0; a < 3; ++a) t.lg[a] = L.lg[a];
    t.max_nb = max_nb;
    t.hist_words = hist_c;
    t.data_off = kWorkTable + L.table_bytes;
    t.n_direct = direct_c;
    t.row_cap = L.rows;
    t.direct_segs = dsegs_c;
    *reinterpret_cast<BrickTable*>(tb) = t;
    const bool fits = segs_c <= L.total_segments && rows_c <= L.rows && bricks_c <= L.bricks;
    const WorkView wv = work_view(work, t.data_off, t.hist_words, t.bricks);
    const bool room = wv.rec_off <= work_bytes;
    uint32_t* w = reinterpret_cast<uint32_t*>(work);
    const int32_t st = bad ? kStatusInvalid : (fits ? 0 : kStatusLaunch);
    w[kWStatus] = (uint32_t)st;
    w[kWOk] = (st == 0 && room && bricks_c > 0) ? 1u : 0u;
    w[kWDirectAll] = room ? 0u : 1u;
    for (int x = 0; x < kXcds; ++x) w[kWQueues + x] = 0u;
    *wv.pieces = 0;
}

// The plan of a batch: one block reads the caller's scenes (the device
// vox_scene array), checks each against the argument rules, decides which
// scenes the brick kernels serve (8-byte-aligned segment arrays, volumes the
// bricks cover; with the Euclidean N, a diagonal below 16385) and which the
// direct kernels serve, numbers the histogram rows and bricks of all brick
// scenes (block scans), and writes the table, the status word, the brick
// queues and the flags.  A scene that breaks a rule, or scenes beyond the
// launch bounds, stop the whole call (nothing is written).  When the
// histograms and brick offsets do not fit the workspace, the direct kernels
// serve every scene.
__global__ __launch_bounds__(kPlanBlock) void k_brick_plan(const vox_scene* __restrict__ scenes, BrickLaunch L,
                                                           uint8_t* __restrict__ work, uint64_t work_bytes) {
    __shared__ uint32_t scan32[kPlanBlock / kWave];
    __shared__ uint64_t scan64[kPlanBlock / kWave];
    __shared__ uint32_t bad_s, max_nb_s;
    uint8_t* tb = work + kWorkTable;
    BrickScene* out = reinterpret_cast<BrickScene*>(tb + kTableScenes);
    uint32_t* direct = reinterpret_cast<uint32_t*>(out + L.n_scenes);
    if (threadIdx.x == 0) {
        bad_s = 0;
        max_nb_s = 0;
    }
    __syncthreads();
    uint32_t rows_c = 0, bricks_c = 0, direct_c = 0;
    uint64_t hist_c = 0, segs_c = 0, dsegs_c = 0;
    for (uint32_t c0 = 0; c0 < L.n_scenes; c0 += kPlanBlock) {
        const uint32_t i = c0 + threadIdx.x;
        BrickScene b{};
        uint32_t rows = 0, nb = 0, isd = 0;
        uint64_t hist = 0, n = 0;
        if (i < L.n_scenes) {
            const vox_scene in = scenes[i];
            if (!plan_scene(in, L.lg, L.segs_per_row, b)) atomicOr(&bad_s, 1u);
            isd = (b.flags & kSceneDirect) ? 1u : 0u;
            rows = b.rows;
            nb = isd ? 0u : b.bg.nbricks;
            hist = (uint64_t)rows * nb;
            n = b.n > 0 ? (uint64_t)b.n : 0u;
            atomicMax(&max_nb_s, nb);
        }
        uint32_t t_rows, t_nb, t_d;
        uint64_t t_hist, t_n, t_dn;
        const uint32_t x_rows = block_exclusive_sum<kPlanBlock>(rows, scan32, t_rows);
        const uint32_t x_nb = block_exclusive_sum<kPlanBlock>(nb, scan32, t_nb);
        const uint32_t x_d = block_exclusive_sum<kPlanBlock>(isd, scan32, t_d);
        const uint64_t x_hist = block_exclusive_sum<kPlanBlock>(hist, scan64, t_hist);
        (void)block_exclusive_sum<kPlanBlock>(n, scan64, t_n);
        (void)block_exclusive_sum<kPlanBlock>(isd ? n : 0u, scan64, t_dn);
        if (i < L.n_scenes) {
            b.row_base = rows_c + x_rows;
            b.brick_base = bricks_c + x_nb;
            b.hist_off = hist_c + x_hist;
            out[i] = b;
            if (isd) direct[direct_c + x_d] = i;
        }
        rows_c += t_rows;
        bricks_c += t_nb;
        direct_c += t_d;
        hist_c += t_hist;
        segs_c += t_n;
        dsegs_c += t_dn;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    write_table(work, L, work_bytes, rows_c, bricks_c, direct_c, max_nb_s, hist_c, segs_c, dsegs_c, bad_s != 0);
}

// Scene of every histogram row and of every brick (tables of several
// scenes); workgroups take scenes in turn.
__global__ __launch_bounds__(256) void k_brick_expand(uint8_t* __restrict__ work) {
    const uint8_t* tb = work + kWorkTable;
    const TableView tv = table_view(tb);
    if (reinterpret_cast<const uint32_t*>(work)[kWOk] == 0 || tv.row_scene == nullptr) return;
    uint32_t* row_scene = const_cast<uint32_t*>(tv.row_scene);
    uint32_t* brick_scene = const_cast<uint32_t*>(tv.brick_scene);
    for (uint32_t s = blockIdx.x; s < tv.h.n_scenes; s += gridDim.x) {
        const BrickScene& sc = tv.scenes[s];
        if (sc.flags & kSceneDirect) continue;
        for (uint32_t r = threadIdx.x; r < sc.rows; r += blockDim.x) row_scene[sc.row_base + r] = s;
        for (uint32_t b = threadIdx.x; b < sc.bg.nbricks; b += blockDim.x) brick_scene[sc.brick_base + b] = s;
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
constexpr int kStageBig = 8192;   // ... by the histogram when its counters leave room
constexpr uint32_t kBigStageBricks = 8192;  // bricks per scene up to which they do
constexpr int kOrderBins = 64;

// Staged segments ordered by their estimated number of pieces (walk_estimate),
// longest walks first, so the lanes of a wave walk segments of (nearly)
// equal piece counts: they all start together and finish together.  Bucket
// kOrderBins - est, the longest (est >= kOrderBins) in bucket 0.  The buckets
// fall into the classes of walk_parts: 8 parts (bucket 0), 4 (buckets 1-32),
// 2 (33-48) and 1 (49-63), so each class is a contiguous run of the order.
template <int kN>
struct Stage {
    StagedSeg seg[kN];
    uint16_t order[kN];
    uint32_t bins[kOrderBins];  // bucket sizes, then bucket starts, then bucket ends
    uint32_t nvalid;
    uint32_t claim;             // next group of the walk (walk_ordered)
};
static_assert(kOrderBins == 64 && kMaxWalkParts == 8, "walk classes: buckets 0, 1-32, 33-48, 49-63");
constexpr int kBinEnd8 = 0, kBinEnd4 = 32, kBinEnd2 = 48;  // last bucket of each class

__device__ __forceinline__ uint32_t order_bin(const StagedSeg& g, const BrickGeom& bg) {
    const int32_t p0[3] = {g.p0[0], g.p0[1], g.p0[2]}, p1[3] = {g.p1[0], g.p1[1], g.p1[2]};
    const uint32_t est = walk_estimate(p0, p1, bg.lg);
    return (uint32_t)kOrderBins - (est < (uint32_t)kOrderBins ? est : (uint32_t)kOrderBins);
}

// Loads segments [base, base + cnt) into the stage (all threads of the
// block), writes counts, flags out-of-volume segments, and builds the order
// of the in-volume ones.
template <int kN>
__device__ __forceinline__ void stage_segments(const int32_t* __restrict__ segs, int64_t base, uint32_t cnt,
                                               const BrickGeom& bg, bool euclid, Stage<kN>& st,
                                               int32_t* __restrict__ counts, bool& bad) {
    if (threadIdx.x < kOrderBins) st.bins[threadIdx.x] = 0;
    lds_barrier();
    // Bit t of `mine` marks this thread's t-th segment as in the volume.
    uint32_t mine = 0;
    int slot = 0;
    for (uint32_t t = threadIdx.x; t < cnt; t += kHistBlock, ++slot) {
        const Seg g = load_seg<true>(segs, base + t);
        const bool inside = in_volume(g, bg);
        if (counts) {
            // Counts: N + 1 for the Chebyshev N; with the Euclidean N 0
            // outside the volume here, the voxels after duplicate removal
            // inside it from the histogram's count pass (euclid_counts).
            if (euclid) {
                if (!inside) counts[base + t] = 0;
            } else {
                const int64_t c = seg_length(g) + 1;
                counts[base + t] = (int32_t)(c > 0x7FFFFFFFll ? 0x7FFFFFFFll : c);
            }
        }
        StagedSeg s;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            s.p0[ax] = (uint16_t)g.p0[ax];
            s.p1[ax] = (uint16_t)g.p1[ax];
        }
        st.seg[t] = s;
        if (inside) {
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
        if (threadIdx.x == kWave - 1) {
            st.nvalid = incl;
            st.claim = 0;
        }
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
static_assert(kStage / kHistBlock <= 32 && kStageBig / kHistBlock <= 32 && kStageBig <= 65536,
              "one validity bit per staged segment and thread; 16-bit order entries");

struct WalkState {
    AxisCross c[3];
    uint32_t N, klo;  // length (Chebyshev or Euclidean), first k inside the current brick
    uint32_t kend;    // last k of the walk's part
};

// floor(sqrt(s)) for s < 2^31: the double square root is correctly rounded,
// so its integer part is exact in this range.
__device__ __forceinline__ uint32_t isqrt31(uint32_t s) { return (uint32_t)__dsqrt_rn((double)s); }

// Walk state at the start of part `part` of `parts` of a walk (the whole
// walk when parts = 1; false for an empty part).  Every coordinate of
// eq. (3) is monotone in k for any N >= max |d_a|, so the brick crossings
// follow the same rules under the Euclidean N of eq. (1)
// (N = floor |P1 - P0| >= max |d_a|).
__device__ __forceinline__ bool walk_init(WalkState& w, const StagedSeg& g, const BrickGeom& bg, bool euclid,
                                          uint32_t part, uint32_t parts) {
    int32_t p0[3], p1[3];
    uint32_t a[3], neg[3], N = 0, ss = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        p0[ax] = g.p0[ax];
        p1[ax] = g.p1[ax];
        const int32_t d = p1[ax] - p0[ax];
        neg[ax] = d < 0;
        a[ax] = (uint32_t)(d < 0 ? -d : d);
        N = a[ax] > N ? a[ax] : N;
        ss += a[ax] * a[ax];
    }
    if (euclid) N = isqrt31(ss);
    uint32_t k0 = 0, k1 = N;
    if (parts > 1u && !part_window(p0, p1, a, neg, N, bg.lg, part, parts, k0, k1)) return false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) cross_init_at(w.c[ax], p0[ax], p1[ax], a[ax], neg[ax], N, bg.lg[ax], k0);
    w.N = N;
    w.klo = k0;
    w.kend = k1;
    return true;
}

// Steps k0 + 1 ... k0 + len (k0 + len <= N) of an in-volume segment under
// the Euclidean N at which some axis moves.  With r_a(k) = (2k a + N - neg_a)
// mod 2N, the remainder of eq. (3)'s division, axis a moves at step k exactly
// when r_a(k - 1) + 2a reaches 2N (a <= N).  One division per axis gives
// r_a(k0); the steps then run on biased 16-bit halves as in the fill
// (N <= 16384 in a brick scene).
__device__ __forceinline__ uint32_t euclid_moves(const StagedSeg& g, uint32_t N, uint32_t k0, uint32_t len) {
    uint32_t a[3], neg[3], r[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int32_t d = (int32_t)g.p1[ax] - (int32_t)g.p0[ax];
        neg[ax] = d < 0;
        a[ax] = (uint32_t)(d < 0 ? -d : d);
    }
    const uint32_t two_n = 2u * N;
    const float rcpd = rcp_down(two_n);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t q;
        divmod_down(2u * __umul24(k0, a[ax]) + N - neg[ax], two_n, rcpd, q, r[ax]);
    }
    u16x2 E = {(uint16_t)(r[0] + 32768u - two_n), (uint16_t)(r[1] + 32768u - two_n)};
    u16x2 Ez = {(uint16_t)(r[2] + 32768u - two_n), 0};
    const u16x2 T = {(uint16_t)(2u * a[0]), (uint16_t)(2u * a[1])};
    const u16x2 Tz = {(uint16_t)(2u * a[2]), 0};
    const u16x2 N2 = {(uint16_t)two_n, (uint16_t)two_n};
    const i16x2 k15 = {15, 15};
    uint32_t moves = 0;
#pragma unroll 4
    for (uint32_t t = 0; t < len; ++t) {
        E = E + T;
        const i16x2 C = __builtin_bit_cast(i16x2, E) >> k15;  // -1 where the axis moves
        E = E + __builtin_bit_cast(u16x2, C) * N2;
        Ez = Ez + Tz;
        const i16x2 Cz = __builtin_bit_cast(i16x2, Ez) >> k15;
        Ez = Ez + __builtin_bit_cast(u16x2, Cz) * N2;
        moves += (__builtin_bit_cast(uint32_t, C) | __builtin_bit_cast(uint32_t, Cz)) != 0u ? 1u : 0u;
    }
    return moves;
}

// Per-wave LDS of the Euclidean counts, one entry per lane: its segment's
// first chunk number, length N and move count.
struct CountScratch {
    uint32_t pre[kWave], n[kWave], cnt[kWave];
};
constexpr size_t kCountScratch = (size_t)(kHistBlock / kWave) * sizeof(CountScratch);

// Voxels (after duplicate removal) of the staged in-volume segments under
// the Euclidean N: 1 + the steps at which some axis moves.  Each wave takes
// 32 segments in walk order (so that a row of 512 segments keeps all 16
// waves busy), one per lane of its first half, cuts them into chunks of 64
// steps (a prefix over the lanes numbers the chunks), and runs the chunks 64
// at a time, one per lane, each lane finding its chunk's segment by binary
// search over the prefix; a segment's moves are summed with LDS atomics.
// counts: the stage's first segment's slot.
constexpr uint32_t kCountGroup = 32;
template <int kN>
__device__ __forceinline__ void euclid_counts(const Stage<kN>& st, int32_t* __restrict__ counts,
                                              CountScratch* scratch) {
    const uint32_t lane = __lane_id();
    CountScratch& w = scratch[threadIdx.x / kWave];
    const uint32_t nvalid = st.nvalid;
    for (uint32_t g0 = (threadIdx.x / kWave) * kCountGroup; g0 < nvalid;
         g0 += (kHistBlock / kWave) * kCountGroup) {
        const uint32_t i = g0 + lane;
        const bool mine = lane < kCountGroup && i < nvalid;
        uint32_t j = 0, N = 0;
        if (mine) {
            j = st.order[i];
            const StagedSeg& g = st.seg[j];
            uint32_t ss = 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int32_t d = (int32_t)g.p1[ax] - (int32_t)g.p0[ax];
                ss += (uint32_t)(d * d);
            }
            N = isqrt31(ss);
        }
        const uint32_t ch = (N + kWave - 1) / kWave;
        const uint32_t incl = wave_inclusive_sum(ch);
        const uint32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
        w.pre[lane] = incl - ch;
        w.n[lane] = N;
        w.cnt[lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t q0 = 0; q0 < total; q0 += kWave) {
            const uint32_t q = q0 + lane;
            if (q < total) {
                // The last lane whose first chunk is at most q owns chunk q.
                uint32_t o = 0;
#pragma unroll
                for (uint32_t step = kWave / 2; step > 0; step >>= 1) o += w.pre[o + step] <= q ? step : 0u;
                const uint32_t n = w.n[o];
                const uint32_t k0 = (q - w.pre[o]) * (uint32_t)kWave;
                const uint32_t len = n - k0 < (uint32_t)kWave ? n - k0 : (uint32_t)kWave;
                atomicAdd(&w.cnt[o], euclid_moves(st.seg[st.order[g0 + o]], n, k0, len));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (mine) counts[j] = (int32_t)(1u + w.cnt[lane]);
        // The scratch is rewritten by the wave's next 64 segments.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Walks the ordered staged segments.  With kSplit the order falls into four
// classes of walk_parts (8, 4, 2 and 1 parts, longest walks first), and the
// walk into groups of 64 part walks: 8 segments of the first class cut into
// 8 parts each, 16 of the second cut into 4, and so on; without, into groups
// of 64 whole walks.  Waves claim groups in order from an LDS counter, so the
// longest groups start first and a wave that finishes early takes the next
// group (no wave waits for a fixed share).  Lanes of a group step their
// walks one brick at a time until the last ends.  The parts cost a division
// or three each at their start: the scatter, whose steps are dear (a record
// store each), gains from them, the histogram (an LDS increment a step) does
// not.
// emit(brick id, klo, khi, staged segment, brick x, y, z, N) per piece,
// [klo, khi] being the segment's k-window inside the brick.  The segment is
// read from LDS once per walk, so what the emitter derives from it alone is
// computed once per walk, not per piece.
template <bool kSplit, int kN, typename Emit>
__device__ __forceinline__ void walk_ordered(Stage<kN>& st, const BrickGeom& bg, bool euclid, Emit emit) {
    const uint32_t lane = __lane_id();
    const uint32_t nvalid = st.nvalid;
    // Ends of the classes in the order, and their first groups (without
    // kSplit every walk is in the last class).
    const uint32_t e8 = kSplit ? st.bins[kBinEnd8] : 0u;
    const uint32_t e4 = kSplit ? st.bins[kBinEnd4] : 0u;
    const uint32_t e2 = kSplit ? st.bins[kBinEnd2] : 0u;
    const uint32_t g4 = (e8 + 7u) >> 3;
    const uint32_t g2 = g4 + ((e4 - e8 + 15u) >> 4);
    const uint32_t g1 = g2 + ((e2 - e4 + 31u) >> 5);
    const uint32_t gt = g1 + ((nvalid - e2 + 63u) >> 6);
    for (;;) {
        uint32_t grp = 0;
        if (lane == 0) grp = atomicAdd(&st.claim, 1u);
        grp = __builtin_amdgcn_readfirstlane(grp);
        if (grp >= gt) break;
        uint32_t lgp, start, end;
        if (grp < g4) {
            lgp = 3; start = grp << 3; end = e8;
        } else if (grp < g2) {
            lgp = 2; start = e8 + ((grp - g4) << 4); end = e4;
        } else if (grp < g1) {
            lgp = 1; start = e4 + ((grp - g2) << 5); end = e2;
        } else {
            lgp = 0; start = e2 + ((grp - g1) << 6); end = nvalid;
        }
        const uint32_t i = start + (lane >> lgp);
        bool active = i < end;
        StagedSeg g = {};
        WalkState w = {};
        if (active) {
            g = st.seg[st.order[i]];
            active = walk_init(w, g, bg, euclid, lane & ((1u << lgp) - 1u), 1u << lgp);
        }
        while (__ballot(active)) {
            uint32_t km = w.c[0].kn < w.c[1].kn ? w.c[0].kn : w.c[1].kn;
            km = km < w.c[2].kn ? km : w.c[2].kn;
            const bool more = km <= w.kend;
            // Brick ids and counts stay below 2^24: 24-bit multiplies.
            if (active)
                emit(__umul24(__umul24((uint32_t)w.c[2].b, (uint32_t)bg.nb[1]) + (uint32_t)w.c[1].b,
                              (uint32_t)bg.nb[0]) +
                         (uint32_t)w.c[0].b,
                     w.klo, more ? km - 1u : w.kend, g, w.c[0].b, w.c[1].b, w.c[2].b, w.N);
            // The rest with selects only (lanes step different segments).
            const bool go = active && more;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) cross_advance(w.c[ax], go && w.c[ax].kn == km);
            w.klo = go ? km : w.klo;
            active = go;
        }
    }
}

// Histogram of one row: its segments' pieces per brick of its scene.
template <int kN>
__device__ __forceinline__ void hist_row(const BrickScene& sc, uint32_t g, Stage<kN>& st, uint32_t* lh,
                                         CountScratch* cscratch, const WorkView& wv) {
    const BrickGeom& bg = sc.bg;
    const uint32_t NB = bg.nbricks;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) lh[b] = 0;
    int64_t lo, hi;
    seg_range(sc.n, (int)g, (int)sc.rows, lo, hi);
    const bool euclid = (sc.flags & kSceneEuclid) != 0;
    bool bad = false;
    for (int64_t base = lo; base < hi; base += kN) {
        const uint32_t cnt = (uint32_t)(hi - base < kN ? hi - base : kN);
        stage_segments(sc.segs, base, cnt, bg, euclid, st, sc.counts, bad);
        walk_ordered<false>(st, bg, euclid,
                            [&](uint32_t b, uint32_t, uint32_t, const StagedSeg&, int32_t, int32_t, int32_t, uint32_t) {
                                atomicAdd(&lh[b], 1u);
                            });
        if (euclid && sc.counts) euclid_counts(st, sc.counts + base, cscratch);
        lds_barrier();
    }
    // (Out-of-volume segments are reported by the scatter, or by the direct
    // kernels when they serve the scene: the status word may still be
    // written by this kernel's first workgroup in a plain call.)
    (void)bad;
    lds_barrier();
    uint32_t* row = wv.hist + sc.hist_off + (size_t)g * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) row[b] = lh[b];
}

// LDS of the histogram kernel: 8 192 staged segments and up to 8 192 brick
// counters, or 4 096 staged segments and up to 16 384 counters; each
// workgroup takes the layout its scene's brick count allows.
constexpr size_t kHistLdsBig = sizeof(Stage<kStageBig>) + (size_t)kBigStageBricks * 4;
constexpr size_t kHistLdsSmall = sizeof(Stage<kStage>) + (size_t)kMaxBricks * 4;
// ... then the per-wave scratch of the Euclidean counts.
constexpr size_t kHistLds = (kHistLdsBig > kHistLdsSmall ? kHistLdsBig : kHistLdsSmall) + kCountScratch;
static_assert(kHistLds <= 163840, "histogram LDS fits a workgroup");

__global__ __launch_bounds__(kHistBlock) void k_brick_hist(uint8_t* __restrict__ work) {
    extern __shared__ __align__(16) uint8_t hist_lds[];
    const TableView tv = table_view(work + kWorkTable);
    const WorkView wv = work_of(work, tv);
    const uint32_t r = xcd_row(blockIdx.x, gridDim.x);
    if (*wv.ok == 0 || r >= tv.h.rows) return;
    const BrickScene sc = tv.scenes[tv.row_scene ? tv.row_scene[r] : 0u];
    const uint32_t g = r - sc.row_base;
    if (sc.bg.nbricks <= kBigStageBricks) {
        auto* st = reinterpret_cast<Stage<kStageBig>*>(hist_lds);
        hist_row(sc, g, *st, reinterpret_cast<uint32_t*>(hist_lds + sizeof(Stage<kStageBig>)),
                 reinterpret_cast<CountScratch*>(hist_lds + kHistLdsBig), wv);
    } else {
        auto* st = reinterpret_cast<Stage<kStage>*>(hist_lds);
        hist_row(sc, g, *st, reinterpret_cast<uint32_t*>(hist_lds + sizeof(Stage<kStage>)),
                 reinterpret_cast<CountScratch*>(hist_lds + kHistLdsSmall), wv);
    }
}

// A plain call's plan and histogram in one launch: every workgroup plans the
// call's one scene (passed by value) itself, the first one also writes the
// table and header words for the kernels that follow (what k_brick_plan
// writes for a single scene), and the workgroups go on to their histogram
// rows when the brick kernels may run.
__global__ __launch_bounds__(kHistBlock) void k_brick_plan_hist(vox_scene one, BrickLaunch L,
                                                               uint8_t* __restrict__ work, uint64_t work_bytes) {
    extern __shared__ __align__(16) uint8_t hist_lds[];
    BrickScene sc;
    const bool valid = plan_scene(one, L.lg, L.segs_per_row, sc);
    const bool isd = (sc.flags & kSceneDirect) != 0;
    sc.row_base = 0;
    sc.brick_base = 0;
    sc.hist_off = 0;
    const uint32_t nb = isd ? 0u : sc.bg.nbricks;
    const uint64_t n = sc.n > 0 ? (uint64_t)sc.n : 0u;
    const uint64_t hist_c = (uint64_t)sc.rows * nb;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        BrickScene* out = reinterpret_cast<BrickScene*>(work + kWorkTable + kTableScenes);
        out[0] = sc;
        if (isd) reinterpret_cast<uint32_t*>(out + 1)[0] = 0u;
        write_table(work, L, work_bytes, sc.rows, nb, isd ? 1u : 0u, nb, hist_c, n, isd ? n : 0u, !valid);
    }
    // The same decision as the ok word written above.
    const WorkView wv = work_view(work, kWorkTable + L.table_bytes, hist_c, nb);
    const bool fits = n <= L.total_segments && sc.rows <= L.rows && nb <= L.bricks;
    if (!valid || !fits || wv.rec_off > work_bytes || nb == 0) return;
    const uint32_t r = xcd_row(blockIdx.x, gridDim.x);
    if (r >= sc.rows) return;
    if (nb <= kBigStageBricks) {
        auto* st = reinterpret_cast<Stage<kStageBig>*>(hist_lds);
        hist_row(sc, r, *st, reinterpret_cast<uint32_t*>(hist_lds + sizeof(Stage<kStageBig>)),
                 reinterpret_cast<CountScratch*>(hist_lds + kHistLdsBig), wv);
    } else {
        auto* st = reinterpret_cast<Stage<kStage>*>(hist_lds);
        hist_row(sc, r, *st, reinterpret_cast<uint32_t*>(hist_lds + sizeof(Stage<kStage>)),
                 reinterpret_cast<CountScratch*>(hist_lds + kHistLdsSmall), wv);
    }
}

constexpr int kBaseBlock = 1024;

// The brick totals pass through LDS in chunks of kBaseChunk bricks: loaded
// coalesced (all of a thread's loads issued before any is used), read in
// runs of consecutive bricks per thread for the scans, and the results (bin
// offsets, item offsets, the brick of each item) staged in LDS and written
// back coalesced: from one workgroup, stores of the threads' runs would each
// touch a memory line of their own.  Entry i of a stage sits at i + i / 32,
// so that the lanes' runs (16 entries apart) fall in different banks.
constexpr uint32_t kBaseChunk = 16384;
constexpr uint32_t kBaseStage = (kBaseChunk + 1024u) + (kBaseChunk + 1024u) / 32;  // a chunk's items at most
__device__ __forceinline__ uint32_t stage_slot(uint32_t i) { return i + (i >> 5); }

template <int kBlock>
__device__ __forceinline__ void stage_in(const uint32_t* __restrict__ src, uint32_t m, uint32_t* st) {
    constexpr int kPer = (int)(kBaseChunk / kBlock);
    uint32_t v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t i = threadIdx.x + (uint32_t)k * kBlock;
        v[k] = i < m ? src[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) st[stage_slot(threadIdx.x + (uint32_t)k * kBlock)] = v[k];
    __syncthreads();
}

template <int kBlock>
__device__ __forceinline__ void stage_out(const uint32_t* st, uint32_t m, uint32_t* __restrict__ dst) {
    for (uint32_t i = threadIdx.x; i < m; i += kBlock) dst[i] = st[stage_slot(i)];
}

// Exclusive scan, from `base`, of f(entry) over the m entries of a stage
// (runs of kBaseChunk / kBlock consecutive entries per thread, one block
// scan of the run sums; lds: kBlock / 64 entries) into the stage `out`;
// returns the sum.
template <int kBlock, typename F>
__device__ __forceinline__ uint64_t scan_stage(const uint32_t* st, uint32_t m, uint64_t base, uint32_t* out,
                                               uint64_t* lds, F f, uint32_t* max_s = nullptr) {
    constexpr uint32_t kRun = kBaseChunk / kBlock;
    const uint32_t r0 = threadIdx.x * kRun;
    uint64_t run = 0;
    uint32_t mx = 0;
    for (uint32_t k = 0; k < kRun && r0 + k < m; ++k) {
        const uint32_t c = st[stage_slot(r0 + k)];
        run += f(c);
        mx = c > mx ? c : mx;
    }
    if (max_s) {
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)mx, d, kWave);
            mx = o > mx ? o : mx;
        }
        if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(max_s, mx);  // (read after the scan's barriers)
    }
    uint64_t sum;
    uint64_t off = base + block_exclusive_sum<kBlock>(run, lds, sum);
    for (uint32_t k = 0; k < kRun && r0 + k < m; ++k) {
        out[stage_slot(r0 + k)] = (uint32_t)off;
        off += f(st[stage_slot(r0 + k)]);
    }
    __syncthreads();
    return sum;
}

// bin_base[b] = sum of totals before global brick b, bin_base[NB] = total,
// by one block of kBlock threads, a chunk at a time.  The direct kernels
// take over when the records do not fit the workspace (or reach 2^32 - 1).
template <int kBlock>
__device__ __forceinline__ uint64_t scan_totals(const WorkView& wv, uint32_t NB, uint64_t work_bytes, uint64_t* lds,
                                                uint32_t* st, uint32_t* ob, uint32_t* max_s) {
    uint64_t total = 0;
    if (threadIdx.x == 0) *max_s = 0u;  // (ordered before the atomics by stage_in's barrier)
    for (uint32_t c0 = 0; c0 < NB; c0 += kBaseChunk) {
        const uint32_t m = NB - c0 < kBaseChunk ? NB - c0 : kBaseChunk;
        stage_in<kBlock>(wv.totals + c0, m, st);
        total += scan_stage<kBlock>(st, m, total, ob, lds, [](uint32_t c) { return (uint64_t)c; }, max_s);
        stage_out<kBlock>(ob, m, wv.bin_base + c0);
        __syncthreads();  // both stages are rewritten by the next chunk (st read by make_items)
    }
    if (threadIdx.x == 0) {
        wv.bin_base[NB] = (uint32_t)total;
        *wv.pieces = total;
        const uint64_t cap = work_bytes > wv.rec_off ? (work_bytes - wv.rec_off) / sizeof(Piece) : 0u;
        if (total > cap || total >= 0xFFFFFFFFull) *wv.direct_all = 1u;
    }
    return total;
}

// The fill's work items (see kSplitShares) when some brick is cut, the same
// way: item_base[b] = items before brick b; the list of cut bricks; the
// brick of each item, staged in LDS (the totals' stage, free by then) and
// written back coalesced; the counts in the header.  With a single chunk the
// stage still holds the totals from scan_totals.  When no brick is cut the
// items are the bricks (n_split = 0 tells the fill and the scatter so, and
// the item arrays are not written).
template <int kBlock>
__device__ __forceinline__ void make_items(const WorkView& wv, uint32_t NB, uint64_t total, uint64_t* lds,
                                           uint32_t* st, uint32_t* ob, uint32_t* n_split_s) {
    const uint64_t T = split_threshold(total);
    if (threadIdx.x == 0) *n_split_s = 0u;  // (ordered before the atomics below by the scan's barriers)
    uint64_t items = 0;
    for (uint32_t c0 = 0; c0 < NB; c0 += kBaseChunk) {
        const uint32_t m = NB - c0 < kBaseChunk ? NB - c0 : kBaseChunk;
        if (NB > kBaseChunk) stage_in<kBlock>(wv.totals + c0, m, st);
        const uint64_t sum = scan_stage<kBlock>(st, m, items, ob, lds, [T](uint32_t c) {
            return (uint64_t)brick_items(c, T);
        });
        stage_out<kBlock>(ob, m, wv.item_base + c0);
        // A brick's items are the difference of its item offset and the
        // next one.  The chunk's cut bricks, then the brick of each of the
        // chunk's items (at most kBaseChunk + 1023 of them) through the
        // totals' stage, free by now, and out coalesced.
        const uint32_t end = (uint32_t)(items + sum);
        __syncthreads();  // every thread's scan reads of st are done
        for (uint32_t i = threadIdx.x; i < m; i += kBlock) {
            const uint32_t o = ob[stage_slot(i)];
            const uint32_t n = (i + 1u < m ? ob[stage_slot(i + 1u)] : end) - o;
            if (n > 1u) wv.split[atomicAdd(n_split_s, 1u)] = c0 + i;
            for (uint32_t j = 0; j < n; ++j) st[stage_slot(o - (uint32_t)items + j)] = c0 + i;
        }
        __syncthreads();
        stage_out<kBlock>(st, (uint32_t)sum, wv.item_brick + items);
        items += sum;
        __syncthreads();  // both stages are rewritten by the next chunk
    }
    if (threadIdx.x == 0) {
        wv.item_base[NB] = (uint32_t)items;
        *wv.n_items = (uint32_t)items;
        *wv.n_split = *n_split_s;
    }
}

constexpr int kColBins = 64;
constexpr int kColSplit = 4;  // row chunks per brick
constexpr int kColRows = (kHistRows + kColSplit - 1) / kColSplit;
constexpr uint32_t kColMaxBlocks = 4096;

// Blocks of 256 threads = 64 global bricks x 4 row chunks (the blocks step
// over all bricks): per brick, exclusive prefix of its scene's histogram
// column over the scene's rows (in place) and the brick total.
__global__ __launch_bounds__(256) void k_brick_colscan(uint8_t* __restrict__ work) {
    __shared__ uint32_t part[kColSplit][kColBins];
    const TableView tv = table_view(work + kWorkTable);
    const WorkView wv = work_of(work, tv);
    if (*wv.ok == 0) return;
    const int bl = threadIdx.x % kColBins;
    const int ch = threadIdx.x / kColBins;
    for (uint32_t gb0 = blockIdx.x * kColBins; gb0 < tv.h.bricks; gb0 += gridDim.x * kColBins) {
        const uint32_t gb = gb0 + bl;
        const bool valid = gb < tv.h.bricks;
        uint32_t b = 0, NB = 0;
        int G = 0;
        uint64_t off = 0;
        if (valid) {
            const BrickScene& sc = tv.scenes[tv.brick_scene ? tv.brick_scene[gb] : 0u];
            b = gb - sc.brick_base;
            NB = sc.bg.nbricks;
            G = (int)sc.rows;
            off = sc.hist_off;
        }
        uint32_t* hist = wv.hist + off;
        const int g0 = ch * kColRows;
        uint32_t v[kColRows];
        uint32_t sum = 0;
#pragma unroll
        for (int r = 0; r < kColRows; ++r) {
            const int g = g0 + r;
            v[r] = (valid && g < G) ? hist[(size_t)g * NB + b] : 0u;
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
            if (valid && g < G) hist[(size_t)g * NB + b] = run;
            run += v[r];
        }
        if (ch == 0 && valid) wv.totals[gb] = tot;
        __syncthreads();
    }
}


// One block: bin_base[b] = sum of totals before global brick b;
// bin_base[bricks] = total.  When the records do not fit the rest of the
// workspace (or their count reaches 2^32 - 1), the direct kernels serve
// every scene instead of the scatter and the fill.
__global__ __launch_bounds__(kBaseBlock) void k_brick_base(uint8_t* __restrict__ work, uint64_t work_bytes) {
    __shared__ uint64_t lds[kBaseBlock / kWave];
    __shared__ uint32_t st[kBaseStage], ob[kBaseStage];
    __shared__ uint32_t n_split_s, max_s;
    const TableView tv = table_view(work + kWorkTable);
    const WorkView wv = work_of(work, tv);
    if (*wv.ok == 0) return;
    const uint64_t total = scan_totals<kBaseBlock>(wv, tv.h.bricks, work_bytes, lds, st, ob, &max_s);
    if ((uint64_t)max_s > split_threshold(total)) {
        make_items<kBaseBlock>(wv, tv.h.bricks, total, lds, st, ob, &n_split_s);
    } else if (threadIdx.x == 0) {
        *wv.n_items = tv.h.bricks;
        *wv.n_split = 0u;
    }
}

// The record of the piece of staged segment g with k-window [klo, khi] in
// brick (bx, by, bz).  Every volume side is at most 16384, so N < 2^15 and
// eq. (3)'s numerator 2 klo a + N stays below 2^31 (divmod_down's domain).
__device__ __forceinline__ Piece piece_record(const StagedSeg& g, uint32_t klo, uint32_t khi, int32_t bx,
                                              int32_t by, int32_t bz, const BrickGeom& bg) {
    int32_t p0[3], d[3];
    uint32_t ad[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        p0[ax] = g.p0[ax];
        d[ax] = (int32_t)g.p1[ax] - p0[ax];
        ad[ax] = (uint32_t)(d[ax] < 0 ? -d[ax] : d[ax]);
    }
    const uint32_t N = ad[0] > ad[1] ? (ad[0] > ad[2] ? ad[0] : ad[2]) : (ad[1] > ad[2] ? ad[1] : ad[2]);
    const uint32_t m = ad[0] == N ? 0u : (ad[1] == N ? 1u : 2u);
    const uint32_t aa = m == 0 ? ad[1] : ad[0], ab = m == 2 ? ad[1] : ad[2];
    const int32_t da = m == 0 ? d[1] : d[0], db = m == 2 ? d[1] : d[2];
    const int32_t dm = m == 0 ? d[0] : (m == 1 ? d[1] : d[2]);
    const uint32_t nega = da < 0, negb = db < 0, negm = dm < 0;
    const uint32_t two_n = N > 0 ? 2u * N : 2u;
    uint32_t qa = 0, ra = 0, qb = 0, rb = 0;
    if (N > 0) {
        const float rcpd = rcp_down(two_n);
        divmod_down(2u * __umul24(klo, aa) + N - nega, two_n, rcpd, qa, ra);
        divmod_down(2u * __umul24(klo, ab) + N - negb, two_n, rcpd, qb, rb);
    }
    const int32_t vm = negm ? -(int32_t)klo : (int32_t)klo;
    const int32_t va = nega ? -(int32_t)qa : (int32_t)qa, vb = negb ? -(int32_t)qb : (int32_t)qb;
    const int32_t x = p0[0] + (m == 0 ? vm : va) - (bx << bg.lg[0]);
    const int32_t y = p0[1] + (m == 1 ? vm : (m == 0 ? va : vb)) - (by << bg.lg[1]);
    const int32_t z = p0[2] + (m == 2 ? vm : vb) - (bz << bg.lg[2]);
    Piece pc;
    pc.e = ((ra + 32768u - two_n) & 0xFFFFu) | ((rb + 32768u - two_n) << 16);
    pc.t = (2u * aa) | ((2u * ab) << 16);
    pc.v = m | (nega << 2) | (negb << 3) | (negm << 4) | (two_n << 16);
    pc.w = (uint32_t)(x + (y << bg.lg[0]) + (z << (bg.lg[0] + bg.lg[1]))) |
           ((khi - klo) << (bg.lg[0] + bg.lg[1] + bg.lg[2]));
    return pc;
}

// The record of a piece under the Euclidean N of eq. (1), where every axis,
// the dominant one too, may stay put at a step: as piece_record, but the
// first word holds klo | 2 a_m << 16 (a_m = |d| of the dominant axis), from
// which the fill derives the three axes' remainders at klo, and the length
// counts the piece's samples k = klo ... khi (duplicates included).  N is at
// most 16384 (the scene's diagonal is below 16385), so 2 klo a + N < 2^31.
__device__ __forceinline__ Piece piece_record_euclid(const StagedSeg& g, uint32_t N, uint32_t klo, uint32_t khi,
                                                     int32_t bx, int32_t by, int32_t bz, const BrickGeom& bg) {
    int32_t p0[3], d[3];
    uint32_t ad[3], c[3] = {0u, 0u, 0u};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        p0[ax] = g.p0[ax];
        d[ax] = (int32_t)g.p1[ax] - p0[ax];
        ad[ax] = (uint32_t)(d[ax] < 0 ? -d[ax] : d[ax]);
    }
    const uint32_t amax = ad[0] > ad[1] ? (ad[0] > ad[2] ? ad[0] : ad[2]) : (ad[1] > ad[2] ? ad[1] : ad[2]);
    const uint32_t m = ad[0] == amax ? 0u : (ad[1] == amax ? 1u : 2u);
    const uint32_t aa = m == 0 ? ad[1] : ad[0], ab = m == 2 ? ad[1] : ad[2];
    const uint32_t am = m == 0 ? ad[0] : (m == 1 ? ad[1] : ad[2]);
    const int32_t da = m == 0 ? d[1] : d[0], db = m == 2 ? d[1] : d[2];
    const int32_t dm = m == 0 ? d[0] : (m == 1 ? d[1] : d[2]);
    const uint32_t two_n = N > 0 ? 2u * N : 2u;
    if (N > 0) {
        const float rcpd = rcp_down(two_n);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            uint32_t r;
            divmod_down(2u * __umul24(klo, ad[ax]) + N - (d[ax] < 0 ? 1u : 0u), two_n, rcpd, c[ax], r);
        }
    }
    const int32_t x = p0[0] + (d[0] < 0 ? -(int32_t)c[0] : (int32_t)c[0]) - (bx << bg.lg[0]);
    const int32_t y = p0[1] + (d[1] < 0 ? -(int32_t)c[1] : (int32_t)c[1]) - (by << bg.lg[1]);
    const int32_t z = p0[2] + (d[2] < 0 ? -(int32_t)c[2] : (int32_t)c[2]) - (bz << bg.lg[2]);
    Piece pc;
    pc.e = klo | ((2u * am) << 16);
    pc.t = (2u * aa) | ((2u * ab) << 16);
    pc.v = m | ((uint32_t)(da < 0) << 2) | ((uint32_t)(db < 0) << 3) | ((uint32_t)(dm < 0) << 4) | (two_n << 16);
    pc.w = (uint32_t)(x + (y << bg.lg[0]) + (z << (bg.lg[0] + bg.lg[1]))) |
           ((khi - klo) << (bg.lg[0] + bg.lg[1] + bg.lg[2]));
    return pc;
}

// In cleared brick scenes, zeroes the bricks cut into several work items
// (their items OR into the volume), one workgroup a brick, before the fill.
__device__ __forceinline__ void zero_cut_bricks(const TableView& tv, const WorkView& wv) {
    const uint32_t ns = *wv.n_split;
    for (uint32_t j = blockIdx.x; j < ns; j += gridDim.x) {
        const uint32_t gb = wv.split[j];
        const BrickScene& sc = tv.scenes[tv.brick_scene ? tv.brick_scene[gb] : 0u];
        if (!(sc.flags & kSceneClear)) continue;
        const BrickGeom& bg = sc.bg;
        const uint32_t lb = gb - sc.brick_base;
        const int32_t org[3] = {(int32_t)(lb % (uint32_t)bg.nb[0]) << bg.lg[0],
                                (int32_t)((lb / (uint32_t)bg.nb[0]) % (uint32_t)bg.nb[1]) << bg.lg[1],
                                (int32_t)(lb / ((uint32_t)bg.nb[0] * (uint32_t)bg.nb[1])) << bg.lg[2]};
        int32_t ext[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int32_t e = bg.dim[ax] - org[ax];
            ext[ax] = e < (1 << bg.lg[ax]) ? e : (1 << bg.lg[ax]);
        }
        // A brick has at most 2^20 bits: 32-bit index arithmetic.
        const uint32_t xws = (uint32_t)ext[0] >> 5, ey = (uint32_t)ext[1];
        const uint32_t words = xws * ey * (uint32_t)ext[2];
        const int64_t row_words = (int64_t)bg.dim[0] >> 5;
        for (uint32_t t = threadIdx.x; t < words; t += blockDim.x) {
            const uint32_t xw = t % xws, r = t / xws;
            const uint32_t y = r % ey, z = r / ey;
            sc.grid[((int64_t)(org[2] + (int32_t)z) * bg.dim[1] + (org[1] + (int32_t)y)) * row_words +
                    (org[0] >> 5) + xw] = 0u;
        }
    }
}

__global__ __launch_bounds__(kHistBlock) void k_brick_scatter(uint8_t* __restrict__ work) {
    extern __shared__ uint32_t cur[];
    __shared__ Stage<kStage> st;
    const TableView tv = table_view(work + kWorkTable);
    const WorkView wv = work_of(work, tv);
    const uint32_t r = xcd_row(blockIdx.x, gridDim.x);
    if (*wv.ok == 0 || *wv.direct_all != 0) return;
    zero_cut_bricks(tv, wv);
    if (r >= tv.h.rows) return;
    const BrickScene sc = tv.scenes[tv.row_scene ? tv.row_scene[r] : 0u];
    const BrickGeom& bg = sc.bg;
    const uint32_t NB = bg.nbricks;
    const uint32_t g = r - sc.row_base;
    const uint32_t* row = wv.hist + sc.hist_off + (size_t)g * NB;
    const uint32_t* base_b = wv.bin_base + sc.brick_base;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) cur[b] = base_b[b] + row[b];
    int64_t lo, hi;
    seg_range(sc.n, (int)g, (int)sc.rows, lo, hi);
    Piece* __restrict__ recs = wv.recs;
    const bool euclid = (sc.flags & kSceneEuclid) != 0;
    bool bad = false;
    for (int64_t base = lo; base < hi; base += kStage) {
        const uint32_t cnt = (uint32_t)(hi - base < kStage ? hi - base : kStage);
        stage_segments(sc.segs, base, cnt, bg, euclid, st, nullptr, bad);
        if (euclid) {
            walk_ordered<true>(st, bg, true, [&](uint32_t b, uint32_t klo, uint32_t khi, const StagedSeg& g,
                                                 int32_t bx, int32_t by, int32_t bz, uint32_t N) {
                const uint32_t pos = atomicAdd(&cur[b], 1u);
                recs[pos] = piece_record_euclid(g, N, klo, khi, bx, by, bz, bg);
            });
        } else {
            walk_ordered<true>(st, bg, false, [&](uint32_t b, uint32_t klo, uint32_t khi, const StagedSeg& g,
                                                  int32_t bx, int32_t by, int32_t bz, uint32_t) {
                const uint32_t pos = atomicAdd(&cur[b], 1u);
                recs[pos] = piece_record(g, klo, khi, bx, by, bz, bg);
            });
        }
        lds_barrier();
    }
    if (bad) atomicOr(wv.status, kStatusOutOfRange);
}

// ------------------------------------------------------------------- fill

template <int LGX, int LGY, int LGZ>
struct BrickShape {
    static constexpr int kBXw = 1 << (LGX - 5);                       // words per row
    static constexpr uint32_t kWords = (uint32_t)kBXw << (LGY + LGZ);
    static constexpr size_t kBytes = (size_t)kWords * 4;
    static constexpr int kMaxLg = LGX > LGY ? (LGX > LGZ ? LGX : LGZ) : (LGY > LGZ ? LGY : LGZ);
};

// Stepping state of a piece at its first voxel, made once per piece by the
// lane that loaded its record and read by the lanes that run its chunks
// (five words):
//   e: E0, the two minor axes' error terms as biased 16-bit halves
//      u = r - 2N + 32768 (r the remainder of eq. (3)'s division at k = klo)
//   t: T, the halves' increments 2a
//   s: S, the minor axes' signed strides in the brick, negated, as 16-bit
//      halves (minor axes a < b in axis order)
//   v: the dominant axis' signed stride (low half) | 2N << 16 (2 when N = 0)
//   w: bit index of the voxel at k = klo inside the brick | (len - 1) << kIdxBits
// and, with the Euclidean N only, where the dominant axis need not move at
// every step:
//   m: its error term as a biased 16-bit half | its increment 2a_m << 16
struct Digest {
    uint32_t e, t, s, v, w, m;
};

template <int LGX, int LGY, int LGZ>
struct DigestBits {
    static constexpr int kIdxBits = LGX + LGY + LGZ;
    static constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
    // Strides up to 2^(LGX+LGY) as signed 16-bit halves; lengths up to the
    // brick's largest side above the bit index.
    static_assert(LGX + LGY <= 14, "strides must fit signed 16-bit halves");
    static_assert(kIdxBits + (LGX > LGY ? (LGX > LGZ ? LGX : LGZ) : (LGY > LGZ ? LGY : LGZ)) <= 32,
                  "bit index and length share a word");
};

// The stepping state of a record's piece (the record holds it but for the
// strides, which follow from the axes, the signs and the brick shape).
template <int LGX, int LGY, int LGZ>
__device__ __forceinline__ Digest digest_record(const u32x4& rec) {
    const uint32_t m = rec.z & 3u, nega = (rec.z >> 2) & 1u, negb = (rec.z >> 3) & 1u, negm = (rec.z >> 4) & 1u;
    // Strides are powers of two: log2 of the dominant axis' and of the
    // minor axes' strides.
    const uint32_t shm = m == 0 ? 0u : (m == 1 ? (uint32_t)LGX : (uint32_t)(LGX + LGY));
    const uint32_t sha = m == 0 ? (uint32_t)LGX : 0u, shb = m == 2 ? (uint32_t)LGX : (uint32_t)(LGX + LGY);
    const int32_t sm = negm ? -(1 << shm) : (1 << shm);
    const int32_t sa = nega ? (1 << sha) : -(1 << sha), sb = negb ? (1 << shb) : -(1 << shb);
    Digest g;
    g.e = rec.x;
    g.t = rec.y;
    g.s = ((uint32_t)sa & 0xFFFFu) | ((uint32_t)sb << 16);
    g.v = ((uint32_t)sm & 0xFFFFu) | (rec.z & 0xFFFF0000u);
    g.w = rec.w;
    g.m = 0u;
    return g;
}

// The same under the Euclidean N (records of piece_record_euclid): the
// remainders of eq. (3)'s divisions at k = klo, for the two minor axes and
// the dominant one, from klo and the increments.  A record holds 2N >= 2 and
// klo, 2a <= 2N <= 32768, so the numerators stay below 2^31.
template <int LGX, int LGY, int LGZ>
__device__ __forceinline__ Digest digest_record_euclid(const u32x4& rec) {
    Digest g = digest_record<LGX, LGY, LGZ>(rec);
    const uint32_t nega = (rec.z >> 2) & 1u, negb = (rec.z >> 3) & 1u, negm = (rec.z >> 4) & 1u;
    const uint32_t two_n = rec.z >> 16 > 1u ? rec.z >> 16 : 2u;
    const uint32_t n = two_n >> 1;
    const uint32_t klo = rec.x & 0xFFFFu, two_am = rec.x >> 16;
    const uint32_t two_a = rec.y & 0xFFFFu, two_b = rec.y >> 16;
    const float rcpd = rcp_down(two_n);
    uint32_t q, ra, rb, rm;
    divmod_down(__umul24(klo, two_a) + n - nega, two_n, rcpd, q, ra);
    divmod_down(__umul24(klo, two_b) + n - negb, two_n, rcpd, q, rb);
    divmod_down(__umul24(klo, two_am) + n - negm, two_n, rcpd, q, rm);
    g.e = ((ra + 32768u - two_n) & 0xFFFFu) | ((rb + 32768u - two_n) << 16);
    g.m = ((rm + 32768u - two_n) & 0xFFFFu) | (two_am << 16);
    return g;
}

// Word of the LDS brick holding bit index idx.  A valid piece stays inside
// its brick; the mask keeps every LDS access inside the brick whatever a
// record holds (the address computation needs a mask anyway, so this costs
// no instruction).
template <int LGX, int LGY, int LGZ>
__device__ __forceinline__ uint32_t brick_word(int32_t idx) {
    return ((uint32_t)idx >> 5) & (BrickShape<LGX, LGY, LGZ>::kWords - 1u);
}

// Sets the bits of chunk j (voxels klo + j*kChunk ... , at most kChunk of
// them; exactly kChunk when kFull) of the piece with digest g.
//
// The dominant axis moves by one voxel per step.  Adding 2a to a minor
// axis' biased half sets its bit 15 exactly when that coordinate advances.
// A packed arithmetic shift turns those bits into 0 / -1 halves, which
// subtract 2N from their halves in one packed multiply-add and add the axes'
// signed strides to the bit index in one packed dot product (with the
// strides stored negated).  Needs 2N <= 32768.  A chunk starts from the
// piece's state advanced by koff = j*kChunk steps: one division per minor
// axis gives the remainders and the numbers of advances Q, and the bit index
// moves by koff dominant strides and Q minor ones (one more dot product,
// with -Q against the negated strides).
template <bool kFull, int kChunk, int LGX, int LGY, int LGZ>
__device__ __forceinline__ void run_chunk(uint32_t* brick, const Digest& g, uint32_t j) {
    using DB = DigestBits<LGX, LGY, LGZ>;
    const uint32_t two_n = g.v >> 16;
    const int32_t sm = (int32_t)(int16_t)(g.v & 0xFFFFu);
    const uint32_t koff = j * (uint32_t)kChunk;
    // Scalars first: this compiler's __builtin_bit_cast of a vector or
    // struct element can read the wrong element.
    const uint32_t ge = g.e, gt = g.t, gs = g.s;
    const u16x2 E0 = __builtin_bit_cast(u16x2, ge);
    const u16x2 T = __builtin_bit_cast(u16x2, gt);
    const i16x2 S = __builtin_bit_cast(i16x2, gs);
    const float rcpd = rcp_down(two_n);
    uint32_t qa, ra, qb, rb;
    divmod_down((uint32_t)E0.x + two_n - 32768u + __umul24(koff, (uint32_t)T.x), two_n, rcpd, qa, ra);
    divmod_down((uint32_t)E0.y + two_n - 32768u + __umul24(koff, (uint32_t)T.y), two_n, rcpd, qb, rb);
    u16x2 E = {(uint16_t)(ra + 32768u - two_n), (uint16_t)(rb + 32768u - two_n)};
    const u16x2 Q = {(uint16_t)qa, (uint16_t)qb};
    const u16x2 Z = {0, 0};
    int32_t idx = __builtin_amdgcn_sdot2(__builtin_bit_cast(i16x2, Z - Q), S,
                                         (int32_t)(g.w & DB::kIdxMask) + (int32_t)koff * sm, false);
    const u16x2 N2 = {(uint16_t)two_n, (uint16_t)two_n};
    const i16x2 k15 = {15, 15};
    if constexpr (kFull) {
#pragma unroll 8
        for (int k = 0; k < kChunk; ++k) {
            atomicOr(&brick[brick_word<LGX, LGY, LGZ>(idx)], 1u << ((uint32_t)idx & 31u));
            E = E + T;
            const i16x2 C = __builtin_bit_cast(i16x2, E) >> k15;  // -1 where the axis advances
            E = E + __builtin_bit_cast(u16x2, C) * N2;
            idx = __builtin_amdgcn_sdot2(C, S, idx, false) + sm;
        }
    } else {
        const uint32_t len = (g.w >> DB::kIdxBits) + 1u;
        const int n = (int)(len - koff < (uint32_t)kChunk ? len - koff : (uint32_t)kChunk);
        for (int k = 0; k < n; ++k) {
            atomicOr(&brick[brick_word<LGX, LGY, LGZ>(idx)], 1u << ((uint32_t)idx & 31u));
            E = E + T;
            const i16x2 C = __builtin_bit_cast(i16x2, E) >> k15;
            E = E + __builtin_bit_cast(u16x2, C) * N2;
            idx = __builtin_amdgcn_sdot2(C, S, idx, false) + sm;
        }
    }
}

// As run_chunk, under the Euclidean N of eq. (1): the dominant axis moves
// only when its own error term carries, so it takes a second packed pair
// (its biased half and a zero half that never carries), whose carry adds
// its stride through a second dot product.  A step that moves no axis sets
// the same bit again.  The chunk's start needs a third division.
template <bool kFull, int kChunk, int LGX, int LGY, int LGZ>
__device__ __forceinline__ void run_chunk_euclid(uint32_t* brick, const Digest& g, uint32_t j) {
    using DB = DigestBits<LGX, LGY, LGZ>;
    const uint32_t two_n = g.v >> 16;
    const int32_t sm = (int32_t)(int16_t)(g.v & 0xFFFFu);
    const uint32_t koff = j * (uint32_t)kChunk;
    const uint32_t ge = g.e, gt = g.t, gs = g.s, gm = g.m;
    const u16x2 E0 = __builtin_bit_cast(u16x2, ge);
    const u16x2 T = __builtin_bit_cast(u16x2, gt);
    const i16x2 S = __builtin_bit_cast(i16x2, gs);
    const uint32_t em0 = gm & 0xFFFFu, two_am = gm >> 16;
    const float rcpd = rcp_down(two_n);
    uint32_t qa, ra, qb, rb, qm, rm;
    divmod_down((uint32_t)E0.x + two_n - 32768u + __umul24(koff, (uint32_t)T.x), two_n, rcpd, qa, ra);
    divmod_down((uint32_t)E0.y + two_n - 32768u + __umul24(koff, (uint32_t)T.y), two_n, rcpd, qb, rb);
    divmod_down(em0 + two_n - 32768u + __umul24(koff, two_am), two_n, rcpd, qm, rm);
    u16x2 E = {(uint16_t)(ra + 32768u - two_n), (uint16_t)(rb + 32768u - two_n)};
    u16x2 Em = {(uint16_t)(rm + 32768u - two_n), 0};
    const u16x2 Tm = {(uint16_t)two_am, 0};
    const i16x2 Sm = {(int16_t)(-sm), 0};  // negated, as S
    const u16x2 Q = {(uint16_t)qa, (uint16_t)qb};
    const u16x2 Z = {0, 0};
    int32_t idx = __builtin_amdgcn_sdot2(__builtin_bit_cast(i16x2, Z - Q), S,
                                         (int32_t)(g.w & DB::kIdxMask) + (int32_t)qm * sm, false);
    const u16x2 N2 = {(uint16_t)two_n, (uint16_t)two_n};
    const i16x2 k15 = {15, 15};
    const uint32_t len = (g.w >> DB::kIdxBits) + 1u;
    const int n = kFull ? kChunk : (int)(len - koff < (uint32_t)kChunk ? len - koff : (uint32_t)kChunk);
#pragma unroll 8
    for (int k = 0; k < n; ++k) {
        atomicOr(&brick[brick_word<LGX, LGY, LGZ>(idx)], 1u << ((uint32_t)idx & 31u));
        E = E + T;
        const i16x2 C = __builtin_bit_cast(i16x2, E) >> k15;
        E = E + __builtin_bit_cast(u16x2, C) * N2;
        Em = Em + Tm;
        const i16x2 Cm = __builtin_bit_cast(i16x2, Em) >> k15;
        Em = Em + __builtin_bit_cast(u16x2, Cm) * N2;
        idx = __builtin_amdgcn_sdot2(Cm, Sm, __builtin_amdgcn_sdot2(C, S, idx, false), false);
    }
}

// Most samples of one piece.  A piece lies in one brick.  With the Chebyshev
// N its dominant coordinate moves by one voxel per k, so it has at most as
// many samples as the brick's longest side L.  With the Euclidean N
// (N <= sqrt(3) a_m) the dominant coordinate moves by more than
// (khi - klo) a_m / N - 1 between klo and khi and by at most L - 1 inside
// the brick, so khi - klo < sqrt(3) L and a piece has at most 7L/4 samples
// (L >= 32).
template <bool kEuclid, int LGX, int LGY, int LGZ>
struct MaxSamples {
    static constexpr uint32_t kSide = 1u << BrickShape<LGX, LGY, LGZ>::kMaxLg;
    static constexpr uint32_t kValue = kEuclid ? kSide * 7u / 4u : kSide;
    static_assert(kSide >= 32, "7L/4 bounds sqrt(3) L + 1");
    static_assert(DigestBits<LGX, LGY, LGZ>::kIdxBits + BrickShape<LGX, LGY, LGZ>::kMaxLg + 1 <= 32,
                  "bit index and length share a word");
};

// Samples of a piece record (from its last word); a record outside the
// bound above (which the scatter never writes) counts as empty, so that
// every loop of the fill stays bounded whatever the workspace holds.
template <bool kEuclid, int LGX, int LGY, int LGZ>
__device__ __forceinline__ uint32_t record_length(uint32_t w) {
    const uint32_t len = (w >> DigestBits<LGX, LGY, LGZ>::kIdxBits) + 1u;
    return len <= MaxSamples<kEuclid, LGX, LGY, LGZ>::kValue ? len : 0u;
}

// A piece record, read once: a non-temporal load, so that the stream of
// records does not push the volume's partly written lines out of the L2.
__device__ __forceinline__ u32x4 load_stream(const u32x4* p) {
    return __builtin_nontemporal_load(p);
}

// A brick's records [lo, hi) in four quarters, one per SIMD of the CU.
constexpr int kQuarters = 4;
constexpr int kSets = 2;  // piece records per lane in a wave group

__device__ __forceinline__ uint32_t quarter_bound(uint32_t lo, uint32_t hi, uint32_t k) {
    return lo + (uint32_t)(((uint64_t)(hi - lo) * k) / kQuarters);
}

// Cursors of the quarters' groups after the first `skip` records of each,
// which the waves take without a claim (first_group).
__device__ __forceinline__ void set_quarters(uint32_t* cursors, uint32_t lo, uint32_t hi, uint32_t skip) {
#pragma unroll
    for (uint32_t k = 0; k < (uint32_t)kQuarters; ++k) cursors[k] = quarter_bound(lo, hi, k) + skip;
}

// The first group of a wave in a brick with records [lo, hi): group `slot`
// of its SIMD's quarter qu (the waves of a SIMD take slots 0, 1, ...), its
// records loaded now.  q_hi: the end of the quarter.
__device__ __forceinline__ void first_group(const u32x4* recv, uint32_t lo, uint32_t hi, uint32_t qu, uint32_t slot,
                                            uint32_t lane, uint32_t& gbase, uint32_t& q_hi, u32x4& r0, u32x4& r1) {
    constexpr uint32_t kGroup = kWave * kSets;
    q_hi = quarter_bound(lo, hi, qu + 1u);
    gbase = quarter_bound(lo, hi, qu) + slot * kGroup;
    r0 = (gbase + lane < q_hi) ? load_stream(recv + gbase + lane) : (u32x4){0u, 0u, 0u, 0u};
    r1 = (gbase + kWave + lane < q_hi) ? load_stream(recv + gbase + kWave + lane) : (u32x4){0u, 0u, 0u, 0u};
}

// Launch shape of the fill kernel: kWgs workgroups per CU, of 1024 threads
// (one per CU) or 512 (two per CU).  A 128 KiB brick takes a whole CU; 64 KiB
// bricks run either way: two workgroups per CU, so that one workgroup's brick
// start and flush overlap the other's voxel work, or, when the volume has
// fewer bricks than that gives slots, one with all 16 waves on its brick.
constexpr int kFillChunk = 32;  // samples per chunk
template <int LGX, int LGY, int LGZ, int kWgs>
struct FillCfg {
    static_assert(kWgs == 1 || (kWgs == 2 && LGX + LGY + LGZ < 20), "two workgroups per CU: 64 KiB bricks");
    static constexpr int kBlock = kWgs == 1 ? 1024 : 512;
    static constexpr int kWgsPerCu = kWgs;
};

// The pieces of one brick that this wave runs: groups of 128 records (two
// per lane: sets 0 and 1), taken from its SIMD's quarter qu of the brick's
// records (waves w and w + 4k share a SIMD), so the four SIMDs get even
// shares of the brick's work.  The first group (gbase, records rn0 and rn1)
// comes loaded (first_group); each next group is claimed and loaded before
// the current one runs.  q_hi: the end of the quarter.  kEuclid: the brick's
// scene uses the Euclidean N of eq. (1).
template <bool kEuclid, int LGX, int LGY, int LGZ, int kEntCap>
__device__ __forceinline__ void fill_records(uint32_t* brick, uint16_t* my_ent, const u32x4* recv,
                                             uint32_t* cursor_s, uint32_t qu, uint32_t q_hi, uint32_t gbase,
                                             u32x4 rn0, u32x4 rn1, uint32_t lane) {
    constexpr int kChunk = kFillChunk;
    constexpr int kGroup = kWave * kSets;  // records per wave group
    constexpr int kMaxChunks = (MaxSamples<kEuclid, LGX, LGY, LGZ>::kValue + kChunk - 1) / kChunk;  // per piece
    // A group with more chunks than the table holds runs its two record sets
    // one after the other.
    constexpr bool kSplit = kEntCap < kGroup * kMaxChunks;
    static_assert(kMaxChunks <= 512, "chunk entries: lane | set << 6 | j << 7");
    static_assert(kEntCap >= kWave * kMaxChunks, "one record set's chunks always fit the table");
    while (gbase < q_hi) {
        const u32x4 r0 = rn0, r1 = rn1;
        const uint32_t len0 = gbase + lane < q_hi ? record_length<kEuclid, LGX, LGY, LGZ>(r0.w) : 0u;
        const uint32_t len1 = gbase + kWave + lane < q_hi ? record_length<kEuclid, LGX, LGY, LGZ>(r1.w) : 0u;
        // The records have arrived (len0/len1 are made from them); the next
        // group's loads are issued only now, so no later wait for these
        // records waits for them too.
        asm volatile("" ::"v"(len0), "v"(len1) : "memory");
        if (lane == 0) gbase = atomicAdd(&cursor_s[qu], (uint32_t)kGroup);
        gbase = __builtin_amdgcn_readfirstlane(gbase);
        rn0 = (gbase + lane < q_hi) ? load_stream(recv + gbase + lane) : (u32x4){0u, 0u, 0u, 0u};
        rn1 = (gbase + kWave + lane < q_hi) ? load_stream(recv + gbase + kWave + lane) : (u32x4){0u, 0u, 0u, 0u};

        // This lane's pieces as stepping states (read by the lanes that
        // run their chunks).
        const Digest d0 = kEuclid ? digest_record_euclid<LGX, LGY, LGZ>(r0) : digest_record<LGX, LGY, LGZ>(r0);
        const Digest d1 = kEuclid ? digest_record_euclid<LGX, LGY, LGZ>(r1) : digest_record<LGX, LGY, LGZ>(r1);
        const uint32_t nf0 = len0 / kChunk, pl0 = len0 % kChunk;
        const uint32_t nf1 = len1 / kChunk, pl1 = len1 % kChunk;
        // Length class of a partial chunk: 3 (longest) ... 0, or 4 (none).
        const uint32_t k0 = pl0 == 0 ? 4u : pl0 * 4u / kChunk, k1 = pl1 == 0 ? 4u : pl1 * 4u / kChunk;

        // Chunks of this lane's pieces: their full chunks, then their
        // partial chunks.  The wave's table lists all full chunks first,
        // then the partial ones in four length classes, longest first, so
        // that most rounds run chunks of one length.  Two packed DPP scans
        // count all five lists.  Sets 0 and 1 share one table, or take
        // turns when their chunks overflow it.
        uint32_t sets = 3u;
        for (;;) {
            const uint32_t u0 = sets & 1u, u1 = sets >> 1;
            const uint32_t f0 = u0 ? nf0 : 0u, f1 = u1 ? nf1 : 0u;
            const uint32_t q0 = u0 ? k0 : 4u, q1 = u1 ? k1 : 4u;
            const uint32_t c3 = (q0 == 3u) + (q1 == 3u), c2 = (q0 == 2u) + (q1 == 2u);
            const uint32_t c1 = (q0 == 1u) + (q1 == 1u), c0 = (q0 == 0u) + (q1 == 0u);
            const uint32_t ia = wave_inclusive_sum_dpp((f0 + f1) | (c3 << 16));
            const uint32_t ib = wave_inclusive_sum_dpp(c2 | (c1 << 10) | (c0 << 20));
            const uint32_t ta = __builtin_amdgcn_readlane(ia, kWave - 1);
            const uint32_t tb = __builtin_amdgcn_readlane(ib, kWave - 1);
            const uint32_t tf = ta & 0xFFFFu;                      // full chunks
            const uint32_t o2 = tf + (ta >> 16);                   // start of class 2
            const uint32_t o1 = o2 + (tb & 0x3FFu);
            const uint32_t o0 = o1 + ((tb >> 10) & 0x3FFu);
            const uint32_t tt = o0 + (tb >> 20);
            if (kSplit && tt > (uint32_t)kEntCap) {
                sets = 1u;  // set 0 now, set 1 next
                continue;
            }
            {
                const uint32_t fb = (ia & 0xFFFFu) - f0 - f1;
                for (uint32_t j = 0; j < f0; ++j) my_ent[fb + j] = (uint16_t)(lane | (j << 7));
                for (uint32_t j = 0; j < f1; ++j) my_ent[fb + f0 + j] = (uint16_t)(lane | 64u | (j << 7));
                // End of this lane's run in each class list.
                const uint32_t e3 = tf + (ia >> 16), e2 = o2 + (ib & 0x3FFu);
                const uint32_t e1 = o1 + ((ib >> 10) & 0x3FFu), e0 = o0 + (ib >> 20);
                if (q0 < 4u) {
                    const uint32_t pos = q0 == 3u ? e3 - c3 : q0 == 2u ? e2 - c2 : q0 == 1u ? e1 - c1 : e0 - c0;
                    my_ent[pos] = (uint16_t)(lane | (nf0 << 7));
                }
                if (q1 < 4u) {
                    const uint32_t pos = q1 == 3u ? e3 - 1u : q1 == 2u ? e2 - 1u : q1 == 1u ? e1 - 1u : e0 - 1u;
                    my_ent[pos] = (uint16_t)(lane | 64u | (nf1 << 7));
                }
            }
            // Make the table writes visible to the wave's own reads below.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

            for (uint32_t q = 0; q < tt; q += kWave) {
                const uint32_t c = q + lane;
                const uint32_t e = c < tt ? my_ent[c] : 0u;
                const int src = (int)((e & 63u) << 2);
                const bool s1 = (e & 64u) != 0u;
                const uint32_t ge0 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d0.e);
                const uint32_t ge1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d1.e);
                const uint32_t gt0 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d0.t);
                const uint32_t gt1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d1.t);
                const uint32_t gs0 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d0.s);
                const uint32_t gs1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d1.s);
                const uint32_t gv0 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d0.v);
                const uint32_t gv1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d1.v);
                const uint32_t gw0 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d0.w);
                const uint32_t gw1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d1.w);
                Digest g = {s1 ? ge1 : ge0, s1 ? gt1 : gt0, s1 ? gs1 : gs0, s1 ? gv1 : gv0, s1 ? gw1 : gw0, 0u};
                if constexpr (kEuclid) {
                    const uint32_t gm0 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d0.m);
                    const uint32_t gm1 = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)d1.m);
                    g.m = s1 ? gm1 : gm0;
                    if (q + kWave <= tf) {
                        run_chunk_euclid<true, kChunk, LGX, LGY, LGZ>(brick, g, e >> 7);
                    } else if (c < tt) {
                        run_chunk_euclid<false, kChunk, LGX, LGY, LGZ>(brick, g, e >> 7);
                    }
                } else {
                    if (q + kWave <= tf) {
                        run_chunk<true, kChunk, LGX, LGY, LGZ>(brick, g, e >> 7);
                    } else if (c < tt) {
                        run_chunk<false, kChunk, LGX, LGY, LGZ>(brick, g, e >> 7);
                    }
                }
            }
            // The table is rewritten by the next pass or group.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (sets != 1u) break;
            sets = 2u;
        }
    }
}


// Persistent fill.  Workgroups take work items (a brick, or part of a cut
// brick) from the work queues (work stealing: bricks differ a lot in work).
// Inside an item the waves work independently, with no workgroup barrier
// until the item is done: a wave takes the next 128 piece records of its
// SIMD's quarter of the item's records (two per lane), turns them into
// digests, cuts the pieces into chunks of at most kChunk voxels, lists the
// chunks in its own LDS table (full chunks first) and runs them in rounds of
// 64, one chunk per lane, reading each chunk's digest from the owning lane
// with ds_bpermute.  The next 128 records are loaded while the current ones
// run.
template <int LGX, int LGY, int LGZ, int kWgs>
__global__ __launch_bounds__((FillCfg<LGX, LGY, LGZ, kWgs>::kBlock), kWgs)
void k_brick_fill(uint8_t* __restrict__ work) {
    using Shape = BrickShape<LGX, LGY, LGZ>;
    using Cfg = FillCfg<LGX, LGY, LGZ, kWgs>;
    constexpr int kBlock = Cfg::kBlock, kChunk = kFillChunk;
    constexpr int kWaves = kBlock / kWave;
    constexpr int kMaxChunks = ((int)MaxSamples<true, LGX, LGY, LGZ>::kValue + kChunk - 1) / kChunk;  // per piece
    constexpr int kUpr = Shape::kBXw / 4;  // 16-byte units per brick row
    constexpr int kGroup = kWave * kSets;  // records per wave group
    // Chunk table entries per wave: all chunks of a group when the LDS left
    // by the brick holds them, else a multiple of 64 below that.
    constexpr int kLdsWg = 163840 / Cfg::kWgsPerCu;
    constexpr int kEntFit = ((kLdsWg - (int)Shape::kBytes - 64) / (2 * kWaves)) / kWave * kWave;
    constexpr int kEntCap = kGroup * kMaxChunks < kEntFit ? kGroup * kMaxChunks : kEntFit;
    static_assert(kWave == 64 && kSets == 2, "chunk entries: lane | set << 6 | j << 7");
    // The brick first, so its addresses need no base offset.
    __shared__ __align__(16) uint32_t brick[Shape::kWords];
    __shared__ uint16_t ent[kWaves][kEntCap];  // per-wave chunk tables
    __shared__ uint32_t cursor_s[kQuarters];  // per-SIMD record cursors of the brick
    __shared__ uint32_t next_s[4];

    const TableView tv = table_view(work + kWorkTable);
    const WorkView wv = work_of(work, tv);
    if (*wv.ok == 0 || *wv.direct_all != 0) return;
    const uint32_t NB = tv.h.bricks;  // global bricks of all scenes
    const uint32_t n_items = *wv.n_items, n_split = *wv.n_split;
    const uint32_t lane = __lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    uint16_t* my_ent = ent[wave];
    const u32x4* recv = reinterpret_cast<const u32x4*>(wv.recs);

    // The waves of a SIMD take the first kWaves / 4 groups of its quarter
    // without a claim (first_group); the cursors start after them.
    constexpr uint32_t kSkip = (uint32_t)(kWaves / kQuarters) * (uint32_t)kGroup;
    const uint32_t qu = wave % kQuarters, slot = wave / kQuarters;
    // The next work item (its brick and record range) is claimed by thread 0
    // at the start of the current one, so its memory latency overlaps this
    // item's work.
    if (threadIdx.x == 0) {
        const ItemClaim c = claim_item(wv, blockIdx.x % kXcds, n_items, n_split, NB);
        next_s[0] = c.brick;
        next_s[1] = c.lo;
        next_s[2] = c.hi;
        next_s[3] = c.split;
        set_quarters(cursor_s, c.lo, c.hi, kSkip);
    }
    {
        u32x4* b4 = reinterpret_cast<u32x4*>(brick);
        for (uint32_t w = threadIdx.x; w < Shape::kWords / 4; w += kBlock) b4[w] = (u32x4){0, 0, 0, 0};
    }
    lds_barrier();
    uint32_t b = next_s[0];
    uint32_t p_lo = next_s[1], p_hi = next_s[2], split = next_s[3];
    uint32_t gbase = 0, q_hi = 0;
    u32x4 rn0 = {0u, 0u, 0u, 0u}, rn1 = {0u, 0u, 0u, 0u};
    if (b < NB) first_group(recv, p_lo, p_hi, qu, slot, lane, gbase, q_hi, rn0, rn1);

    while (b < NB) {
        ItemClaim nc = {NB, 0u, 0u, 0u};
        if (threadIdx.x == 0) nc = claim_item(wv, blockIdx.x % kXcds, n_items, n_split, NB);
        // The brick's scene and its place in that scene's volume.
        const uint32_t gb = __builtin_amdgcn_readfirstlane(b);
        const BrickScene& sc = tv.scenes[tv.brick_scene ? tv.brick_scene[gb] : 0u];
        const BrickGeom bg = sc.bg;
        uint32_t* __restrict__ grid = sc.grid;
        const bool clear = (sc.flags & kSceneClear) != 0;
        const uint32_t lb = gb - sc.brick_base;
        const int64_t row_words = (int64_t)bg.dim[0] >> 5;
        const int bx = (int)(lb % (uint32_t)bg.nb[0]);
        const int by = (int)((lb / (uint32_t)bg.nb[0]) % (uint32_t)bg.nb[1]);
        const int bz = (int)(lb / ((uint32_t)bg.nb[0] * (uint32_t)bg.nb[1]));
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
        // (The brick is zero and the cursors set: done before the barrier that
        // ended the previous brick.)

        // This wave's pieces of the brick.
        if (sc.flags & kSceneEuclid)
            fill_records<true, LGX, LGY, LGZ, kEntCap>(brick, my_ent, recv, cursor_s, qu, q_hi, gbase, rn0, rn1,
                                                       lane);
        else
            fill_records<false, LGX, LGY, LGZ, kEntCap>(brick, my_ent, recv, cursor_s, qu, q_hi, gbase, rn0, rn1,
                                                        lane);
        // Hand over the next item (read by all after the barrier).
        if (threadIdx.x == 0) {
            next_s[0] = nc.brick;
            next_s[1] = nc.lo;
            next_s[2] = nc.hi;
            next_s[3] = nc.split;
        }
        lds_barrier();  // every wave done with this item
        const uint32_t b_next = next_s[0], lo_next = next_s[1], hi_next = next_s[2], split_next = next_s[3];
        // The next item's first group is loaded before the flush's stores:
        // a wait for a load also waits for every store issued before it, so
        // loaded after the flush its records would arrive only once the
        // whole brick had been written.
        if (b_next < NB) first_group(recv, lo_next, hi_next, qu, slot, lane, gbase, q_hi, rn0, rn1);

        // Flush: brick rows -> volume words, zeroing the brick on the way.
        // The owner of a whole brick writes every word of it, so a clearing
        // call needs no other pass.  A brick with no pieces in a scene that
        // ORs into its volume changes nothing: no flush (its LDS copy is
        // still zero).  An item holding part of a cut brick ORs its nonzero
        // words into the volume with device atomics (the other items of the
        // brick do the same; the scatter zeroed the brick first in a cleared
        // volume).
        const int rows = (clear || p_lo != p_hi) ? ext[1] * ext[2] : 0;
        // Whole 16-byte units when the volume's rows hold whole brick rows.
        const bool vec = Shape::kBXw % 4 == 0 && (bg.dim[0] & ((1 << LGX) - 1)) == 0;
        const bool full_y = ext[1] == (1 << LGY);  // rows per slab a power of two
        if (split) {
            const int xws = ext[0] >> 5;  // whole words: dim_x and the brick origin are multiples of 32
            const int total = rows * xws;
            for (int t = threadIdx.x; t < total; t += kBlock) {
                const int xw = t % xws, r = t / xws;
                const int y = r % ext[1], z = r / ext[1];
                uint32_t* src = &brick[(((uint32_t)z << LGY) | (uint32_t)y) * (uint32_t)Shape::kBXw + xw];
                const uint32_t v = *src;
                *src = 0u;  // zero for the next item
                if (v != 0u)
                    __hip_atomic_fetch_or(grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words +
                                              (org[0] >> 5) + xw,
                                          v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else if (vec && full_y) {
            // 16-byte units, kUpr per row, rows full width and full slabs:
            // a thread's units share their row in the slab and their part of
            // the row, and step by a fixed number of slabs (kBlock units are
            // a whole number of slabs in every compiled shape).
            constexpr int kRowsPerStep = kBlock / kUpr;
            static_assert(kBlock % kUpr == 0 && kRowsPerStep % (1 << LGY) == 0, "whole slabs per step");
            constexpr int kSlabsPerStep = kRowsPerStep >> LGY;
            const int units = rows * kUpr;
            const int part = (int)threadIdx.x % kUpr, r0 = (int)threadIdx.x / kUpr;
            const int y = r0 & ((1 << LGY) - 1), z0 = r0 >> LGY;
            u32x4* src = reinterpret_cast<u32x4*>(
                &brick[(((uint32_t)z0 << LGY) | (uint32_t)y) * (uint32_t)Shape::kBXw + 4u * part]);
            global_u32x4* dst = (global_u32x4*)(
                grid + ((int64_t)(org[2] + z0) * bg.dim[1] + (org[1] + y)) * row_words + (org[0] >> 5) + 4 * part);
            const int64_t dst_step = (int64_t)kSlabsPerStep * bg.dim[1] * row_words / 4;  // in 16-byte units
            for (int t = threadIdx.x; t < units; t += kBlock) {
                const u32x4 v = *src;
                *src = (u32x4){0u, 0u, 0u, 0u};  // zero for the next item
                if (clear) {
                    *dst = v;
                } else {
                    *dst = *dst | v;
                }
                src += kBlock;
                dst += dst_step;
            }
        } else if (vec) {
            // 16-byte units, kUpr per row, rows full width.
            const int units = rows * kUpr;
            for (int t = threadIdx.x; t < units; t += kBlock) {
                const int part = t % kUpr, r = t / kUpr;
                const int y = full_y ? (r & ((1 << LGY) - 1)) : r % ext[1];
                const int z = full_y ? (r >> LGY) : r / ext[1];
                u32x4* src = reinterpret_cast<u32x4*>(
                    &brick[(((uint32_t)z << LGY) | (uint32_t)y) * (uint32_t)Shape::kBXw + 4u * part]);
                const u32x4 v = *src;
                *src = (u32x4){0u, 0u, 0u, 0u};  // zero for the next item
                global_u32x4* dst = (global_u32x4*)(
                    grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words + (org[0] >> 5) +
                    4 * part);
                if (clear) {
                    *dst = v;
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
                uint32_t* src = &brick[(((uint32_t)z << LGY) | (uint32_t)y) * (uint32_t)Shape::kBXw + xw];
                const uint32_t v = *src;
                *src = 0u;  // zero for the next item
                global_u32* dst = (global_u32*)grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words +
                                (org[0] >> 5) + xw;
                if (clear) *dst = v;
                else *dst |= v;
            }
        }
        // Every word that can hold a bit (inside the volume) was read and
        // zeroed above; the others were never set.  Next item:
        b = b_next;
        p_lo = lo_next;
        p_hi = hi_next;
        split = split_next;
        if (threadIdx.x == 0) set_quarters(cursor_s, p_lo, p_hi, kSkip);
        lds_barrier();
    }
}

// ------------------------------------------------------- direct scenes

constexpr int kDirectBlock = 256;

// The scenes the direct kernels serve: those the brick path does not take
// (flagged by the plan), or every scene when the records did not fit.
// Nothing runs after a failed plan.
__device__ __forceinline__ bool direct_scenes(const uint8_t* work, const TableView& tv, uint32_t& count,
                                              bool& all) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(work);
    if (w[kWStatus] & (uint32_t)(kStatusInvalid | kStatusLaunch)) return false;
    all = w[kWDirectAll] != 0;
    count = all ? tv.h.n_scenes : tv.h.n_direct;
    return count > 0;
}

// Zeroes the volumes of the cleared direct scenes (before the fill; the
// direct kernel sets their bits after it).
__global__ __launch_bounds__(kDirectBlock) void k_batch_direct_clear(uint8_t* __restrict__ work) {
    const TableView tv = table_view(work + kWorkTable);
    const int64_t t0 = (int64_t)blockIdx.x * kDirectBlock + threadIdx.x;
    const int64_t ts = (int64_t)gridDim.x * kDirectBlock;
    uint32_t nd;
    bool all;
    if (!direct_scenes(work, tv, nd, all)) return;
    for (uint32_t j = 0; j < nd; ++j) {
        const BrickScene& sc = tv.scenes[all ? j : tv.direct[j]];
        if (!(sc.flags & kSceneClear)) continue;
        const int64_t nwords = ((int64_t)sc.bg.dim[0] * sc.bg.dim[1] * sc.bg.dim[2] + 31) / 32;
        clear_words(sc.grid, nwords, t0, ts);
    }
}

// The segments of the direct scenes, one device atomic per voxel
// (direct_segments, vox_direct.h).
__global__ __launch_bounds__(kDirectBlock) void k_batch_direct(uint8_t* __restrict__ work) {
    const TableView tv = table_view(work + kWorkTable);
    uint32_t nd;
    bool all;
    if (!direct_scenes(work, tv, nd, all)) return;
    int32_t* status = reinterpret_cast<int32_t*>(work) + kWStatus;
    const int64_t wave0 = (int64_t)blockIdx.x * (kDirectBlock / kWave) + threadIdx.x / kWave;
    const int64_t ws = (int64_t)gridDim.x * (kDirectBlock / kWave);
    for (uint32_t j = 0; j < nd; ++j) {
        const BrickScene sc = tv.scenes[all ? j : tv.direct[j]];
        const int32_t dx = sc.bg.dim[0], dy = sc.bg.dim[1], dz = sc.bg.dim[2];
        const bool a8 = (sc.flags & kSceneA8) != 0;
        if (sc.flags & kSceneEuclid) {
            if (a8)
                direct_segments<true, true>(sc.segs, sc.n, dx, dy, dz, sc.grid, sc.counts, status, wave0, ws);
            else
                direct_segments<false, true>(sc.segs, sc.n, dx, dy, dz, sc.grid, sc.counts, status, wave0, ws);
        } else {
            if (a8)
                direct_segments<true, false>(sc.segs, sc.n, dx, dy, dz, sc.grid, sc.counts, status, wave0, ws);
            else
                direct_segments<false, false>(sc.segs, sc.n, dx, dy, dz, sc.grid, sc.counts, status, wave0, ws);
        }
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

bool brick_geometry_for(int32_t dx, int32_t dy, int32_t dz, const int lg[3], BrickGeom& bg) {
    return brick_geometry(dx, dy, dz, lg, bg);
}

// 256 x 64 x 64 bricks (128 KiB of LDS) when the volume still has at least
// 4096 of them, i.e. 16 per CU for the work stealing to balance; otherwise
// 256 x 64 x 32.  Rows of 256 voxels are 32 bytes, whole memory sectors.
void default_brick_lg(int32_t dx, int32_t dy, int32_t dz, int lg[3]) {
    const int64_t big = ((int64_t)(dx + 255) >> 8) * ((dy + 63) >> 6) * ((dz + 63) >> 6);
    lg[0] = 8;
    lg[1] = 6;
    lg[2] = big >= 4096 ? 6 : 5;
}

// Worst case of pieces: every segment crossing every brick boundary of
// every axis once.
uint64_t max_pieces(int64_t n, const BrickGeom& bg) {
    return (uint64_t)n * (uint64_t)(1 + (bg.nb[0] - 1) + (bg.nb[1] - 1) + (bg.nb[2] - 1));
}

static uint64_t table_bytes(uint32_t n_scenes, uint32_t rows, uint32_t bricks) {
    uint64_t b = kTableScenes + (uint64_t)n_scenes * (sizeof(BrickScene) + 4u);
    if (n_scenes > 1) b += 4ull * ((uint64_t)rows + bricks);
    return up256(b);
}

BrickLaunch batch_launch(uint32_t n_scenes, uint64_t total_segments, const int lg[3]) {
    BrickLaunch L;
    L.n_scenes = n_scenes;
    L.total_segments = total_segments;
    // Rows of scene s: min(256, max(1, ceil(n_s / per_row))) <= 1 + n_s / per_row,
    // with the plain calls' rows of 512 segments for a single scene.
    const uint64_t per_row = n_scenes == 1 ? (uint64_t)kSegsPerRowPlain : (uint64_t)kSegsPerRow;
    uint64_t rows = (uint64_t)n_scenes + (total_segments + per_row - 1) / per_row;
    const uint64_t rmax = (uint64_t)n_scenes * kHistRows;
    L.rows = (uint32_t)(rows < rmax ? rows : rmax);
    L.bricks = (uint32_t)((uint64_t)n_scenes * kMaxBricks);
    for (int a = 0; a < 3; ++a) L.lg[a] = lg[a];
    L.table_bytes = table_bytes(n_scenes, L.rows, L.bricks);
    L.direct_kernels = true;
    L.segs_per_row = (uint32_t)per_row;
    return L;
}

// Table, histograms (each scene's rows times at most kMaxBricks bricks),
// brick totals, offsets and work items.
size_t batch_fixed_bytes(const BrickLaunch& L) {
    return (size_t)(kWorkTable + L.table_bytes + brick_data_bytes((uint64_t)L.rows * kMaxBricks, L.bricks));
}

BrickLaunch plain_launch(int64_t n, const BrickGeom& bg) {
    BrickLaunch L;
    L.n_scenes = 1;
    L.total_segments = (uint64_t)n;
    L.rows = hist_rows(n, kSegsPerRowPlain);
    L.segs_per_row = (uint32_t)kSegsPerRowPlain;
    L.bricks = bg.nbricks;
    for (int a = 0; a < 3; ++a) L.lg[a] = bg.lg[a];
    L.table_bytes = table_bytes(1, L.rows, L.bricks);
    // The caller's workspace holds the worst case of records.
    L.direct_kernels = false;
    return L;
}

size_t brick_workspace_bytes(int64_t n, const BrickGeom& bg) {
    const BrickLaunch L = plain_launch(n, bg);
    return (size_t)(kWorkTable + L.table_bytes + brick_data_bytes((uint64_t)L.rows * bg.nbricks, L.bricks) +
                    max_pieces(n, bg) * sizeof(Piece));
}

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

// Persistent fill workgroups: wgs_per_cu per compute unit (0: for 64 KiB
// bricks two, unless the launch has fewer bricks than two per CU, then one
// of 1024 threads), and no more than the launch can have work items (a
// workgroup without one would only take a CU slot).
template <int LGX, int LGY, int LGZ>
static hipError_t launch_fill(uint8_t* work, int wgs_per_cu, uint32_t max_bricks, hipStream_t stream) {
    const int cus = device_cus();
    int per = 1;
    if constexpr (LGX + LGY + LGZ < 20)
        per = wgs_per_cu == 1 || wgs_per_cu == 2 ? wgs_per_cu : (max_bricks < 2u * (uint32_t)cus ? 1 : 2);
    int wgs = cus * per;
    if ((uint64_t)wgs > (uint64_t)max_bricks + kMaxExtraItems) wgs = (int)(max_bricks + kMaxExtraItems);
    if constexpr (LGX + LGY + LGZ < 20) {
        if (per == 2) {
            k_brick_fill<LGX, LGY, LGZ, 2><<<wgs, FillCfg<LGX, LGY, LGZ, 2>::kBlock, 0, stream>>>(work);
            return hipGetLastError();
        }
    }
    k_brick_fill<LGX, LGY, LGZ, 1><<<wgs, FillCfg<LGX, LGY, LGZ, 1>::kBlock, 0, stream>>>(work);
    return hipGetLastError();
}

hipError_t launch_bricks(const void* d_scenes, const void* one, const BrickLaunch& L, int fill_wgs_per_cu,
                         void* d_work, size_t work_bytes, hipStream_t stream) {
    if (L.n_scenes < 1 || L.rows < 1 || L.bricks < 1 || !brick_shape_supported(L.lg)) return hipErrorInvalidValue;
    uint8_t* work = static_cast<uint8_t*>(d_work);
    hipError_t e;
    {
        static hipError_t attr = [] {
            hipError_t r = hipFuncSetAttribute((const void*)k_brick_hist, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kHistLds);
            if (r != hipSuccess) return r;
            r = hipFuncSetAttribute((const void*)k_brick_plan_hist, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kHistLds);
            if (r != hipSuccess) return r;
            return hipFuncSetAttribute((const void*)k_brick_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kMaxBricks * sizeof(uint32_t)));
        }();
        if (attr != hipSuccess) return attr;
    }
    // A plain call (its one scene by value; the brick geometry keeps it to at
    // most kMaxBricks bricks): the plan runs inside the histogram launch,
    // five launches in all; a batch (a device scene array) takes seven or
    // more.
    if (one) {
        if (L.n_scenes != 1 || L.bricks > kMaxBricks) return hipErrorInvalidValue;
        KernelTimer t("brick_plan_hist", stream);
        k_brick_plan_hist<<<L.rows, kHistBlock, kHistLds, stream>>>(*static_cast<const vox_scene*>(one), L, work,
                                                                    (uint64_t)work_bytes);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        {
            KernelTimer t("brick_plan", stream);
            k_brick_plan<<<1, kPlanBlock, 0, stream>>>(static_cast<const vox_scene*>(d_scenes), L, work,
                                                       (uint64_t)work_bytes);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (L.n_scenes > 1) {
            KernelTimer t("brick_expand", stream);
            const uint32_t wgs = L.n_scenes < 2048u ? L.n_scenes : 2048u;
            k_brick_expand<<<wgs, 256, 0, stream>>>(work);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        {
            KernelTimer t("brick_hist", stream);
            k_brick_hist<<<L.rows, kHistBlock, kHistLds, stream>>>(work);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        KernelTimer t("brick_colscan", stream);
        uint32_t blocks = (L.bricks + kColBins - 1) / kColBins;
        if (blocks > kColMaxBlocks) blocks = kColMaxBlocks;
        k_brick_colscan<<<blocks, 256, 0, stream>>>(work);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        KernelTimer t("brick_base", stream);
        k_brick_base<<<1, kBaseBlock, 0, stream>>>(work, (uint64_t)work_bytes);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (L.direct_kernels) {
        KernelTimer t("batch_direct_clear", stream);
        k_batch_direct_clear<<<2048, kDirectBlock, 0, stream>>>(work);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        KernelTimer t("brick_scatter", stream);
        const size_t scatter_lds = (size_t)(L.n_scenes > 1 ? kMaxBricks : L.bricks) * sizeof(uint32_t);
        k_brick_scatter<<<L.rows, kHistBlock, scatter_lds, stream>>>(work);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        KernelTimer t("brick_fill", stream);
        const int* lg = L.lg;
        if (lg[0] == 8 && lg[1] == 6 && lg[2] == 5) e = launch_fill<8, 6, 5>(work, fill_wgs_per_cu, L.bricks, stream);
        else if (lg[0] == 8 && lg[1] == 6 && lg[2] == 6) e = launch_fill<8, 6, 6>(work, fill_wgs_per_cu, L.bricks, stream);
        else if (lg[0] == 7 && lg[1] == 6 && lg[2] == 6) e = launch_fill<7, 6, 6>(work, fill_wgs_per_cu, L.bricks, stream);
        else if (lg[0] == 7 && lg[1] == 7 && lg[2] == 6) e = launch_fill<7, 7, 6>(work, fill_wgs_per_cu, L.bricks, stream);
        else e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (L.direct_kernels) {
        KernelTimer t("batch_direct", stream);
        k_batch_direct<<<4096, kDirectBlock, 0, stream>>>(work);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace vox

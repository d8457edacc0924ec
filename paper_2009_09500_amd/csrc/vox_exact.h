// Exact integer helpers of the brick path: brick walk of a segment and the
// k-window of a segment inside an axis interval.  Host and device, so the
// host-side checks exercise the very code the kernels run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vox.h"
#include "vox_device.h"
#include "vox_internal.h"

namespace vox {

// ----------------------------------------------------------- exact helpers

// ceil(x / y) for y >= 1; exact.  Small numerators (all volumes up to 4096
// voxels a side) use a float estimate corrected by one integer step.
__host__ __device__ __forceinline__ uint32_t div_ceil_u64(uint64_t x, uint32_t y) {
    if (x < (1ull << 24)) {
        uint32_t xi = (uint32_t)x;
        uint32_t q = (uint32_t)((float)xi / (float)y);
        // q is within one of floor(x / y).
        int32_t r = (int32_t)(xi - q * y);
        if (r < 0) { q -= 1; r += (int32_t)y; }
        else if (r >= (int32_t)y) { q += 1; r -= (int32_t)y; }
        return q + (r != 0 ? 1u : 0u);
    }
    return (uint32_t)((x + y - 1) / y);
}

// floor(x / y) and remainder, exact, same fast path.
__host__ __device__ __forceinline__ void divmod_u64(uint64_t x, uint32_t y, uint32_t& q, uint32_t& r) {
    if (x < (1ull << 24)) {
        uint32_t xi = (uint32_t)x;
        uint32_t qq = (uint32_t)((float)xi / (float)y);
        int32_t rr = (int32_t)(xi - qq * y);
        if (rr < 0) { qq -= 1; rr += (int32_t)y; }
        else if (rr >= (int32_t)y) { qq += 1; rr -= (int32_t)y; }
        q = qq;
        r = (uint32_t)rr;
        return;
    }
    uint64_t qq = x / y;
    q = (uint32_t)qq;
    r = (uint32_t)(x - qq * y);
}

constexpr uint32_t kNever = 0xFFFFFFFFu;

// First k at which the offset q(k) along an axis reaches m (m >= 1), or
// kNever if it never does (m > a).  a >= 1 when m <= a.
__host__ __device__ __forceinline__ uint32_t k_reach(uint32_t m, uint32_t a, uint32_t N, uint32_t neg) {
    if (m > a) return kNever;
    // Dominant axis: q(k) = k exactly.
    if (a == N) return m;
    uint64_t x = 2ull * N * m - N + neg;
    return div_ceil_u64(x, 2u * a);
}

// Brick crossings along one axis.  Crossing t happens at
// k_t = ceil(X_t / D) with D = 2a and X_t = 2 N m_t - N + neg, where m_t
// grows by the brick size B per crossing, so X_t grows by 2 N B = Q D + R
// (0 <= R < D).  Keeping the slack sl = k_t D - X_t in [0, D):
//   k_{t+1} = k_t + Q + [sl < R],  sl_{t+1} = sl + [sl < R] D - R,
// one division pair per axis and segment, none per crossing.
struct AxisCross {
    int32_t b, bend, dir;  // current brick, last brick, direction
    uint32_t kn;           // k of the next crossing, kNever if none
    uint32_t sl, Q, R, D;
};

// Crossing state of one axis at step k0 of the walk: the brick holding the
// axis coordinate at k0 and the next crossing after it.  The coordinate's
// offset from p0 at k0 is eq. (3)'s quotient there, (2 k0 a + N - neg) div 2N
// (k0 itself on an axis with a = N, 0 at k0 = 0); the next crossing is where
// the offset reaches the brick's far face, m, measured from p0.
__host__ __device__ __forceinline__ void cross_init_at(AxisCross& c, int32_t p0, int32_t p1, uint32_t a,
                                                       uint32_t neg, uint32_t N, int lg, uint32_t k0) {
    uint32_t off = 0;
    if (a == N) {
        off = k0;
    } else if (a != 0 && k0 != 0) {
        uint32_t r;
        divmod_u64(2ull * k0 * a + N - neg, 2u * N, off, r);
    }
    c.b = (neg ? p0 - (int32_t)off : p0 + (int32_t)off) >> lg;
    c.bend = p1 >> lg;
    c.dir = neg ? -1 : 1;
    c.kn = kNever;
    c.sl = c.Q = c.R = 0;
    c.D = 1;
    if (c.b == c.bend) return;
    const uint32_t m = neg ? (uint32_t)(p0 - (c.b << lg) + 1) : (uint32_t)(((c.b + 1) << lg) - p0);
    const uint32_t B = 1u << lg;
    if (a == N) {  // dominant axis: crossings exactly B apart
        c.kn = m;
        c.Q = B;
        return;
    }
    c.D = 2u * a;
    uint32_t q, r;
    divmod_u64(2ull * N * m - N + neg, c.D, q, r);
    c.kn = r ? q + 1u : q;
    c.sl = r ? c.D - r : 0u;
    divmod_u64(2ull * N * B, c.D, c.Q, c.R);
}

__host__ __device__ __forceinline__ void cross_init(AxisCross& c, int32_t p0, int32_t p1, uint32_t a,
                                                    uint32_t neg, uint32_t N, int lg) {
    cross_init_at(c, p0, p1, a, neg, N, lg, 0u);
}

// Advances an axis if `hit` (its crossing c.kn has just happened), written
// with selects only so that a wave stepping many segments does not branch.
__host__ __device__ __forceinline__ void cross_advance(AxisCross& c, bool hit) {
    const int32_t nb = c.b + c.dir;
    const bool last = nb == c.bend;
    const uint32_t carry = c.sl < c.R ? 1u : 0u;
    const uint32_t kn = last ? kNever : c.kn + c.Q + carry;
    const uint32_t sl = last ? c.sl : c.sl + (carry ? c.D : 0u) - c.R;
    c.b = hit ? nb : c.b;
    c.kn = hit ? kn : c.kn;
    c.sl = hit ? sl : c.sl;
}

// Advances an axis whose crossing c.kn has just happened.
__host__ __device__ __forceinline__ void cross_step(AxisCross& c) { cross_advance(c, true); }

struct SegAxes {
    int32_t p0[3];
    int32_t p1[3];
    uint32_t a[3];
    uint32_t neg[3];
    uint32_t N;
};

__host__ __device__ __forceinline__ SegAxes seg_axes(const Seg& g) {
    SegAxes s;
    s.N = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        s.p0[ax] = g.p0[ax];
        s.p1[ax] = g.p1[ax];
        int32_t d = g.p1[ax] - g.p0[ax];
        s.neg[ax] = d < 0;
        s.a[ax] = (uint32_t)(d < 0 ? -d : d);
        s.N = s.a[ax] > s.N ? s.a[ax] : s.N;
    }
    return s;
}

// Cutting a walk into parts.  A long segment crosses many bricks, and the
// lanes of a wave that walk segments side by side wait for the longest, so
// the kernels cut a walk of an estimated `est` pieces into walk_parts(est)
// parts (power-of-two sizes, so that a wave takes segments of one part count
// at a time) and walk the parts on separate lanes.  The estimate is
// 1 + sum_a |brick_a(P1) - brick_a(P0)|, exact unless axes cross at the same
// k.  The cuts lie at brick crossings of one axis, so the parts' pieces are
// exactly the whole walk's: the same records, found in a shorter time.
constexpr uint32_t kMaxWalkParts = 8;
__host__ __device__ __forceinline__ uint32_t walk_estimate(const int32_t p0[3], const int32_t p1[3],
                                                           const int32_t lg[3]) {
    uint32_t est = 1;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int32_t db = (p1[ax] >> lg[ax]) - (p0[ax] >> lg[ax]);
        est += (uint32_t)(db < 0 ? -db : db);
    }
    return est;
}
__host__ __device__ __forceinline__ uint32_t walk_parts(uint32_t est) {
    return est >= 64u ? 8u : (est >= 32u ? 4u : (est >= 16u ? 2u : 1u));
}

// k-window [k0, k1] of part `part` of `parts`.  The cuts follow the axis that
// spans the most bricks (the first such axis), nbs of them: part i holds its
// bricks [i nbs / parts, (i + 1) nbs / parts) in walk order, from the step
// that enters the first to the step before the one that leaves the last.
// Crossing t of that axis is the step at which the offset from p0 reaches
// m0 + t B (m0: the start brick's far face, B: the brick size).  Returns
// false for a part with no brick (nbs < parts).
__host__ __device__ __forceinline__ bool part_window(const int32_t p0[3], const int32_t p1[3], const uint32_t a[3],
                                                     const uint32_t neg[3], uint32_t N, const int32_t lg[3],
                                                     uint32_t part, uint32_t parts, uint32_t& k0, uint32_t& k1) {
    int32_t q0 = p0[0], l = lg[0];
    uint32_t nbs = 0, as = a[0], ns = neg[0];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int32_t db = (p1[ax] >> lg[ax]) - (p0[ax] >> lg[ax]);
        const uint32_t n = (uint32_t)(db < 0 ? -db : db) + 1u;
        const bool more = n > nbs;
        nbs = more ? n : nbs;
        q0 = more ? p0[ax] : q0;
        l = more ? lg[ax] : l;
        as = more ? a[ax] : as;
        ns = more ? neg[ax] : ns;
    }
    const uint32_t j0 = part * nbs / parts, j1 = (part + 1u) * nbs / parts;
    if (j0 == j1) return false;
    const int32_t b0 = q0 >> l;
    const uint32_t m0 = ns ? (uint32_t)(q0 - (b0 << l) + 1) : (uint32_t)(((b0 + 1) << l) - q0);
    const uint32_t B = 1u << l;
    k0 = j0 == 0u ? 0u : k_reach(m0 + (j0 - 1u) * B, as, N, ns);
    k1 = j1 == nbs ? N : k_reach(m0 + (j1 - 1u) * B, as, N, ns) - 1u;
    return true;
}

// Walks the bricks of part `part` of `parts` of one in-volume segment in
// order (parts = 1: the whole walk), calling emit(brick id, klo, khi) with
// the k-window [klo, khi] of the segment inside each brick: a window ends
// where the next crossing begins, or at the part's end.
template <typename Emit>
__host__ __device__ __forceinline__ void walk_bricks_part(const SegAxes& s, const BrickGeom& bg, uint32_t part,
                                                          uint32_t parts, Emit emit) {
    uint32_t k0 = 0, k1 = s.N;
    if (parts > 1u && !part_window(s.p0, s.p1, s.a, s.neg, s.N, bg.lg, part, parts, k0, k1)) return;
    AxisCross c[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) cross_init_at(c[ax], s.p0[ax], s.p1[ax], s.a[ax], s.neg[ax], s.N, bg.lg[ax], k0);
    uint32_t klo = k0;
    while (true) {
        uint32_t km = c[0].kn < c[1].kn ? c[0].kn : c[1].kn;
        km = km < c[2].kn ? km : c[2].kn;
        const bool more = km <= k1;
        emit((uint32_t)((c[2].b * bg.nb[1] + c[1].b) * bg.nb[0] + c[0].b), klo, more ? km - 1u : k1);
        if (!more) break;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) cross_advance(c[ax], c[ax].kn == km);
        klo = km;
    }
}

template <typename Emit>
__host__ __device__ __forceinline__ void walk_bricks(const SegAxes& s, const BrickGeom& bg, Emit emit) {
    walk_bricks_part(s, bg, 0u, 1u, emit);
}

__host__ __device__ __forceinline__ bool in_volume(const Seg& g, const BrickGeom& bg) {
    bool ok = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
        ok &= (g.p0[ax] >= 0) & (g.p0[ax] < bg.dim[ax]) & (g.p1[ax] >= 0) & (g.p1[ax] < bg.dim[ax]);
    return ok;
}

// First and last k of the segment inside [lo, hi] on one axis.
__host__ __device__ __forceinline__ void axis_window(int32_t p0, uint32_t a, uint32_t neg, uint32_t N, int32_t lo,
                                            int32_t hi, uint32_t& kin, uint32_t& kout) {
    if (a == 0) {
        bool in = p0 >= lo && p0 <= hi;
        kin = in ? 0u : kNever;
        kout = in ? N : 0u;
        return;
    }
    if (!neg) {
        // v = p0 + q, q from 0 to a.
        kin = p0 >= lo ? 0u : k_reach((uint32_t)(lo - p0), a, N, 0u);
        uint32_t e = hi >= p0 ? k_reach((uint32_t)(hi - p0 + 1), a, N, 0u) : 0u;
        kout = e == kNever ? N : e - 1u;
        if (hi < p0) kin = kNever;
    } else {
        // v = p0 - q.
        kin = p0 <= hi ? 0u : k_reach((uint32_t)(p0 - hi), a, N, 1u);
        uint32_t e = p0 >= lo ? k_reach((uint32_t)(p0 - lo + 1), a, N, 1u) : 0u;
        kout = e == kNever ? N : e - 1u;
        if (p0 < lo) kin = kNever;
    }
}

// k-window [klo, khi] (inclusive; klo > khi when empty) of a segment inside
// the box [lo, hi] (inclusive per axis).
__host__ __device__ __forceinline__ void box_window(const SegAxes& s, const int32_t lo[3], const int32_t hi[3],
                                                    uint32_t& klo, uint32_t& khi) {
    klo = 0;
    khi = s.N;
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t kin, kout;
        axis_window(s.p0[ax], s.a[ax], s.neg[ax], s.N, lo[ax], hi[ax], kin, kout);
        klo = kin > klo ? kin : klo;
        khi = kout < khi ? kout : khi;
    }
}

// Brick decomposition of a dx*dy*dz volume into bricks of 2^lg voxels per
// axis; false when the brick path cannot serve it (rows not whole words, or
// more bricks than one LDS histogram holds).
__host__ __device__ inline bool brick_geometry(int32_t dx, int32_t dy, int32_t dz, const int lg[3],
                                               BrickGeom& bg) {
    // Rows of whole words; end points of staged segments and pieces are
    // 16-bit.
    if (dx % 32 != 0 || lg[0] < 5 || dx > 16384 || dy > 16384 || dz > 16384) return false;
    const int32_t dim[3] = {dx, dy, dz};
    uint64_t nb = 1;
    for (int ax = 0; ax < 3; ++ax) {
        bg.dim[ax] = dim[ax];
        bg.lg[ax] = lg[ax];
        bg.nb[ax] = (dim[ax] + (1 << lg[ax]) - 1) >> lg[ax];
        nb *= (uint64_t)bg.nb[ax];
    }
    if (nb > (uint64_t)kMaxBricks) return false;
    bg.nbricks = (uint32_t)nb;
    return true;
}


// Work items of the fill.  A brick's records are the work of one workgroup,
// and a brick can hold far more than a workgroup's fair share of a launch
// (a small dense volume in a batch is a single brick of millions of
// voxels), which would leave one workgroup running long after the others.
// So a brick with more than T records, T = max(kSplitMinRecords,
// ceil(total / kSplitShares)), becomes ceil(records / T) items, each with
// an even part of its records, set in LDS by its own workgroup and ORed
// into the volume with device atomics (the scatter zeroes such a brick
// first in a cleared volume).  Since every cut brick holds more than
// T records, the items beyond one per brick number at most
// total / T <= kSplitShares, and so do the cut bricks.
constexpr uint32_t kSplitShares = 1024;
constexpr uint32_t kSplitMinRecords = 4096;
constexpr uint32_t kMaxExtraItems = kSplitShares;

__host__ __device__ inline uint64_t split_threshold(uint64_t total) {
    const uint64_t t = total / kSplitShares + (total % kSplitShares != 0u ? 1u : 0u);
    return t > kSplitMinRecords ? t : kSplitMinRecords;
}
__host__ __device__ inline uint32_t brick_items(uint32_t records, uint64_t T) {
    if (records <= T) return 1u;               // every brick when T >= 2^32
    return (records - 1u) / (uint32_t)T + 1u;  // ceil(records / T), T < records < 2^32
}
// Records [lo, hi) of item j of the k items of a brick whose records are
// [first, first + count).
__host__ __device__ inline void item_range(uint32_t first, uint32_t count, uint32_t j, uint32_t k, uint32_t& lo,
                                           uint32_t& hi) {
    lo = first + (uint32_t)((uint64_t)count * j / k);
    hi = first + (uint32_t)((uint64_t)count * (j + 1u) / k);
}

// The argument rules of a bit-volume scene (those of vox_segments_to_grid):
// n in [0, 2^31 - 2], segs non-null when n > 0 and 4-byte aligned, each side
// in [1, 2^20] with at most 2^38 voxels, grid non-null and 16-byte aligned,
// counts 4-byte aligned, flags within VOX_GRID_CLEAR | VOX_GRID_EUCLID.
__host__ __device__ inline bool scene_valid(const vox_scene& in) {
    const uintptr_t segs = (uintptr_t)in.segs, grid = (uintptr_t)in.grid, counts = (uintptr_t)in.counts;
    if (in.n < 0 || in.n > (int64_t(1) << 31) - 2) return false;
    if (in.n > 0 && segs == 0) return false;
    if ((segs & 3u) != 0 || grid == 0 || (grid & 15u) != 0 || (counts & 3u) != 0) return false;
    const int64_t lim = int64_t(1) << 20;
    if (in.dim_x < 1 || in.dim_y < 1 || in.dim_z < 1 || in.dim_x > lim || in.dim_y > lim || in.dim_z > lim)
        return false;
    if ((int64_t)in.dim_x * in.dim_y * in.dim_z > (int64_t(1) << 38)) return false;
    return (in.flags & ~(uint32_t)(VOX_GRID_CLEAR | VOX_GRID_EUCLID)) == 0;
}

// With the Euclidean N of eq. (1), the brick path needs N <= 16384 for every
// segment (the fill keeps error terms below 2N in biased 16-bit halves); an
// in-volume segment's N is at most the volume's diagonal, so the volume's
// diagonal decides.
__host__ __device__ inline bool euclid_bricks_ok(int32_t dx, int32_t dy, int32_t dz) {
    const int64_t sx = dx - 1, sy = dy - 1, sz = dz - 1;
    return sx * sx + sy * sy + sz * sz < (int64_t)16385 * 16385;
}

// One scene of a launch, as the plan kernel enters it in the table (bases
// left zero): the brick path serves it when its segment array is 8-byte
// aligned and its volume takes bricks of 2^lg (and, with the Euclidean N,
// when its diagonal is below 16385); otherwise it is flagged for the direct
// kernels.  False (and a direct entry
// with no segments) when the scene breaks an argument rule.
__host__ __device__ inline bool plan_scene(const vox_scene& in, const int32_t lg[3], int64_t segs_per_row,
                                           BrickScene& out) {
    const bool valid = scene_valid(in);
    out = BrickScene{};
    out.segs = reinterpret_cast<const int32_t*>(in.segs);
    out.counts = in.counts;
    out.grid = in.grid;
    out.n = valid ? in.n : 0;
    out.bg.dim[0] = in.dim_x;
    out.bg.dim[1] = in.dim_y;
    out.bg.dim[2] = in.dim_z;
    uint32_t f = 0;
    if (in.flags & VOX_GRID_CLEAR) f |= kSceneClear;
    if (in.flags & VOX_GRID_EUCLID) f |= kSceneEuclid;
    if (((uintptr_t)in.segs & 7u) == 0) f |= kSceneA8;
    const int lgi[3] = {lg[0], lg[1], lg[2]};
    BrickGeom bg;
    if (valid && (f & kSceneA8) && (!(f & kSceneEuclid) || euclid_bricks_ok(in.dim_x, in.dim_y, in.dim_z)) &&
        brick_geometry(in.dim_x, in.dim_y, in.dim_z, lgi, bg)) {
        out.bg = bg;
        out.rows = hist_rows(in.n, segs_per_row);
    } else {
        f |= kSceneDirect;
        out.rows = 0;
        out.bg.nbricks = 0;
    }
    out.flags = f;
    return valid;
}

}  // namespace vox

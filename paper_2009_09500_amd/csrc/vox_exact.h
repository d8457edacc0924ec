// Exact integer helpers of the brick path: brick walk of a segment and the
// k-window of a segment inside an axis interval.  Host and device, so the
// host-side checks exercise the very code the kernels run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
    uint64_t x = 2ull * N * m - N + neg;
    return div_ceil_u64(x, 2u * a);
}

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

// Walks the bricks of one in-volume segment in order, calling emit(brick id).
template <typename Emit>
__host__ __device__ __forceinline__ void walk_bricks(const SegAxes& s, const BrickGeom& bg, Emit emit) {
    int32_t b[3], bend[3];
    uint32_t kn[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        b[ax] = s.p0[ax] >> bg.lg[ax];
        bend[ax] = s.p1[ax] >> bg.lg[ax];
        kn[ax] = kNever;
        if (b[ax] != bend[ax]) {
            uint32_t m = s.neg[ax] ? (uint32_t)(s.p0[ax] - (b[ax] << bg.lg[ax]) + 1)
                                   : (uint32_t)(((b[ax] + 1) << bg.lg[ax]) - s.p0[ax]);
            kn[ax] = k_reach(m, s.a[ax], s.N, s.neg[ax]);
        }
    }
    while (true) {
        emit((uint32_t)((b[2] * bg.nb[1] + b[1]) * bg.nb[0] + b[0]));
        uint32_t km = kn[0] < kn[1] ? kn[0] : kn[1];
        km = km < kn[2] ? km : kn[2];
        if (km == kNever) break;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (kn[ax] == km) {
                b[ax] += s.neg[ax] ? -1 : 1;
                kn[ax] = kNever;
                if (b[ax] != bend[ax]) {
                    uint32_t m = s.neg[ax] ? (uint32_t)(s.p0[ax] - (b[ax] << bg.lg[ax]) + 1)
                                           : (uint32_t)(((b[ax] + 1) << bg.lg[ax]) - s.p0[ax]);
                    kn[ax] = k_reach(m, s.a[ax], s.N, s.neg[ax]);
                }
            }
        }
    }
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
inline bool brick_geometry(int32_t dx, int32_t dy, int32_t dz, const int lg[3], BrickGeom& bg) {
    if (dx % 32 != 0 || lg[0] < 5) return false;
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

}  // namespace vox

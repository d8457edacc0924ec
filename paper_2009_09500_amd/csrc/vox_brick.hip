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
// coordinate crosses a brick boundary.  With q(k) = floor((2 k a + N - neg)
// / 2N) the offset along an axis (a = |d|, neg = d < 0), the first k with
// q(k) >= m is ceil((2 N m - N + neg) / 2a) (for 1 <= m <= a; q never exceeds
// a).  That gives the piece list and each piece's k-range exactly.
//
// Pipeline (one stream, no host synchronisation):
//   init      status word and work counter to zero
//   hist      per segment: count N+1, range check, walk its bricks and count
//             pieces per brick in an LDS histogram; one histogram row per
//             workgroup
//   colscan   per brick, exclusive prefix of the rows over workgroups, and
//             the brick's piece total
//   base      exclusive scan of the brick totals -> bin offsets
//   scatter   the same walk again, appending segment ids into the bins
//   bricks    persistent workgroups take bricks from an atomic counter,
//             clip every piece to the brick, set the bits with LDS atomic OR
//             and flush the brick to the volume
#include "vox_device.h"
#include "vox_exact.h"
#include "vox_internal.h"

namespace vox {

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

template <bool kAligned8>
__global__ __launch_bounds__(kHistBlock) void k_brick_hist(const int32_t* __restrict__ segs, int64_t n,
                                                           BrickGeom bg, uint32_t* __restrict__ hist,
                                                           int32_t* __restrict__ counts,
                                                           int32_t* __restrict__ status) {
    extern __shared__ uint32_t lh[];
    const uint32_t NB = bg.nbricks;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) lh[b] = 0;
    __syncthreads();
    int64_t lo, hi;
    seg_range(n, blockIdx.x, gridDim.x, lo, hi);
    bool bad = false;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kHistBlock) {
        Seg g = load_seg<kAligned8>(segs, i);
        if (counts) {
            int64_t c = seg_length(g) + 1;
            counts[i] = (int32_t)(c > 0x7FFFFFFFll ? 0x7FFFFFFFll : c);
        }
        if (!in_volume(g, bg)) {
            bad = true;
            continue;
        }
        SegAxes s = seg_axes(g);
        walk_bricks(s, bg, [&](uint32_t b) { atomicAdd(&lh[b], 1u); });
    }
    if (bad) atomicOr(status, kStatusOutOfRange);
    __syncthreads();
    uint32_t* row = hist + (size_t)blockIdx.x * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) row[b] = lh[b];
}

// Thread per brick: exclusive prefix of hist[g][b] over g (in place) and the
// brick's total.
__global__ __launch_bounds__(256) void k_brick_colscan(uint32_t* __restrict__ hist, int G, uint32_t NB,
                                                       uint32_t* __restrict__ totals) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= NB) return;
    uint32_t run = 0;
    for (int g = 0; g < G; ++g) {
        uint32_t* p = hist + (size_t)g * NB + b;
        uint32_t v = *p;
        *p = run;
        run += v;
    }
    totals[b] = run;
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

template <bool kAligned8>
__global__ __launch_bounds__(kHistBlock) void k_brick_scatter(const int32_t* __restrict__ segs, int64_t n,
                                                              BrickGeom bg, const uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ bin_base,
                                                              uint32_t* __restrict__ ids) {
    extern __shared__ uint32_t cur[];
    const uint32_t NB = bg.nbricks;
    const uint32_t* row = hist + (size_t)blockIdx.x * NB;
    for (uint32_t b = threadIdx.x; b < NB; b += kHistBlock) cur[b] = bin_base[b] + row[b];
    __syncthreads();
    int64_t lo, hi;
    seg_range(n, blockIdx.x, gridDim.x, lo, hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kHistBlock) {
        Seg g = load_seg<kAligned8>(segs, i);
        if (!in_volume(g, bg)) continue;
        SegAxes s = seg_axes(g);
        walk_bricks(s, bg, [&](uint32_t b) {
            uint32_t pos = atomicAdd(&cur[b], 1u);
            ids[pos] = (uint32_t)i;
        });
    }
}

// Piece of a segment inside the current brick, staged in LDS.
struct Piece {
    int32_t p0[3];
    int32_t d[3];
    uint32_t klo, khi;  // inclusive; klo > khi = empty
};

template <int kBlock, int kBatch, int kChunk, bool kAligned8, bool kVec4>
__global__ __launch_bounds__(kBlock) void k_brick_fill(const int32_t* __restrict__ segs, BrickGeom bg,
                                                       const uint32_t* __restrict__ ids,
                                                       const uint32_t* __restrict__ bin_base,
                                                       uint32_t* __restrict__ grid, uint32_t clear,
                                                       uint32_t* __restrict__ work_counter) {
    static_assert(kBatch == kBlock, "one piece per thread and batch");
    extern __shared__ __align__(16) uint32_t brick[];
    __shared__ Piece pieces[kBatch];
    __shared__ uint32_t coff[kBatch + 1];
    __shared__ uint32_t red[kBlock / kWave];
    __shared__ uint32_t item_s;

    const uint32_t NB = bg.nbricks;
    const int BXw = 1 << (bg.lg[0] - 5);       // words per brick row
    const uint32_t brick_words = (uint32_t)BXw << (bg.lg[1] + bg.lg[2]);
    const int64_t row_words = (int64_t)bg.dim[0] >> 5;

    while (true) {
        if (threadIdx.x == 0) item_s = atomicAdd(work_counter, 1u);
        __syncthreads();
        const uint32_t item = item_s;
        if (item >= NB) break;
        const uint32_t b = item;
        const int bx = (int)(b % (uint32_t)bg.nb[0]);
        const int by = (int)((b / (uint32_t)bg.nb[0]) % (uint32_t)bg.nb[1]);
        const int bz = (int)(b / ((uint32_t)bg.nb[0] * (uint32_t)bg.nb[1]));
        const int32_t org[3] = {bx << bg.lg[0], by << bg.lg[1], bz << bg.lg[2]};
        int32_t ext[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            int32_t e = bg.dim[ax] - org[ax];
            ext[ax] = e < (1 << bg.lg[ax]) ? e : (1 << bg.lg[ax]);
        }

        for (uint32_t w = threadIdx.x; w < brick_words; w += kBlock) brick[w] = 0u;

        const uint32_t p_lo = bin_base[b], p_hi = bin_base[b + 1];
        for (uint32_t p0 = p_lo; p0 < p_hi; p0 += kBatch) {
            __syncthreads();  // brick cleared / previous batch consumed
            uint32_t nch = 0;
            for (uint32_t t = threadIdx.x; t < kBatch; t += kBlock) {
                Piece pc;
                pc.klo = 1u;
                pc.khi = 0u;
                uint32_t chunks = 0;
                if (p0 + t < p_hi) {
                    const uint32_t i = ids[p0 + t];
                    Seg g = load_seg<kAligned8>(segs, (int64_t)i);
                    SegAxes s = seg_axes(g);
                    uint32_t klo = 0, khi = s.N;
                    if (s.N > 0) {
                        const int32_t hi3[3] = {org[0] + ext[0] - 1, org[1] + ext[1] - 1, org[2] + ext[2] - 1};
                        box_window(s, org, hi3, klo, khi);
                    }
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        pc.p0[ax] = s.p0[ax];
                        pc.d[ax] = s.p1[ax] - s.p0[ax];
                    }
                    pc.klo = klo;
                    pc.khi = khi;
                    if (klo <= khi) chunks = (khi - klo) / kChunk + 1;
                }
                pieces[t] = pc;
                // kBatch == kBlock: one piece per thread.
                nch = chunks;
            }
            uint32_t tot;
            uint32_t ex = block_exclusive_sum<kBlock>(nch, red, tot);
            if (threadIdx.x < kBatch) coff[threadIdx.x] = ex;
            if (threadIdx.x == 0) coff[kBatch] = tot;
            __syncthreads();

            for (uint32_t c = threadIdx.x; c < tot; c += kBlock) {
                // Piece of chunk c: largest j with coff[j] <= c.
                int lo = 0, hi = kBatch - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (coff[mid] <= c) lo = mid; else hi = mid - 1;
                }
                const Piece pc = pieces[lo];
                const uint32_t k0 = pc.klo + (c - coff[lo]) * kChunk;
                const uint32_t k1 = k0 + kChunk - 1 < pc.khi ? k0 + kChunk - 1 : pc.khi;
                uint32_t a[3], neg[3], N = 0;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    neg[ax] = pc.d[ax] < 0;
                    a[ax] = (uint32_t)(pc.d[ax] < 0 ? -pc.d[ax] : pc.d[ax]);
                    N = a[ax] > N ? a[ax] : N;
                }
                // Voxel k0 and the stepping state of the two minor axes.
                const int m = a[0] == N ? 0 : (a[1] == N ? 1 : 2);
                const int32_t stride[3] = {1, 1 << bg.lg[0], 1 << (bg.lg[0] + bg.lg[1])};
                int32_t idx = 0;
                int32_t e[3], step[3];
                uint32_t two_a[3];
                const uint32_t two_n = 2u * N;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    uint32_t q = 0, r = 0;
                    if (N > 0) divmod_u64(2ull * k0 * a[ax] + N - neg[ax], two_n, q, r);
                    int32_t v = pc.p0[ax] + (neg[ax] ? -(int32_t)q : (int32_t)q);
                    idx += (v - org[ax]) * stride[ax];
                    e[ax] = (int32_t)r - (int32_t)two_n;   // in [-2N, 0)
                    two_a[ax] = 2u * a[ax];
                    step[ax] = neg[ax] ? -stride[ax] : stride[ax];
                }
                const int i1 = m == 0 ? 1 : 0;
                const int i2 = m == 2 ? 1 : 2;
                const int32_t sm = step[m], s1 = step[i1], s2 = step[i2];
                int32_t e1 = e[i1], e2 = e[i2];
                const int32_t t1 = (int32_t)two_a[i1], t2 = (int32_t)two_a[i2];
                const int32_t tn = (int32_t)two_n;
                const int len = (int)(k1 - k0) + 1;
#pragma unroll 4
                for (int k = 0; k < len; ++k) {
                    atomicOr(&brick[(uint32_t)idx >> 5], 1u << ((uint32_t)idx & 31u));
                    idx += sm;
                    e1 += t1;
                    if (e1 >= 0) { e1 -= tn; idx += s1; }
                    e2 += t2;
                    if (e2 >= 0) { e2 -= tn; idx += s2; }
                }
            }
        }
        __syncthreads();

        // Flush: brick row (y, z) -> volume words.  The owner writes every word
        // of its brick, so a clearing call needs no other pass.
        const int xw0 = org[0] >> 5;
        const int xws = ext[0] >> 5;
        const int rows = ext[1] * ext[2];
        if (kVec4) {
            // Rows of exactly 4 words, 16-byte aligned in the volume.
            for (int r = threadIdx.x; r < rows; r += kBlock) {
                const int y = r % ext[1], z = r / ext[1];
                const uint4 v = *reinterpret_cast<const uint4*>(&brick[((uint32_t)z << bg.lg[1] | (uint32_t)y) * 4u]);
                uint4* dst = reinterpret_cast<uint4*>(
                    grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words + xw0);
                if (clear) {
                    __builtin_nontemporal_store(v.x, &dst->x);
                    __builtin_nontemporal_store(v.y, &dst->y);
                    __builtin_nontemporal_store(v.z, &dst->z);
                    __builtin_nontemporal_store(v.w, &dst->w);
                } else {
                    uint4 o = *dst;
                    *dst = make_uint4(o.x | v.x, o.y | v.y, o.z | v.z, o.w | v.w);
                }
            }
        } else {
            const int total = rows * xws;
            for (int t = threadIdx.x; t < total; t += kBlock) {
                const int xw = t % xws, r = t / xws;
                const int y = r % ext[1], z = r / ext[1];
                const uint32_t v = brick[(((uint32_t)z << bg.lg[1]) | (uint32_t)y) * (uint32_t)BXw + xw];
                uint32_t* dst = grid + ((int64_t)(org[2] + z) * bg.dim[1] + (org[1] + y)) * row_words + xw0 + xw;
                if (clear) *dst = v;
                else *dst |= v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- host side

constexpr int kFillBlock = 512;
constexpr int kFillBatch = 512;
constexpr int kFillChunk = 16;

void default_brick_lg(int32_t dx, int32_t dy, int32_t dz, int lg[3]) {
    (void)dx; (void)dy; (void)dz;
    lg[0] = 7;  // 128
    lg[1] = 7;  // 128
    lg[2] = 6;  // 64
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
    b += align_up((size_t)max_pieces(n, bg) * sizeof(uint32_t));       // ids
    return b;
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
    uint32_t* ids = reinterpret_cast<uint32_t*>(p);
    const size_t hist_lds = (size_t)bg.nbricks * sizeof(uint32_t);
    hipError_t e;
    {
        KernelTimer t("brick_init", stream);
        k_brick_init<<<1, 64, 0, stream>>>(status, counter);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
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
        k_brick_colscan<<<(bg.nbricks + 255) / 256, 256, 0, stream>>>(hist, G, bg.nbricks, totals);
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
            k_brick_scatter<true><<<G, kHistBlock, hist_lds, stream>>>(segs, n, bg, hist, bin_base, ids);
        else
            k_brick_scatter<false><<<G, kHistBlock, hist_lds, stream>>>(segs, n, bg, hist, bin_base, ids);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;

    const size_t brick_lds = ((size_t)1 << (bg.lg[0] + bg.lg[1] + bg.lg[2])) / 8;
    const bool vec4 = bg.lg[0] == 7 && (bg.dim[0] % 128) == 0;
    int dev = 0;
    hipGetDevice(&dev);
    int cus = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int wgs = cus > 0 ? cus : 256;
    if ((uint32_t)wgs > bg.nbricks) wgs = (int)bg.nbricks;
    const uint32_t clear = (flags & 1u) ? 1u : 0u;
    KernelTimer t("brick_fill", stream);
#define VOX_FILL(A8, V4)                                                                              \
    do {                                                                                              \
        auto kern = k_brick_fill<kFillBlock, kFillBatch, kFillChunk, A8, V4>;                         \
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,           \
                            (int)brick_lds);                                                          \
        kern<<<wgs, kFillBlock, brick_lds, stream>>>(segs, bg, ids, bin_base, grid, clear, counter);  \
    } while (0)
    if (aligned8) {
        if (vec4) VOX_FILL(true, true); else VOX_FILL(true, false);
    } else {
        if (vec4) VOX_FILL(false, true); else VOX_FILL(false, false);
    }
#undef VOX_FILL
    return hipGetLastError();
}

}  // namespace vox

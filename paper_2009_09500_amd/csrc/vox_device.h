// Device-side building blocks shared by the voxelization kernels (gfx950,
// wave64).  Internal to the HIP library; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vox {

constexpr int kWave = 64;

// One segment as read from the caller's AoS array: start point and end
// point.  Loaded with three 8-byte loads when the array is 8-byte aligned
// (every torch allocation is), else six 4-byte loads.
struct Seg {
    int32_t p0[3];
    int32_t p1[3];
};

template <bool kAligned8>
__device__ __forceinline__ Seg load_seg(const int32_t* __restrict__ segs, int64_t i) {
    Seg s;
    const int32_t* p = segs + 6 * i;
    if constexpr (kAligned8) {
        const int2* q = reinterpret_cast<const int2*>(p);
        int2 a = q[0], b = q[1], c = q[2];
        s.p0[0] = a.x; s.p0[1] = a.y; s.p0[2] = b.x;
        s.p1[0] = b.y; s.p1[1] = c.x; s.p1[2] = c.y;
    } else {
        s.p0[0] = p[0]; s.p0[1] = p[1]; s.p0[2] = p[2];
        s.p1[0] = p[3]; s.p1[1] = p[4]; s.p1[2] = p[5];
    }
    return s;
}

// Chebyshev length N = max_a |p1_a - p0_a| in 64 bits (int32 inputs may
// differ by up to 2^32 - 1).
__device__ __forceinline__ int64_t seg_length(const Seg& s) {
    int64_t n = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int64_t d = (int64_t)s.p1[a] - (int64_t)s.p0[a];
        d = d < 0 ? -d : d;
        n = d > n ? d : n;
    }
    return n;
}

// Euclidean length of the paper's eq. (1), N_e = int(|p1 - p0|): the integer
// square root of dx^2 + dy^2 + dz^2.  For end points within 2^31 of each
// other the sum stays below 2^64 (and below 2^53, where the double square
// root is within one of the result, for every input the library accepts:
// int16 lists, volumes up to 2^20 a side); the integer corrections make it
// exact.
__device__ __forceinline__ uint32_t euclid_length(const Seg& s) {
    uint64_t ss = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t d = (int64_t)s.p1[a] - (int64_t)s.p0[a];
        ss += (uint64_t)(d * d);
    }
    uint64_t r = (uint64_t)sqrt((double)ss);
    while (r * r > ss) --r;
    while ((r + 1) * (r + 1) <= ss) ++r;
    return (uint32_t)r;
}

__device__ __forceinline__ bool in_int16(const Seg& s) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ok &= (s.p0[a] >= -32768) & (s.p0[a] <= 32767) & (s.p1[a] >= -32768) & (s.p1[a] <= 32767);
    }
    return ok;
}

// Domain of the int32 lists: every |p1_a - p0_a| < 2^30, so N < 2^30 and the
// stepping's remainders (below 2N) plus their increments (at most 2N) stay
// below 2^32.
__device__ __forceinline__ bool span_below_2p30(const Seg& s) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t d = (int64_t)s.p1[a] - (int64_t)s.p0[a];
        ok &= (d < (int64_t(1) << 30)) & (d > -(int64_t(1) << 30));
    }
    return ok;
}

// Exact incremental evaluation of voxel k of a segment along one axis.
//
// With N the Chebyshev length, d = p1 - p0 and a = |d|, the coordinate is
//   d >= 0:  p0 + floor((2 k a + N) / 2N)
//   d <  0:  p0 - floor((2 k a + N - 1) / 2N)
// (the second is the first with d negated and floor(x + 1/2) mirrored).
// Keeping q = numerator / 2N and r = numerator mod 2N, k -> k + 1 adds 2a
// to the numerator; as 2a <= 2N the quotient grows by at most one:
//   r += 2a;  if (r >= 2N) { r -= 2N; ++q; }
// This is Bresenham's error term; it reproduces the division exactly.
// floor(x / y) and remainder for x < 2^31, 2 <= y < 2^16 and quotients
// below 2^15, from a hardware reciprocal estimate corrected in integers
// (exact).  rcp_down(y) is the reciprocal (within one ulp) scaled by
// 1 - 2^-20: x (rounded once in float) times it is below x / y by a relative
// 2^-20 +- 2^-22, so its integer part is the quotient or one less (the
// quotient is below 2^15, so the shortfall stays below one), and one
// upward correction makes it exact.
//
// The scaling and the division are host+device so that a host program can
// run them with the reciprocal estimate off by -1, 0 and +1 ulp (the
// hardware's stated error), checking the exactness claim on the CPU.
__host__ __device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return (a & 0xFFFFFFu) * (b & 0xFFFFFFu);
#endif
}

__host__ __device__ __forceinline__ float rcp_bias_down(float rcp) { return rcp * (1.0f - 0x1p-20f); }

__device__ __forceinline__ float rcp_down(uint32_t y) {
    return rcp_bias_down(__builtin_amdgcn_rcpf((float)y));
}

__host__ __device__ __forceinline__ void divmod_down(uint32_t x, uint32_t y, float rcpd, uint32_t& q,
                                                     uint32_t& r) {
    uint32_t qq = (uint32_t)((float)x * rcpd);
    uint32_t rr = x - mul_u24(qq, y);
    if (rr >= y) {
        ++qq;
        rr -= y;
    }
    q = qq;
    r = rr;
}

struct AxisStep {
    uint32_t q, r, two_a;
};

// Quotients and remainders of (2 k a + N - neg) / 2N, per axis, for N >= 1
// and k <= N.  Up to N = 32767 the numerators stay below 2^31 and the
// quotients at most a < 2^15, so one reciprocal serves all three axes
// (divmod_down); beyond that, 64-bit divisions.
__device__ __forceinline__ void axis_init3(const uint32_t a[3], const uint32_t neg[3], uint32_t N, uint32_t k,
                                           AxisStep st[3]) {
    const uint32_t two_n = 2u * N;
    if (N <= 32767u) {
        const float rcpd = rcp_down(two_n);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            st[ax].two_a = 2u * a[ax];
            divmod_down(2u * k * a[ax] + N - neg[ax], two_n, rcpd, st[ax].q, st[ax].r);
        }
    } else {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            st[ax].two_a = 2u * a[ax];
            const uint64_t num = 2ull * k * a[ax] + N - neg[ax];
            const uint64_t q = num / two_n;
            st[ax].q = (uint32_t)q;
            st[ax].r = (uint32_t)(num - q * two_n);
        }
    }
}

__device__ __forceinline__ void axis_step(AxisStep& st, uint32_t two_n) {
    st.r += st.two_a;
    bool c = st.r >= two_n;
    st.r = c ? st.r - two_n : st.r;
    st.q += c ? 1u : 0u;
}

// Lanes per segment where a wave takes several segments at once, one sample
// per lane (a power of two dividing 64).
constexpr int kSampleLanes = 16;

// The samples of one segment as taken by one of its kSampleLanes lanes:
// samples k, k + kSampleLanes, k + 2 kSampleLanes, ...  q_a and r_a are the
// quotient and remainder of (2 k a + N - neg) / 2N.  Because a <= N, the
// step from k - 1 to k moves axis a (by one) exactly when it carries, that is
// when r_a(k) < 2a, so a lane knows on its own whether its sample starts a
// new voxel.  start() divides once (one reciprocal for all three axes up to
// N = 32767, where the numerators stay below 2^31 and the quotients below
// 2^15; 64-bit divisions beyond); next() moves on by kSampleLanes samples
// with the per-segment stride (dq, dr) = divmod(kSampleLanes * 2a, 2N), one
// add and one correction per axis.  Both return whether the sample moved
// (true at k = 0).  Samples past N get meaningless values.
struct SampleAt {
    uint32_t two_a[3], num0[3], dq[3], dr[3];
    uint32_t q[3], r[3];
    bool neg[3];
    uint32_t N, two_n;

    __device__ __forceinline__ void init(const Seg& g, uint32_t n) {
        N = n;
        two_n = 2u * n;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int32_t d = g.p1[ax] - g.p0[ax];
            neg[ax] = d < 0;
            two_a[ax] = 2u * (uint32_t)(d < 0 ? -d : d);
            num0[ax] = n - (neg[ax] ? 1u : 0u);
        }
    }

    __device__ __forceinline__ bool start(uint32_t k) {
        bool moved = k == 0;
        if (N == 0) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) q[ax] = r[ax] = dq[ax] = dr[ax] = 0;
        } else if (N <= 32767u) {
            const float rcpd = rcp_down(two_n);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                divmod_down(__umul24(k, two_a[ax]) + num0[ax], two_n, rcpd, q[ax], r[ax]);
                divmod_down(kSampleLanes * two_a[ax], two_n, rcpd, dq[ax], dr[ax]);
                moved |= r[ax] < two_a[ax];
            }
        } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const uint64_t num = (uint64_t)k * two_a[ax] + num0[ax];
                q[ax] = (uint32_t)(num / two_n);
                r[ax] = (uint32_t)(num - (uint64_t)q[ax] * two_n);
                const uint32_t s = kSampleLanes * two_a[ax];
                dq[ax] = s / two_n;
                dr[ax] = s - dq[ax] * two_n;
                moved |= r[ax] < two_a[ax];
            }
        }
        return moved;
    }

    __device__ __forceinline__ bool next() {
        bool moved = false;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const uint32_t t = r[ax] + dr[ax];
            const bool c = t >= two_n;
            r[ax] = c ? t - two_n : t;
            q[ax] += dq[ax] + (c ? 1u : 0u);
            moved |= r[ax] < two_a[ax];
        }
        return moved;
    }

    __device__ __forceinline__ int32_t coord(const Seg& g, int ax) const {
        return g.p0[ax] + (neg[ax] ? -(int32_t)q[ax] : (int32_t)q[ax]);
    }
};

// ------------------------------------------------------------ block scans

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Inclusive sum over the 64 lanes of a wave with DPP moves (rows of 16:
// shifts by 1, 2, 4, 8; then row 15 broadcast into rows 1 and 3, lane 31
// into rows 2 and 3).  All lanes must be active.
__device__ __forceinline__ uint32_t wave_inclusive_sum_dpp(uint32_t x) {
    uint32_t s = x;
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x111, 0xf, 0xf, true);  // row_shr:1
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x112, 0xf, 0xf, true);  // row_shr:2
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x114, 0xf, 0xf, true);  // row_shr:4
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x118, 0xf, 0xf, true);  // row_shr:8
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x142, 0xa, 0xf, false); // row_bcast:15
    s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x143, 0xc, 0xf, false); // row_bcast:31
    return s;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Exclusive prefix sum over the block (one value per thread, thread order).
// `lds` needs kBlock/64 entries; returns the block total in `total`.
template <int kBlock, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* lds, T& total) {
    constexpr int kWaves = kBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    T incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) lds[w] = incl;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        T x = lds[i];
        pre += (i < w) ? x : T(0);
        tot += x;
    }
    __syncthreads();
    total = tot;
    return pre + incl - v;
}

template <int kBlock, typename T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
    constexpr int kWaves = kBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) lds[w] = v;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) tot += lds[i];
    __syncthreads();
    return tot;
}

}  // namespace vox

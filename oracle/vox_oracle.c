/*
 * CPU oracle for parametric voxelization of 3D line segments.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, single-threaded,
 * obviously-correct statement of what the HIP path must produce.  It shares
 * no code, header, table or helper with the HIP library; only the tests, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * The method (arXiv 2009.09500, Section 3):
 *   - a point of segment SE is G = S + (E - S) t, 0 <= t <= 1 (unnumbered
 *     equation opening Section 3);
 *   - with t_k = k / N the sample points are G_k = S + W k, W = (E - S) / N,
 *     k = 0, 1, ..., N (eq. (2)-(3));
 *   - the algorithm of Fig. 3 takes, for every k, the voxel that contains
 *     G_k and emits the voxels as the array V^(k).
 *
 * Readings fixed where the paper is silent or inconsistent:
 *   - N is the Chebyshev length max(|dx|,|dy|,|dz|) (the paper's eq. (1)
 *     uses the integer part of the Euclidean length);
 *   - k runs 0..N as in eq. (2)-(3), not 1..N as printed in Fig. 3, so both
 *     end points are emitted and a segment has N + 1 voxels;
 *   - voxel centres sit at integer coordinates and the voxel containing a
 *     coordinate x is floor(x + 1/2) (round half up), which for
 *     x = P0 + k d / N is exactly P0 + floor((2 k d + N) / (2 N));
 *   - S == E (N == 0) gives the single voxel S;
 *   - segments keep input order and voxels run from S to E.
 *
 * All arithmetic is int64: for int32 end points |d| < 2^32, so 2 k d + N
 * stays far below 2^63.
 *
 * A second set of functions (vox_oracle_*_euclid, at the end) states the
 * paper's literal variant with the Euclidean N of eq. (1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* floor(a / b) for b > 0, rounding toward minus infinity. */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    int64_t r = a % b;
    if (r != 0 && a < 0)
        q -= 1;
    return q;
}

static int64_t abs64(int64_t v) { return v < 0 ? -v : v; }

/* N = max(|dx|,|dy|,|dz|) of one segment (Fig. 3, "Defining N"). */
int64_t vox_oracle_length(const int32_t *seg)
{
    int64_t n = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t d = abs64((int64_t)seg[3 + a] - (int64_t)seg[a]);
        if (d > n)
            n = d;
    }
    return n;
}

/* Voxel k of a segment: P0 + round_half_up(k * (P1 - P0) / N), eq. (3). */
void vox_oracle_voxel(const int32_t *seg, int64_t k, int64_t out[3])
{
    int64_t N = vox_oracle_length(seg);
    for (int a = 0; a < 3; ++a) {
        int64_t p0 = seg[a];
        int64_t d = (int64_t)seg[3 + a] - p0;
        if (N == 0)
            out[a] = p0;
        else
            out[a] = p0 + floor_div(2 * k * d + N, 2 * N);
    }
}

/* counts[i] = N_i + 1, the number of voxels of segment i. */
void vox_oracle_counts(const int32_t *segs, int64_t n, int32_t *counts)
{
    for (int64_t i = 0; i < n; ++i)
        counts[i] = (int32_t)(vox_oracle_length(segs + 6 * i) + 1);
}

/* offsets[i] = sum_{j<i} (N_j + 1), offsets[n] = total; returns total. */
int64_t vox_oracle_offsets(const int32_t *segs, int64_t n, int64_t *offsets)
{
    int64_t run = 0;
    for (int64_t i = 0; i < n; ++i) {
        offsets[i] = run;
        run += vox_oracle_length(segs + 6 * i) + 1;
    }
    offsets[n] = run;
    return run;
}

/* Concatenated voxel lists, x,y,z interleaved as int16, segments in input
 * order, voxels from S to E.  Writes nothing and returns -1 if the total
 * exceeds `capacity` voxels or a coordinate leaves the int16 range;
 * otherwise returns the total. */
int64_t vox_oracle_list(const int32_t *segs, int64_t n, int16_t *out, int64_t capacity)
{
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        for (int a = 0; a < 6; ++a)
            if (s[a] < -32768 || s[a] > 32767)
                return -1;
        total += vox_oracle_length(s) + 1;
    }
    if (total > capacity)
        return -1;
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        int64_t N = vox_oracle_length(s);
        for (int64_t k = 0; k <= N; ++k) {
            int64_t v[3];
            vox_oracle_voxel(s, k, v);
            out[3 * j + 0] = (int16_t)v[0];
            out[3 * j + 1] = (int16_t)v[1];
            out[3 * j + 2] = (int16_t)v[2];
            ++j;
        }
    }
    return total;
}

/* The same lists with int32 coordinates, for segments whose voxels leave
 * the int16 range (the paper's longest single segments have 10^6 voxels,
 * Section 5).  Domain: every |P1_a - P0_a| < 2^30.  Writes nothing and
 * returns -1 if a segment is outside it or the total exceeds `capacity`
 * voxels; otherwise returns the total. */
int64_t vox_oracle_list32(const int32_t *segs, int64_t n, int32_t *out, int64_t capacity)
{
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        for (int a = 0; a < 3; ++a)
            if (abs64((int64_t)s[3 + a] - (int64_t)s[a]) >= ((int64_t)1 << 30))
                return -1;
        total += vox_oracle_length(s) + 1;
    }
    if (total > capacity)
        return -1;
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        int64_t N = vox_oracle_length(s);
        for (int64_t k = 0; k <= N; ++k) {
            int64_t v[3];
            vox_oracle_voxel(s, k, v);
            out[3 * j + 0] = (int32_t)v[0];
            out[3 * j + 1] = (int32_t)v[1];
            out[3 * j + 2] = (int32_t)v[2];
            ++j;
        }
    }
    return total;
}

/* Packed occupancy bit-volume of dims dx*dy*dz: voxel (x,y,z) is bit
 * b = (z*dy + y)*dx + x, stored in 32-bit word b/32 at bit b%32 (LSB first).
 * With clear != 0 the volume starts empty, otherwise bits are ORed into the
 * existing words.  Returns -1 (after the optional clear, writing no voxel) if
 * an end point lies outside the volume, else the number of voxels set
 * (duplicates counted). */
int64_t vox_oracle_grid(const int32_t *segs, int64_t n, int32_t dx, int32_t dy,
                        int32_t dz, uint32_t *grid, int clear)
{
    int64_t nbits = (int64_t)dx * dy * dz;
    int64_t nwords = (nbits + 31) / 32;
    if (clear)
        memset(grid, 0, (size_t)nwords * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        for (int e = 0; e < 2; ++e) {
            const int32_t *p = s + 3 * e;
            if (p[0] < 0 || p[0] >= dx || p[1] < 0 || p[1] >= dy || p[2] < 0 || p[2] >= dz)
                return -1;
        }
    }
    int64_t set = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        int64_t N = vox_oracle_length(s);
        for (int64_t k = 0; k <= N; ++k) {
            int64_t v[3];
            vox_oracle_voxel(s, k, v);
            int64_t b = (v[2] * dy + v[1]) * dx + v[0];
            grid[b / 32] |= (uint32_t)1u << (b % 32);
            ++set;
        }
    }
    return set;
}

/* ------------------------------------------------------------------------
 * Euclidean-length variant: the paper's own eq. (1) for N.
 *
 *   - N_e = int(|E - S|), the integer part of the Euclidean length, computed
 *     exactly as the integer square root of dx^2 + dy^2 + dz^2;
 *   - samples G_k = S + k (E - S) / N_e, k = 0..N_e (eq. (2)-(3) with this
 *     N), each mapped to the voxel containing it by the same round-half-up
 *     rule as above: P0 + floor((2 k d + N_e) / (2 N_e));
 *   - since |d_a| <= N_e, neighbouring samples may fall in one voxel: a
 *     sample in the same voxel as the sample before it adds no voxel
 *     (consecutive duplicates removed);
 *   - S == E (N_e == 0) gives the single voxel S.
 * Defined for end points whose differences stay below 2^31 in magnitude
 * (int16 lists, volumes up to 2^20 voxels a side); sums of squares then fit
 * 64 bits and every product below fits int64.
 * ------------------------------------------------------------------------ */

/* Largest r with r * r <= v, by bisection over [0, 2^32). */
static uint64_t isqrt_u64(uint64_t v)
{
    uint64_t lo = 0, hi = 4294967296ull;
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (mid * mid <= v)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

/* N_e = int(|E - S|) of one segment (eq. (1)). */
int64_t vox_oracle_length_euclid(const int32_t *seg)
{
    uint64_t ss = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t d = (int64_t)seg[3 + a] - (int64_t)seg[a];
        ss += (uint64_t)(d * d);
    }
    return (int64_t)isqrt_u64(ss);
}

/* Voxel of sample k (0 <= k <= N_e), before duplicates are removed. */
void vox_oracle_sample_euclid(const int32_t *seg, int64_t k, int64_t out[3])
{
    int64_t N = vox_oracle_length_euclid(seg);
    for (int a = 0; a < 3; ++a) {
        int64_t p0 = seg[a];
        int64_t d = (int64_t)seg[3 + a] - p0;
        if (N == 0)
            out[a] = p0;
        else
            out[a] = p0 + floor_div(2 * k * d + N, 2 * N);
    }
}

/* Visits the voxels of one segment (duplicates removed) in order; writes
 * them to out (3 int64 each) when out is not NULL; returns their number. */
static int64_t euclid_voxels(const int32_t *seg, int64_t *out)
{
    int64_t N = vox_oracle_length_euclid(seg);
    int64_t prev[3] = {0, 0, 0};
    int64_t m = 0;
    for (int64_t k = 0; k <= N; ++k) {
        int64_t v[3];
        vox_oracle_sample_euclid(seg, k, v);
        if (k > 0 && v[0] == prev[0] && v[1] == prev[1] && v[2] == prev[2])
            continue;
        if (out) {
            out[3 * m + 0] = v[0];
            out[3 * m + 1] = v[1];
            out[3 * m + 2] = v[2];
        }
        prev[0] = v[0];
        prev[1] = v[1];
        prev[2] = v[2];
        ++m;
    }
    return m;
}

/* counts[i] = number of voxels of segment i (duplicates removed). */
void vox_oracle_counts_euclid(const int32_t *segs, int64_t n, int32_t *counts)
{
    for (int64_t i = 0; i < n; ++i)
        counts[i] = (int32_t)euclid_voxels(segs + 6 * i, NULL);
}

/* offsets[i] = sum_{j<i} counts[j], offsets[n] = total; returns total. */
int64_t vox_oracle_offsets_euclid(const int32_t *segs, int64_t n, int64_t *offsets)
{
    int64_t run = 0;
    for (int64_t i = 0; i < n; ++i) {
        offsets[i] = run;
        run += euclid_voxels(segs + 6 * i, NULL);
    }
    offsets[n] = run;
    return run;
}

/* Concatenated lists as vox_oracle_list, with the Euclidean N and
 * consecutive duplicates removed. */
int64_t vox_oracle_list_euclid(const int32_t *segs, int64_t n, int16_t *out, int64_t capacity)
{
    int64_t total = 0;
    int64_t longest = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        for (int a = 0; a < 6; ++a)
            if (s[a] < -32768 || s[a] > 32767)
                return -1;
        int64_t c = euclid_voxels(s, NULL);
        total += c;
        if (c > longest)
            longest = c;
    }
    if (total > capacity)
        return -1;
    int64_t *buf = (int64_t *)malloc((size_t)(longest > 0 ? longest : 1) * 3 * sizeof(int64_t));
    if (!buf)
        return -1;
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = euclid_voxels(segs + 6 * i, buf);
        for (int64_t m = 0; m < c; ++m, ++j) {
            out[3 * j + 0] = (int16_t)buf[3 * m + 0];
            out[3 * j + 1] = (int16_t)buf[3 * m + 1];
            out[3 * j + 2] = (int16_t)buf[3 * m + 2];
        }
    }
    free(buf);
    return total;
}

/* Bit-volume as vox_oracle_grid with the Euclidean N (duplicates set the
 * same bit; the count returned is of voxels after removing consecutive
 * duplicates). */
int64_t vox_oracle_grid_euclid(const int32_t *segs, int64_t n, int32_t dx, int32_t dy,
                               int32_t dz, uint32_t *grid, int clear)
{
    int64_t nbits = (int64_t)dx * dy * dz;
    int64_t nwords = (nbits + 31) / 32;
    if (clear)
        memset(grid, 0, (size_t)nwords * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        for (int e = 0; e < 2; ++e) {
            const int32_t *p = s + 3 * e;
            if (p[0] < 0 || p[0] >= dx || p[1] < 0 || p[1] >= dy || p[2] < 0 || p[2] >= dz)
                return -1;
        }
    }
    int64_t set = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *s = segs + 6 * i;
        int64_t N = vox_oracle_length_euclid(s);
        for (int64_t k = 0; k <= N; ++k) {
            int64_t v[3];
            vox_oracle_sample_euclid(s, k, v);
            int64_t b = (v[2] * dy + v[1]) * dx + v[0];
            grid[b / 32] |= (uint32_t)1u << (b % 32);
        }
        set += euclid_voxels(s, NULL);
    }
    return set;
}


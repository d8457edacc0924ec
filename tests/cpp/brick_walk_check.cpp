// Host-side driver for the exact brick helpers of the HIP library
// (paper_2009_09500_amd/csrc/vox_exact.h): prints, for every segment read
// from stdin, the bricks walk_bricks visits and the k-window box_window gives
// inside each of them, and checks that the walk cut into 2, 4 and 8 parts
// (walk_bricks_part) visits the same bricks with the same windows.  Built and
// run by tests/test_brick_math.py (CPU only).
//
// argv[1] == "euclid": the walk takes the Euclidean N of eq. (1),
// floor(|P1 - P0|), instead of the Chebyshev N.
// stdin:  dx dy dz lgx lgy lgz n, then n lines x0 y0 z0 x1 y1 z1
// stdout: per segment one line "i: b klo khi; b klo khi; ..."
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "vox_exact.h"

namespace {

uint32_t isqrt64(uint64_t s) {
    uint64_t r = (uint64_t)std::sqrt((double)s);
    while (r * r > s) --r;
    while ((r + 1) * (r + 1) <= s) ++r;
    return (uint32_t)r;
}

struct Piece {
    uint32_t b, klo, khi;
    bool operator==(const Piece& o) const { return b == o.b && klo == o.klo && khi == o.khi; }
};

}  // namespace

int main(int argc, char** argv) {
    const bool euclid = argc > 1 && std::strcmp(argv[1], "euclid") == 0;
    int dims[3], lg[3];
    long long n;
    if (scanf("%d %d %d %d %d %d %lld", &dims[0], &dims[1], &dims[2], &lg[0], &lg[1], &lg[2], &n) != 7)
        return 2;
    vox::BrickGeom bg;
    if (!vox::brick_geometry(dims[0], dims[1], dims[2], lg, bg)) return 3;
    for (long long i = 0; i < n; ++i) {
        vox::Seg g;
        if (scanf("%d %d %d %d %d %d", &g.p0[0], &g.p0[1], &g.p0[2], &g.p1[0], &g.p1[1], &g.p1[2]) != 6)
            return 4;
        printf("%lld:", i);
        if (!vox::in_volume(g, bg)) {
            printf(" out\n");
            continue;
        }
        vox::SegAxes s = vox::seg_axes(g);
        if (euclid) {
            uint64_t ss = 0;
            for (int ax = 0; ax < 3; ++ax) ss += (uint64_t)s.a[ax] * s.a[ax];
            s.N = isqrt64(ss);
        }
        std::vector<Piece> whole;
        vox::walk_bricks(s, bg, [&](uint32_t b, uint32_t klo, uint32_t khi) { whole.push_back({b, klo, khi}); });
        bool parts_ok = true;
        for (uint32_t parts = 2; parts <= vox::kMaxWalkParts; parts *= 2) {
            std::vector<Piece> cut;
            for (uint32_t p = 0; p < parts; ++p)
                vox::walk_bricks_part(s, bg, p, parts, [&](uint32_t b, uint32_t klo, uint32_t khi) {
                    cut.push_back({b, klo, khi});
                });
            if (!(cut == whole)) {
                printf(" MISMATCH parts %u;", parts);
                parts_ok = false;
            }
        }
        if (!parts_ok) {
            printf("\n");
            continue;
        }
        for (const Piece& pc : whole) {
            const uint32_t b = pc.b;
            int bx = (int)(b % (uint32_t)bg.nb[0]);
            int by = (int)((b / (uint32_t)bg.nb[0]) % (uint32_t)bg.nb[1]);
            int bz = (int)(b / ((uint32_t)bg.nb[0] * (uint32_t)bg.nb[1]));
            int32_t lo[3] = {bx << lg[0], by << lg[1], bz << lg[2]};
            int32_t hi[3];
            for (int ax = 0; ax < 3; ++ax) {
                int32_t e = dims[ax] - lo[ax];
                e = e < (1 << lg[ax]) ? e : (1 << lg[ax]);
                hi[ax] = lo[ax] + e - 1;
            }
            // The walk's own window and the clipped window must agree.
            uint32_t klo = 0, khi = 0;
            if (s.N > 0) vox::box_window(s, lo, hi, klo, khi);
            if (klo != pc.klo || khi != pc.khi) {
                printf(" MISMATCH walk %u %u box %u %u;", pc.klo, pc.khi, klo, khi);
                continue;
            }
            printf(" %u %u %u;", b, klo, khi);
        }
        printf("\n");
    }
    return 0;
}

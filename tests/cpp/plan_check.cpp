// Host-side driver for the per-scene planning rule of the HIP library
// (plan_scene in paper_2009_09500_amd/csrc/vox_exact.h, the code the plan
// kernel runs for each scene of a batch): prints what the plan enters in the
// scene table.  Built and run by tests/test_batch_plan.py (CPU only).
//
// stdin:  lgx lgy lgz segs_per_row count, then count lines
//         "segs n dim_x dim_y dim_z flags grid counts" (addresses as integers)
// stdout: per scene "valid flags rows nbricks nbx nby nbz dimx dimy dimz n"
#include <cstdio>

#include "vox_exact.h"

int main() {
    int lg[3];
    int count;
    long long per_row;
    if (scanf("%d %d %d %lld %d", &lg[0], &lg[1], &lg[2], &per_row, &count) != 5) return 2;
    for (int i = 0; i < count; ++i) {
        unsigned long long segs, grid, counts;
        long long n;
        int dx, dy, dz;
        unsigned flags;
        if (scanf("%llu %lld %d %d %d %u %llu %llu", &segs, &n, &dx, &dy, &dz, &flags, &grid, &counts) != 8)
            return 3;
        vox_scene in;
        in.segs = reinterpret_cast<const vox_segment*>((uintptr_t)segs);
        in.n = n;
        in.dim_x = dx;
        in.dim_y = dy;
        in.dim_z = dz;
        in.flags = flags;
        in.grid = reinterpret_cast<uint32_t*>((uintptr_t)grid);
        in.counts = reinterpret_cast<int32_t*>((uintptr_t)counts);
        const int32_t lgi[3] = {lg[0], lg[1], lg[2]};
        vox::BrickScene b;
        const bool valid = vox::plan_scene(in, lgi, per_row, b);
        printf("%d %u %u %u %d %d %d %d %d %d %lld\n", valid ? 1 : 0, b.flags, b.rows, b.bg.nbricks, b.bg.nb[0],
               b.bg.nb[1], b.bg.nb[2], b.bg.dim[0], b.bg.dim[1], b.bg.dim[2], (long long)b.n);
    }
    return 0;
}

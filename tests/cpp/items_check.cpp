// Host-side check of the fill's work items (vox_exact.h: split_threshold,
// brick_items, item_range), built and run by tests/test_brick_math.py (CPU
// only).  For brick totals drawn from several distributions (uniform, heavy
// tailed, a few huge bricks, totals near 2^32): the items beyond one per
// brick and the cut bricks stay within kMaxExtraItems (the size of their
// tables in the workspace), and the items of every brick tile its records
// exactly, each part non-empty.  Prints "ok" or the first failure.
#include <cstdio>
#include <random>
#include <vector>

#include "vox_exact.h"

int main() {
    std::mt19937_64 rng(20090950);
    for (int trial = 0; trial < 4000; ++trial) {
        const uint32_t nb = 1u + (uint32_t)(rng() % 20000u);
        std::vector<uint32_t> tot(nb, 0u);
        const int kind = trial % 5;
        for (uint32_t b = 0; b < nb; ++b) {
            if (kind == 0) tot[b] = (uint32_t)(rng() % 5000u);
            else if (kind == 1) tot[b] = (uint32_t)(rng() % 3u == 0 ? rng() % (1u << 20) : rng() % 64u);
            else if (kind == 2) tot[b] = 0u;
            else if (kind == 3) tot[b] = (uint32_t)(rng() % (1u << 12));
            else tot[b] = (uint32_t)(rng() % 100u);
        }
        if (kind == 2)
            for (int h = 0; h < 5; ++h) tot[rng() % nb] = (uint32_t)(rng() % 0xFFFFFFFFull);
        if (kind == 4) tot[rng() % nb] = 0xFFFFFFFFu;
        uint64_t total = 0;
        for (uint32_t c : tot) total += c;
        const uint64_t T = vox::split_threshold(total);
        uint64_t extra = 0, cut = 0;
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t k = vox::brick_items(tot[b], T);
            if (k < 1u || (k > 1u && (uint64_t)tot[b] <= T)) {
                printf("trial %d brick %u: %u items for %u records (T %llu)\n", trial, b, k, tot[b],
                       (unsigned long long)T);
                return 1;
            }
            extra += k - 1u;
            cut += k > 1u ? 1u : 0u;
            // Record offsets are 32-bit: the fill runs only when all records
            // stay below 2^32 - 1 (else the direct kernels serve the call),
            // so a brick's records start at most 2^32 - 1 - count.
            const uint32_t first = (uint32_t)((0xFFFFFFFFull - tot[b]) / 2u);
            uint32_t expect = first;
            for (uint32_t j = 0; j < k; ++j) {
                uint32_t lo, hi;
                vox::item_range(first, tot[b], j, k, lo, hi);
                if (lo != expect || hi < lo || (k > 1u && hi == lo) || (uint64_t)(hi - lo) > T) {
                    printf("trial %d brick %u item %u of %u: [%u, %u)\n", trial, b, j, k, lo, hi);
                    return 1;
                }
                expect = hi;
            }
            if (expect != first + tot[b]) {
                printf("trial %d brick %u: items end at %u\n", trial, b, expect);
                return 1;
            }
        }
        if (extra > vox::kMaxExtraItems || cut > vox::kMaxExtraItems) {
            printf("trial %d: %llu extra items, %llu cut bricks\n", trial, (unsigned long long)extra,
                   (unsigned long long)cut);
            return 1;
        }
    }
    printf("ok\n");
    return 0;
}

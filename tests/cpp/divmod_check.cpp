// Host check of the reciprocal-based exact division every kernel relies on
// (divmod_down and rcp_bias_down of paper_2009_09500_amd/csrc/vox_device.h,
// the library's own code built for the host): the remainders and quotients
// of eq. (3)'s numerators (2 k a + N - neg) / 2N, taken from a float
// reciprocal estimate and one integer correction.
//
// The hardware reciprocal (v_rcp_f32) is accurate to one ulp, so the estimate
// is one of the floats next to the correctly rounded 1/y.  For each of them
// (-1, 0 and +1 ulp), every divisor y in [2, 2^16) and every quotient
// q < min(2^15, 2^31 / y), the check divides x = q y and x = q y - 1 (the
// first and last numerators of each quotient, where a wrong estimate shows
// first), plus random numerators in the domain, and compares with integer
// division.  Prints the number of cases and mismatches; exit status 1 on a
// mismatch.  Built and run by tests/test_divmod.py (CPU only).
//
// argv[1] (optional): largest divisor + 1 (default 65536); argv[2]: threads;
// argv[3] = "unbiased": use the estimate without the downward scaling (a
// planted mistake the check must catch).
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "vox_device.h"

namespace {

struct Tally {
    uint64_t cases = 0, bad = 0;
    uint32_t bx = 0, by = 0;
    int bulp = 0;
};

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline bool one(uint32_t x, uint32_t y, float rcpd) {
    uint32_t q, r;
    vox::divmod_down(x, y, rcpd, q, r);
    return q == x / y && r == x % y;
}

bool g_unbiased = false;

void run(uint32_t y0, uint32_t y1, uint32_t ystep, Tally& t) {
    uint64_t seed = 0x51ED2700ull + y0;
    for (uint32_t y = y0; y < y1; y += ystep) {
        const float exact = 1.0f / (float)y;  // correctly rounded (y is exact in float)
        const float rcps[3] = {std::nextafterf(exact, 0.0f), exact, std::nextafterf(exact, 2.0f)};
        // Quotients below 2^15 and numerators below 2^31.
        uint64_t qmax = (((uint64_t)1 << 31) - 1) / y;
        if (qmax > 32767) qmax = 32767;
        const uint64_t xmax = (qmax + 1) * y - 1 < (((uint64_t)1 << 31) - 1) ? (qmax + 1) * y - 1
                                                                                : (((uint64_t)1 << 31) - 1);
        for (int u = 0; u < 3; ++u) {
            const float rcpd = g_unbiased ? rcps[u] : vox::rcp_bias_down(rcps[u]);
            uint64_t bad = 0, cases = 0;
            for (uint64_t q = 0; q <= qmax; ++q) {
                const uint32_t x = (uint32_t)(q * y);
                bool ok = one(x, y, rcpd);
                if (q > 0) ok &= one(x - 1, y, rcpd);
                cases += q > 0 ? 2 : 1;
                if (!ok) {
                    ++bad;
                    if (t.bad == 0 && bad == 1) {
                        t.bx = x;
                        t.by = y;
                        t.bulp = u - 1;
                    }
                }
            }
            // The last numerator of the last quotient, and random ones.
            bool ok = one((uint32_t)xmax, y, rcpd);
            for (int i = 0; i < 64; ++i) ok &= one((uint32_t)(splitmix(seed) % (xmax + 1)), y, rcpd);
            cases += 65;
            if (!ok) ++bad;
            t.cases += cases;
            t.bad += bad;
        }
    }
}

}  // namespace

int main(int argc, char** argv) {
    const uint32_t yend = argc > 1 ? (uint32_t)strtoul(argv[1], nullptr, 10) : 65536u;
    unsigned nt = argc > 2 ? (unsigned)strtoul(argv[2], nullptr, 10) : std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    g_unbiased = argc > 3 && std::string(argv[3]) == "unbiased";
    std::vector<Tally> tl(nt);
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nt; ++i) th.emplace_back([&, i] { run(2 + i, yend, nt, tl[i]); });
    for (auto& t : th) t.join();
    Tally all;
    for (const auto& t : tl) {
        all.cases += t.cases;
        if (t.bad && !all.bad) {
            all.bx = t.bx;
            all.by = t.by;
            all.bulp = t.bulp;
        }
        all.bad += t.bad;
    }
    printf("cases %llu mismatches %llu", (unsigned long long)all.cases, (unsigned long long)all.bad);
    if (all.bad) printf(" first x=%u y=%u ulp=%d", all.bx, all.by, all.bulp);
    printf("\n");
    return all.bad ? 1 : 0;
}

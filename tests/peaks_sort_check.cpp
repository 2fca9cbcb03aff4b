// Checks the candidate ordering of sas_peaks (host helper) against a plain
// stable sort with the field comparison, on seeded random records: narrow
// ranges (radix path), full 32-bit ranges (comparison fallback), negative
// bins, equal counts, and sizes 0, 1 and 2.  Exit status 0 when all agree.
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2509_26279_amd/csrc/peaks_sort.h"

struct Rec {
    uint32_t v_idx;
    int32_t bx, by;
    uint16_t count, flags;
};

static bool canon(const Rec &a, const Rec &b) {
    return a.v_idx != b.v_idx ? a.v_idx < b.v_idx : a.by != b.by ? a.by < b.by : a.bx < b.bx;
}
static bool bycount(const Rec &a, const Rec &b) {
    return a.count != b.count ? a.count > b.count : canon(a, b);
}

static bool same(const std::vector<Rec> &a, const std::vector<Rec> &b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i].v_idx != b[i].v_idx || a[i].bx != b[i].bx || a[i].by != b[i].by ||
            a[i].count != b[i].count || a[i].flags != b[i].flags)
            return false;
    return true;
}

int main() {
    std::mt19937_64 rng(20260926);
    int fails = 0, cases = 0;
    struct Shape { int64_t n; int64_t vmax, ylo, yhi, xlo, xhi; int cmax; };
    const Shape shapes[] = {
        {0, 10, 0, 5, 0, 5, 30},
        {1, 10, 0, 5, 0, 5, 30},
        {2, 10, -3, 5, -7, 5, 30},
        {3128, 84351, 0, 1023, 0, 511, 100},
        {5000, 1229685, -900, 900, -800, 800, 60},
        {4000, 4294967295LL, -2147483648LL, 2147483647LL, -2147483648LL, 2147483647LL, 65535},
        {4000, 1000, -2147483648LL, 2147483647LL, 0, 3, 65535},
        {2000, 3, 0, 1, 0, 1, 2},
    };
    for (const Shape &sh : shapes) {
        for (int rep = 0; rep < 3; ++rep) {
            // distinct (v_idx, by, bx): draw, then drop repeats
            std::vector<Rec> c;
            std::uniform_int_distribution<int64_t> dv(0, sh.vmax), dy(sh.ylo, sh.yhi),
                dx(sh.xlo, sh.xhi), dc(0, sh.cmax);
            for (int64_t i = 0; i < sh.n; ++i)
                c.push_back(Rec{(uint32_t)dv(rng), (int32_t)dx(rng), (int32_t)dy(rng),
                                (uint16_t)dc(rng), (uint16_t)(i & 1)});
            std::sort(c.begin(), c.end(), canon);
            c.erase(std::unique(c.begin(), c.end(),
                                [](const Rec &a, const Rec &b) {
                                    return a.v_idx == b.v_idx && a.by == b.by && a.bx == b.bx;
                                }),
                    c.end());
            std::shuffle(c.begin(), c.end(), rng);
            for (int order = 0; order < 2; ++order) {
                std::vector<Rec> want = c, got = c;
                std::stable_sort(want.begin(), want.end(), order ? bycount : canon);
                sas::sort_candidates(got, order == 1);
                ++cases;
                if (!same(want, got)) {
                    ++fails;
                    std::printf("mismatch: n=%zu order=%d vmax=%lld\n", c.size(), order,
                                (long long)sh.vmax);
                }
            }
        }
    }
    std::printf("%d cases, %d mismatches\n", cases, fails);
    return fails ? 1 : 0;
}

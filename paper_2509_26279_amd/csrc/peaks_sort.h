// Host-side ordering of the candidates that sas_peaks returns (plain C++, no
// HIP): the canonical order (v_idx, by, bx) ascending, or count descending
// and then canonical.  A vote emits one record per (velocity, bin), so the
// canonical triple is unique and both orders are total.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

namespace sas {

template <class C>
inline bool canonical_less(const C &a, const C &b) {
    if (a.v_idx != b.v_idx) return a.v_idx < b.v_idx;
    if (a.by != b.by) return a.by < b.by;
    return a.bx < b.bx;
}

template <class C>
inline bool by_count_less(const C &a, const C &b) {
    if (a.count != b.count) return a.count > b.count;
    return canonical_less(a, b);
}

// Sorts c in place.  Each record gets the mixed-radix key
//   ((k_count * NV + v_idx - v_min) * NY + by - by_min) * NX + bx - bx_min,
// with k_count = count_max - count for the by-count order (0 otherwise) and
// NV, NY, NX the ranges of the fields over c: the key is strictly monotone in
// the order.  When the key range fits in 64 bits a stable LSD radix sort of
// (key, position) pairs orders the records in as many 8-bit passes as the
// range needs; otherwise std::sort with the field comparison does.
template <class C>
inline void sort_candidates(std::vector<C> &c, bool by_count) {
    const size_t n = c.size();
    if (n < 2) return;
    uint32_t v0 = c[0].v_idx, v1 = c[0].v_idx;
    int32_t y0 = c[0].by, y1 = c[0].by, x0 = c[0].bx, x1 = c[0].bx;
    uint32_t k1 = c[0].count, k0 = c[0].count;
    for (const C &r : c) {
        v0 = std::min<uint32_t>(v0, r.v_idx);
        v1 = std::max<uint32_t>(v1, r.v_idx);
        y0 = std::min<int32_t>(y0, r.by);
        y1 = std::max<int32_t>(y1, r.by);
        x0 = std::min<int32_t>(x0, r.bx);
        x1 = std::max<int32_t>(x1, r.bx);
        k0 = std::min<uint32_t>(k0, r.count);
        k1 = std::max<uint32_t>(k1, r.count);
    }
    typedef unsigned __int128 u128;
    const u128 nv = (u128)(v1 - v0) + 1;
    const u128 ny = (u128)((int64_t)y1 - y0) + 1;
    const u128 nx = (u128)((int64_t)x1 - x0) + 1;
    const u128 nk = by_count ? (u128)(k1 - k0) + 1 : 1;
    // each factor is at most 2^32, so the product of the first three fits
    const u128 range = nv * ny * nx;
    if (range > (((u128)1 << 64) - 1) / nk) {
        if (by_count)
            std::sort(c.begin(), c.end(), by_count_less<C>);
        else
            std::sort(c.begin(), c.end(), canonical_less<C>);
        return;
    }
    const uint64_t top = (uint64_t)(range * nk - 1);  // the largest key
    int bits = 0;
    while (bits < 64 && (top >> bits) != 0) ++bits;
    typedef std::pair<uint64_t, uint32_t> KP;
    std::vector<KP> a(n), b(n);
    for (size_t i = 0; i < n; ++i) {
        const C &r = c[i];
        const uint64_t kc = by_count ? (uint64_t)(k1 - r.count) : 0;
        const uint64_t key =
            ((kc * (uint64_t)nv + (r.v_idx - v0)) * (uint64_t)ny + (uint64_t)((int64_t)r.by - y0)) *
                (uint64_t)nx +
            (uint64_t)((int64_t)r.bx - x0);
        a[i] = KP(key, (uint32_t)i);
    }
    for (int sh = 0; sh < bits; sh += 8) {
        size_t cnt[257] = {0};
        for (const KP &p : a) ++cnt[((p.first >> sh) & 255) + 1];
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (const KP &p : a) b[cnt[(p.first >> sh) & 255]++] = p;
        a.swap(b);
    }
    std::vector<C> out(n);
    for (size_t i = 0; i < n; ++i) out[i] = c[a[i].second];
    c.swap(out);
}

}  // namespace sas

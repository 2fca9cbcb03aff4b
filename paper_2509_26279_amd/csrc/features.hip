// Candidate features for learned vetting.
//
// One wave per candidate (v, bx, by).  Lanes take epochs; for its epoch a
// lane reads the window-index runs covering the bin's preimage
// [bx b + S(v), (bx + 1) b + S(v)) x [by b + S(vy), ...) with S(v) =
// ceil(v d / 65536) (the exact Step-2 bin of Sec. 2.1, as in the vote), and
// accumulates in FP64 over the contributing detections:
//   count, SNR sum / max / min, residual sums r_x, r_y, r^2, the time
//   coordinate tau = d / D and its products with r, per-slice counts and
//   residual sums (slice = min(3, floor(4 d / D))), epoch presence.
// Wave reductions then give the 32 features:
//   f0 c/E  f1 n/E  f2 min d/D  f3 (max d - min d)/D  f4 longest epoch run/E
//   f5 vx/vmax  f6 vy/vmax  f7 |v|/vmax  f8 sum snr/E  f9 max snr - 3
//   f10 min snr - 3  f11 mean snr - 3  f12, f13 mean r  f14, f15 std r
//   f16, f17 least-squares slope of r against tau (0 if all d equal)
//   f18..f25 per-slice mean r_x, r_y  f26..f29 slice fractions
//   f30 (n - c)/n  f31 RMS of r about the least-squares lines (x and y)
// with r_x = (65536 x - vx d) / (65536 b) - bx - 1/2.
#include "internal.h"

namespace sas {
namespace {

constexpr int FT = 256;  // threads per block: 4 candidates at a time

__device__ inline int32_t shift_q8(int32_t v, int32_t d) {
    return (int32_t)(((int64_t)v * (int64_t)d + 65535) >> 16);
}

// Neighbour key of a candidate: lattice velocity index (v / s rounded half
// up) and bin, packed 11 + 11 + 15 + 15 bits above a 12-bit count; all ones
// when a component is out of range (such a candidate has no neighbours).
constexpr uint64_t kNoNeighbourKey = ~(uint64_t)0;

__device__ inline int64_t lattice_index(int32_t v, int32_t s) {
    const int64_t n = 2 * (int64_t)v + s, d = 2 * (int64_t)s;
    return n >= 0 ? n / d : -((-n + d - 1) / d);  // floor
}

__device__ inline bool packable(int64_t ix, int64_t iy, int64_t bx, int64_t by) {
    return ix >= -1022 && ix <= 1022 && iy >= -1022 && iy <= 1022 && bx >= -16382 &&
           bx <= 16382 && by >= -16382 && by <= 16382;
}

__device__ inline uint64_t pack_key(int64_t ix, int64_t iy, int64_t bx, int64_t by) {
    return ((uint64_t)(ix + 1024) << 53) | ((uint64_t)(iy + 1024) << 42) |
           ((uint64_t)(bx + 16384) << 27) | ((uint64_t)(by + 16384) << 12);
}

__global__ void k_neighbour_keys(FeatureArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_cand) return;
    const sas_candidate cd = a.cand[i];
    const int64_t ix = lattice_index(a.vel[2 * (int64_t)cd.v_idx], a.spacing);
    const int64_t iy = lattice_index(a.vel[2 * (int64_t)cd.v_idx + 1], a.spacing);
    a.keys[i] = packable(ix, iy, cd.bx, cd.by)
                    ? pack_key(ix, iy, cd.bx, cd.by) | (uint64_t)min((int)cd.count, 4095)
                    : kNoNeighbourKey;
}

// Largest count among the candidates with packed key `want` (count bits
// clear), or -1 when there is none.
__device__ inline int find_key(const uint64_t *keys, int64_t n, uint64_t want) {
    const uint64_t w = want >> 12;
    int64_t lo = 0, hi = n;  // first key whose upper bits are >= w
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> 12) < w) lo = mid + 1; else hi = mid;
    }
    int best = -1;
    for (; lo < n && (keys[lo] >> 12) == w; ++lo) best = max(best, (int)(keys[lo] & 4095));
    return best;
}

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int64_t wmin_i(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}
__device__ inline int64_t wmax_i(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__global__ void __launch_bounds__(FT) k_features(FeatureArgs a, const uint64_t *nkeys) {
    const int lane = __lane_id();
    const int64_t wave_id = ((int64_t)blockIdx.x * FT + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * FT) >> 6;
    const PreparedCatalog &c = a.cat;
    const int E = c.n_epochs;
    const int lb = a.log2b;
    const double D = (double)a.span;
    const double inv_b = 1.0 / (65536.0 * (double)(1 << lb));
    for (int64_t k = wave_id; k < a.n_cand; k += n_waves) {
        const sas_candidate cd = a.cand[k];
        const int32_t vx = a.vel[2 * (int64_t)cd.v_idx], vy = a.vel[2 * (int64_t)cd.v_idx + 1];
        double n = 0, ssum = 0, rxs = 0, rys = 0, rxx = 0, ryy = 0;
        double ts = 0, tts = 0, txs = 0, tys = 0;
        double sn[4] = {0, 0, 0, 0}, sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
        int64_t dmin = INT64_MAX, dmax = INT64_MIN, dpmin = INT64_MAX, dpmax = INT64_MIN;
        double dup = 0;
        uint64_t pres0 = 0, pres1 = 0, pres2 = 0, pres3 = 0;  // epoch presence, 4 x 64 bits
        for (int e0 = 0; e0 < E; e0 += 64) {
            const int e = e0 + lane;
            bool has = false;
            if (e < E) {
                const int32_t d = c.dt[e];
                if (d >= 0) {
                    const int64_t xlo = ((int64_t)cd.bx << lb) + shift_q8(vx, d);
                    const int64_t ylo = ((int64_t)cd.by << lb) + shift_q8(vy, d);
                    const int64_t xhi = xlo + ((int64_t)1 << lb), yhi = ylo + ((int64_t)1 << lb);
                    if (xhi > c.x0 && xlo < c.x1 && yhi > c.y0 && ylo < c.y1) {
                        const int cx0 = (int)((max(xlo, (int64_t)c.x0) - c.x0) >> c.cell_log2);
                        const int cx1 = (int)((min(xhi, (int64_t)c.x1) - 1 - c.x0) >> c.cell_log2);
                        const int cy0 = (int)((max(ylo, (int64_t)c.y0) - c.y0) >> c.cell_log2);
                        const int cy1 = (int)((min(yhi, (int64_t)c.y1) - 1 - c.y0) >> c.cell_log2);
                        const int sl = (int)min((int64_t)3, (4 * (int64_t)d) / a.span);
                        const double tau = (double)d / D;
                        for (int cy = cy0; cy <= cy1; ++cy) {
                            const int64_t base = ((int64_t)e * c.ncy + cy) * c.ncx;
                            const int32_t j1 = c.off[base + cx1 + 1];
                            for (int32_t j = c.off[base + cx0]; j < j1; ++j) {
                                const int2 p = c.sxy[j];
                                if (p.x < xlo || p.x >= xhi || p.y < ylo || p.y >= yhi) continue;
                                const double rx = (double)((int64_t)65536 * p.x - (int64_t)vx * d) * inv_b -
                                                  (double)cd.bx - 0.5;
                                const double ry = (double)((int64_t)65536 * p.y - (int64_t)vy * d) * inv_b -
                                                  (double)cd.by - 0.5;
                                const double s = a.snr ? (double)a.snr[c.sidx[j]] : 0.0;
                                if (has) dup += 1;
                                has = true;
                                n += 1;
                                ssum += s;
                                rxs += rx;
                                rys += ry;
                                rxx += rx * rx;
                                ryy += ry * ry;
                                ts += tau;
                                tts += tau * tau;
                                txs += tau * rx;
                                tys += tau * ry;
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    if (q == sl) {
                                        sn[q] += 1;
                                        sx[q] += rx;
                                        sy[q] += ry;
                                    }
                                }
                                dmin = min(dmin, (int64_t)d);
                                dmax = max(dmax, (int64_t)d);
                            }
                        }
                        if (has) {
                            dpmin = min(dpmin, (int64_t)d);
                            dpmax = max(dpmax, (int64_t)d);
                        }
                    }
                }
            }
            const uint64_t bal = __ballot(has);
            if (e0 == 0) pres0 = bal;
            else if (e0 == 64) pres1 = bal;
            else if (e0 == 128) pres2 = bal;
            else pres3 = bal;
        }
        n = wsum(n);
        float f[kFeatures];
        for (int q = 0; q < kFeatures; ++q) f[q] = 0.0f;
        // every lane holds the wave totals after the reductions
        ssum = wsum(ssum);
        rxs = wsum(rxs);
        rys = wsum(rys);
        rxx = wsum(rxx);
        ryy = wsum(ryy);
        ts = wsum(ts);
        tts = wsum(tts);
        txs = wsum(txs);
        tys = wsum(tys);
        dup = wsum(dup);
        dmin = wmin_i(dmin);
        dmax = wmax_i(dmax);
        dpmin = wmin_i(dpmin);
        dpmax = wmax_i(dpmax);
        for (int q = 0; q < 4; ++q) {
            sn[q] = wsum(sn[q]);
            sx[q] = wsum(sx[q]);
            sy[q] = wsum(sy[q]);
        }
        if (n > 0) {
            int cnt = 0, best = 0, run = 0;
            for (int e = 0; e < E; ++e) {  // longest run of consecutive present epochs
                const uint64_t w = e < 64 ? pres0 : e < 128 ? pres1 : e < 192 ? pres2 : pres3;
                const bool p = (w >> (e & 63)) & 1;
                cnt += p;
                run = p ? run + 1 : 0;
                best = max(best, run);
            }
            const double mx = rxs / n, my = rys / n;
            const double vmax = a.vmax > 0 ? a.vmax : 1.0;
            f[0] = (float)(cnt / (double)E);
            f[1] = (float)(n / E);
            f[2] = (float)((double)dpmin / D);
            f[3] = (float)((double)(dpmax - dpmin) / D);
            f[4] = (float)(best / (double)E);
            f[5] = (float)(vx / vmax);
            f[6] = (float)(vy / vmax);
            f[7] = (float)(sqrt((double)vx * vx + (double)vy * vy) / vmax);
            f[8] = (float)(ssum / E);
            f[11] = (float)(ssum / n - 3.0);
            f[12] = (float)mx;
            f[13] = (float)my;
            f[14] = (float)sqrt(fmax(rxx / n - mx * mx, 0.0));
            f[15] = (float)sqrt(fmax(ryy / n - my * my, 0.0));
            const double sxx = rxx - n * mx * mx, syy = ryy - n * my * my;
            double sse = sxx + syy;  // about the means, then about the fitted lines
            if (dmax > dmin) {
                const double mt = ts / n, stt = tts - n * mt * mt;
                const double sxt = txs - n * mt * mx, syt = tys - n * mt * my;
                f[16] = (float)(sxt / stt);
                f[17] = (float)(syt / stt);
                sse -= (sxt * sxt + syt * syt) / stt;
            }
            f[31] = (float)sqrt(fmax(sse, 0.0) / (2.0 * n));
            for (int q = 0; q < 4; ++q) {
                if (sn[q] > 0) {
                    f[18 + 2 * q] = (float)(sx[q] / sn[q]);
                    f[19 + 2 * q] = (float)(sy[q] / sn[q]);
                }
                f[26 + q] = (float)(sn[q] / n);
            }
            f[30] = (float)((n - cnt) / n);
        }
        // neighbouring candidates: lane q < 81 takes offset q (base 3 digits - 1)
        {
            double ncnt = 0.0, nbest = 0.0;
            if (a.spacing > 0 && nkeys) {
                const int64_t ix = lattice_index(vx, a.spacing), iy = lattice_index(vy, a.spacing);
                for (int q = lane; q < 81; q += 64) {
                    if (q == 40) continue;  // the candidate itself
                    const int64_t dx = q % 3 - 1, dy = (q / 3) % 3 - 1;
                    const int64_t ex = (q / 9) % 3 - 1, ey = q / 27 - 1;
                    if (!packable(ix, iy, cd.bx, cd.by) ||
                        !packable(ix + dx, iy + dy, (int64_t)cd.bx + ex, (int64_t)cd.by + ey))
                        continue;
                    const int c = find_key(nkeys, a.n_cand,
                                           pack_key(ix + dx, iy + dy, (int64_t)cd.bx + ex,
                                                    (int64_t)cd.by + ey));
                    if (c >= 0) {
                        ncnt += 1.0;
                        nbest = fmax(nbest, (double)c);
                    }
                }
            }
            ncnt = wsum(ncnt);
            nbest = wmax(nbest);
            const double own = (double)min((int)cd.count, 4095);
            f[9] = (float)(ncnt / 80.0);
            f[10] = (float)(ncnt > 0 && own > 0 ? nbest / own : 0.0);
        }
        if (lane < kFeatures) {
            float mine = 0.0f;
#pragma unroll
            for (int q = 0; q < kFeatures; ++q) mine = lane == q ? f[q] : mine;
            a.feat[k * kFeatures + lane] = mine;
        }
    }
}

}  // namespace

hipError_t launch_features(const FeatureArgs &a, hipStream_t stream) {
    if (a.n_cand <= 0) return hipSuccess;
    uint64_t *sorted = nullptr;
    if (a.spacing > 0) {
        hipLaunchKernelGGL(k_neighbour_keys, dim3((unsigned)((a.n_cand + 255) / 256)), dim3(256), 0,
                           stream, a);
        hipError_t e = launch_radix_sort_u64(a.keys, a.keys_alt, a.n_cand, 12, 64, a.hist,
                                             a.hist_blocksum, stream, &sorted);
        if (e != hipSuccess) return e;
    }
    const int64_t blocks = (a.n_cand + FT / 64 - 1) / (FT / 64);
    hipLaunchKernelGGL(k_features, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(FT), 0,
                       stream, a, (const uint64_t *)sorted);
    return hipGetLastError();
}

}  // namespace sas

// Refine, Gather and iterate (Steps 4-6 of Sec. 2.1) on the GPU.
//
// Step 4 fits a straight trajectory to each cluster by the multivariate
// regression of Sec. 2 (X = t, Y = (x, y)), with the mean and covariance of
// the Minimum Covariance Determinant subset in place of the sample ones.
// FAST-MCD (Rousseeuw and Van Driessen 1999) finds that subset: from random
// 4-point starts (an input table), C-steps - the mean and covariance of the
// current subset, the Mahalanobis distance of every point, the h closest as
// the next subset - never raise the determinant; two C-steps per start, the
// 10 lowest determinants iterated to convergence, the lowest wins.  Step 5
// gathers the catalog detections within the radius of the fitted line
// through the vote's window index; Step 6 repeats until the gathered set
// stops changing.
//
// One workgroup per cluster (grid-stride over clusters).  The point set
// (at most kMaxPoints) lives in LDS as t (h since t0), x, y (px) in FP64;
// the eight waves take the starts; a C-step ranks the distances exactly
// (each point counts the points before it, ties to the lower position), so
// the chosen subset does not depend on any reduction order.
//
// Rules shared with the reference definition: a point set is ordered by
// catalog index; h = (n + 4) / 2; a start whose 4 points repeat, or whose
// covariance is degenerate (det <= 1e-12 S_tt S_xx S_yy), is dropped; a
// degenerate subset ends its C-steps; at most 30 C-steps per refined start
// and 10 rounds; fewer than 5 points end the iteration.
#include <math.h>

#include "internal.h"

namespace sas {
namespace {

constexpr int RT = 512;             // threads per cluster workgroup
constexpr int RW = RT / 64;
constexpr int kMaxPoints = 512;     // points of one set held in LDS
constexpr int kMaskWords = kMaxPoints / 32;
constexpr int kPtsPerLane = kMaxPoints / 64;  // the wave's points per lane, at most
constexpr int kBest = 10;
constexpr int kMaxCsteps = 30;
constexpr int kMaxRounds = 10;
constexpr int kMinPoints = 5;
constexpr double kDegenerate = 1e-12;

struct Cov {
    double mu[3];
    double s[6];  // tt, tx, ty, xx, xy, yy (normalised by the point count)
};

__device__ inline double det3(const double *s) {
    return s[0] * (s[3] * s[5] - s[4] * s[4]) - s[1] * (s[1] * s[5] - s[4] * s[2]) +
           s[2] * (s[1] * s[4] - s[3] * s[2]);
}

__device__ inline bool degenerate(const double *s) {
    return det3(s) <= kDegenerate * s[0] * s[3] * s[5];
}

// Inverse of the symmetric 3x3 matrix s (same layout), by cofactors.
__device__ inline void inv3(const double *s, double *v) {
    const double c00 = s[3] * s[5] - s[4] * s[4];
    const double c01 = s[2] * s[4] - s[1] * s[5];
    const double c02 = s[1] * s[4] - s[2] * s[3];
    const double c11 = s[0] * s[5] - s[2] * s[2];
    const double c12 = s[1] * s[2] - s[0] * s[4];
    const double c22 = s[0] * s[3] - s[1] * s[1];
    const double d = s[0] * c00 + s[1] * c01 + s[2] * c02;
    v[0] = c00 / d;
    v[1] = c01 / d;
    v[2] = c02 / d;
    v[3] = c11 / d;
    v[4] = c12 / d;
    v[5] = c22 / d;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Shared {
    double zt[kMaxPoints], zx[kMaxPoints], zy[kMaxPoints];
    double d2[RW][kMaxPoints];
    double dets[kMaxRefineStarts];
    int32_t cur[kMaxPoints];  // catalog indices of the current set, ascending
    int32_t nxt[kMaxPoints];  // gathered set
    int32_t tmp[kMaxPoints];
    uint32_t mask[kBest][kMaskWords];
    Cov cov[kBest];
    double cdet[kBest];
    int32_t top[kBest];
    int32_t n_top, n_nxt, overflow;
};

// Mean and covariance of the points whose flag is set (lane-held flags of
// points lane + 64 k), by the wave; all lanes get the result.
template <int KPL>
__device__ Cov wave_moments(const Shared &sh, int n, const bool *in, int cnt) {
    const int lane = __lane_id();
    Cov c;
    double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
        const int i = lane + 64 * k;
        if (i < n && in[k]) {
            a0 += sh.zt[i];
            a1 += sh.zx[i];
            a2 += sh.zy[i];
        }
    }
    c.mu[0] = wave_sum(a0) / cnt;
    c.mu[1] = wave_sum(a1) / cnt;
    c.mu[2] = wave_sum(a2) / cnt;
    double s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
        const int i = lane + 64 * k;
        if (i < n && in[k]) {
            const double dt = sh.zt[i] - c.mu[0], dx = sh.zx[i] - c.mu[1], dy = sh.zy[i] - c.mu[2];
            s[0] += dt * dt;
            s[1] += dt * dx;
            s[2] += dt * dy;
            s[3] += dx * dx;
            s[4] += dx * dy;
            s[5] += dy * dy;
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) c.s[q] = wave_sum(s[q]) / cnt;
    return c;
}

// One C-step by the wave: distances from (mu, S^-1) into its d2 row, then
// in[k] = point lane + 64 k is among the h closest (ties to the lower
// position).  Returns whether the subset changed.
template <int KPL>
__device__ bool c_step(Shared &sh, int n, int h, const Cov &c, bool *in) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    double v[6];
    inv3(c.s, v);
    double *d2 = sh.d2[wave];
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
        const int i = lane + 64 * k;
        if (i < n) {
            const double a = sh.zt[i] - c.mu[0], b = sh.zx[i] - c.mu[1], e = sh.zy[i] - c.mu[2];
            d2[i] = a * (v[0] * a + v[1] * b + v[2] * e) + b * (v[1] * a + v[3] * b + v[4] * e) +
                    e * (v[2] * a + v[4] * b + v[5] * e);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int rank[KPL];
    double mine[KPL];
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
        rank[k] = 0;
        mine[k] = (lane + 64 * k < n) ? d2[lane + 64 * k] : 0.0;
    }
    // blocks of U distances loaded before they are compared (the loads of a
    // block are in flight together; fewer when each lane holds many points)
    constexpr int U = KPL <= 2 ? 8 : 2;
    int j = 0;
    for (; j + U <= n; j += U) {
        double dj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) dj[u] = d2[j + u];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < KPL; ++k) {
                const int i = lane + 64 * k;
                rank[k] += (dj[u] < mine[k] || (dj[u] == mine[k] && j + u < i)) ? 1 : 0;
            }
    }
    for (; j < n; ++j) {
        const double dj = d2[j];
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const int i = lane + 64 * k;
            rank[k] += (dj < mine[k] || (dj == mine[k] && j < i)) ? 1 : 0;
        }
    }
    bool changed = false;
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
        const bool nin = lane + 64 * k < n && rank[k] < h;
        changed |= nin != in[k];
        in[k] = nin;
    }
    __builtin_amdgcn_wave_barrier();  // d2 is read before the next step writes it
    return __any(changed);
}

// The first two C-steps of start s (both phases take this same path); the
// subset flags and its moments on return.  False when the start is dropped.
template <int KPL>
__device__ bool start_steps(Shared &sh, int n, int h, const uint32_t *starts, int s, bool *in,
                            Cov &c) {
    const int lane = __lane_id();
    int j[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) j[q] = (int)(starts[4 * s + q] % (uint32_t)n);
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (j[a] == j[b]) return false;
    // mean and covariance of the 4 points (every lane computes them)
    double mu[3] = {0, 0, 0};
    for (int q = 0; q < 4; ++q) {
        mu[0] += sh.zt[j[q]];
        mu[1] += sh.zx[j[q]];
        mu[2] += sh.zy[j[q]];
    }
    Cov c0;
    for (int r = 0; r < 3; ++r) c0.mu[r] = mu[r] / 4;
    double s6[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 4; ++q) {
        const double dt = sh.zt[j[q]] - c0.mu[0], dx = sh.zx[j[q]] - c0.mu[1],
                     dy = sh.zy[j[q]] - c0.mu[2];
        s6[0] += dt * dt;
        s6[1] += dt * dx;
        s6[2] += dt * dy;
        s6[3] += dx * dx;
        s6[4] += dx * dy;
        s6[5] += dy * dy;
    }
    for (int q = 0; q < 6; ++q) c0.s[q] = s6[q] / 4;
    if (degenerate(c0.s)) return false;
#pragma unroll
    for (int k = 0; k < KPL; ++k) in[k] = false;
    c_step<KPL>(sh, n, h, c0, in);  // 4 points -> h points
    c = wave_moments<KPL>(sh, n, in, h);
    if (!degenerate(c.s) && c_step<KPL>(sh, n, h, c, in)) c = wave_moments<KPL>(sh, n, in, h);
    (void)lane;
    return true;
}

// Ascending sort of a[0, m) (distinct or not) into out by rank counting.
__device__ void sort_into(const int32_t *a, int m, int32_t *out) {
    for (int i = threadIdx.x; i < m; i += RT) {
        const int32_t v = a[i];
        int r = 0;
        for (int j = 0; j < m; ++j) r += (a[j] < v || (a[j] == v && j < i)) ? 1 : 0;
        out[r] = v;
    }
}

// FAST-MCD on the n points in LDS (KPL >= ceil(n / 64) points per lane):
// the first stage scores every start by the determinant after two C-steps,
// the kBest lowest (ties to the earlier start) are iterated until the subset
// holds; their subsets, moments and determinants are left in sh.
template <int KPL>
__device__ void mcd_stages(Shared &sh, const RefineArgs &a, int n, int h) {
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    (void)tid;
    // FAST-MCD, first stage: two C-steps from every start
    for (int s = wave; s < a.n_starts; s += RW) {
        bool in[KPL];
        Cov cv;
        const bool ok = start_steps<KPL>(sh, n, h, a.starts, s, in, cv);
        if (lane == 0) sh.dets[s] = ok ? det3(cv.s) : INFINITY;
    }
    __syncthreads();
    if (wave == 0) {  // the kBest lowest (det, start)
        int nt = 0;
        double last_d = -INFINITY;
        int last_s = -1;
        for (; nt < kBest; ++nt) {
            double bd = INFINITY;
            int bs = -1;
            for (int s = lane; s < a.n_starts; s += 64) {
                const double d = sh.dets[s];
                const bool after = d > last_d || (d == last_d && s > last_s);
                if (after && d != INFINITY && (d < bd || (d == bd && s < bs) || bs < 0)) {
                    bd = d;
                    bs = s;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double od = __shfl_xor(bd, o, 64);
                const int os = __shfl_xor(bs, o, 64);
                if (os >= 0 && (bs < 0 || od < bd || (od == bd && os < bs))) {
                    bd = od;
                    bs = os;
                }
            }
            if (bs < 0) break;
            if (lane == 0) sh.top[nt] = bs;
            last_d = bd;
            last_s = bs;
        }
        if (lane == 0) sh.n_top = nt;
    }
    __syncthreads();
    const int n_top = sh.n_top;
    // second stage: the best starts iterated until the subset holds
    for (int k = wave; k < n_top; k += RW) {
        bool in[KPL];
        Cov cv;
        start_steps<KPL>(sh, n, h, a.starts, sh.top[k], in, cv);
        for (int it = 0; it < kMaxCsteps; ++it) {
            if (degenerate(cv.s)) break;
            if (!c_step<KPL>(sh, n, h, cv, in)) break;
            cv = wave_moments<KPL>(sh, n, in, h);
        }
#pragma unroll
        for (int q = 0; q < kPtsPerLane; ++q) {
            const uint64_t b = q < KPL ? __ballot(in[q < KPL ? q : 0]) : 0;
            if (lane == 0) {
                sh.mask[k][2 * q] = (uint32_t)b;
                sh.mask[k][2 * q + 1] = (uint32_t)(b >> 32);
            }
        }
        if (lane == 0) {
            sh.cov[k] = cv;
            sh.cdet[k] = det3(cv.s);
        }
    }
    __syncthreads();
}

__device__ inline bool cell_span(int64_t lo, int64_t hi, int32_t f0, int32_t f1, int cl, int *c0,
                                 int *c1) {
    if (hi <= f0 || lo >= f1) return false;
    *c0 = (int)((max(lo, (int64_t)f0) - f0) >> cl);
    *c1 = (int)((min(hi, (int64_t)f1) - 1 - f0) >> cl);
    return true;
}

__global__ void __launch_bounds__(RT) k_refine_clusters(RefineArgs a) {
    __shared__ Shared sh;
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const PreparedCatalog &c = a.cat;
    const double r2max = a.radius_px * a.radius_px;
    for (int64_t cl = blockIdx.x; cl < a.n_clusters; cl += gridDim.x) {
        const int32_t f = a.first[cl], m0 = a.first[cl + 1] - f;
        sas_refined res{};
        res.status = SAS_REFINE_TOO_SMALL;
        int n = m0;
        __syncthreads();  // the previous cluster is done with the shared state
        if (tid == 0) sh.overflow = 0;
        __syncthreads();
        if (f < 0 || m0 < 0 || (int64_t)f + m0 > a.n_members) {
            res.status = SAS_REFINE_BAD_INPUT;
            n = -1;
        } else if (m0 > kMaxPoints) {
            res.status = SAS_REFINE_TOO_LARGE;
            n = -1;
        } else {
            for (int i = tid; i < m0; i += RT) {
                const int32_t q = a.members[f + i];
                if (q < 0 || q >= a.n) sh.overflow = 1;  // a member outside the catalog
                sh.tmp[i] = q;
            }
            __syncthreads();
            if (sh.overflow) {
                res.status = SAS_REFINE_BAD_INPUT;
                n = -1;
            } else {
                sort_into(sh.tmp, m0, sh.cur);
            }
        }
        int32_t n_g = 0;  // gathered by the last fit
        for (int rnd = 1; n >= 0 && rnd <= kMaxRounds; ++rnd) {
            __syncthreads();
            if (n < kMinPoints) {
                res.status = SAS_REFINE_TOO_SMALL;
                break;
            }
            for (int i = tid; i < n; i += RT) {
                const int32_t q = sh.cur[i];
                sh.zt[i] = (double)c.dt[a.epoch[q]] / 65536.0;
                sh.zx[i] = (double)a.x[q] / 256.0;
                sh.zy[i] = (double)a.y[q] / 256.0;
            }
            const int h = (n + 4) / 2;
            __syncthreads();
            switch ((n + 63) >> 6) {
            case 1: mcd_stages<1>(sh, a, n, h); break;
            case 2: mcd_stages<2>(sh, a, n, h); break;
            case 3:
            case 4: mcd_stages<4>(sh, a, n, h); break;
            default: mcd_stages<8>(sh, a, n, h); break;
            }
            const int n_top = sh.n_top;
            if (n_top == 0) {
                res.status = SAS_REFINE_NO_START;
                break;
            }
            __syncthreads();
            int best = 0;
            for (int k = 1; k < n_top; ++k)
                if (sh.cdet[k] < sh.cdet[best]) best = k;
            const Cov cv = sh.cov[best];
            // the regression of Sec. 2 from the MCD mean and covariance
            const double bx = cv.s[1] / cv.s[0], by = cv.s[2] / cv.s[0];
            const double cx = cv.mu[1] - bx * cv.mu[0], cy = cv.mu[2] - by * cv.mu[0];
            res.vx = bx;
            res.vy = by;
            res.x0 = cx;
            res.y0 = cy;
            res.sxx = cv.s[3] - bx * bx * cv.s[0];
            res.sxy = cv.s[4] - bx * by * cv.s[0];
            res.syy = cv.s[5] - by * by * cv.s[0];
            res.n_points = h;
            res.rounds = rnd;
            if (a.subset && cl < a.subset_clusters) {  // the MCD subset (catalog indices)
                for (int i = tid; i < n; i += RT)
                    if ((sh.mask[best][i >> 5] >> (i & 31)) & 1u) {
                        int r = 0;
                        for (int j = 0; j < i; ++j) r += (sh.mask[best][j >> 5] >> (j & 31)) & 1u;
                        a.subset[cl * (int64_t)kMaxPoints + r] = sh.cur[i];
                    }
            }
            // Step 5: the catalog detections within the radius of c + B t
            if (tid == 0) {
                sh.n_nxt = 0;
                sh.overflow = 0;
            }
            __syncthreads();
            for (int e = tid; e < c.n_epochs; e += RT) {
                const int32_t d = c.dt[e];
                if (d < 0) continue;
                const double t = (double)d / 65536.0;
                const double px = cx + bx * t, py = cy + by * t;
                const double lo_x = (px - a.radius_px) * 256.0, hi_x = (px + a.radius_px) * 256.0;
                const double lo_y = (py - a.radius_px) * 256.0, hi_y = (py + a.radius_px) * 256.0;
                if (!(hi_x >= -2147483648.0 && lo_x < 2147483647.0 && hi_y >= -2147483648.0 &&
                      lo_y < 2147483647.0))
                    continue;
                const int64_t xlo = (int64_t)floor(lo_x), xhi = (int64_t)floor(hi_x) + 2;
                const int64_t ylo = (int64_t)floor(lo_y), yhi = (int64_t)floor(hi_y) + 2;
                int cx0, cx1, cy0, cy1;
                if (!cell_span(xlo, xhi, c.x0, c.x1, c.cell_log2, &cx0, &cx1) ||
                    !cell_span(ylo, yhi, c.y0, c.y1, c.cell_log2, &cy0, &cy1))
                    continue;
                for (int cy = cy0; cy <= cy1; ++cy) {
                    const int64_t base = ((int64_t)e * c.ncy + cy) * c.ncx;
                    const int32_t j1 = c.off[base + cx1 + 1];
                    for (int32_t j = c.off[base + cx0]; j < j1; ++j) {
                        const int2 p = c.sxy[j];
                        const int32_t xq = a.weighted ? (p.x >> 8) : p.x;
                        const double ex = (double)xq / 256.0 - px, ey = (double)p.y / 256.0 - py;
                        if (ex * ex + ey * ey <= r2max) {
                            const int q = atomicAdd(&sh.n_nxt, 1);
                            if (q < kMaxPoints) sh.tmp[q] = c.sidx[j];
                        }
                    }
                }
            }
            __syncthreads();
            n_g = sh.n_nxt;
            if (n_g > kMaxPoints) {
                res.status = SAS_REFINE_TOO_LARGE;
                break;
            }
            sort_into(sh.tmp, n_g, sh.nxt);
            __syncthreads();
            // Step 6: stop when the gathered set is the set just fitted
            bool same = n_g == n;
            if (same) {
                int diff = 0;
                for (int i = tid; i < n; i += RT) diff |= sh.nxt[i] != sh.cur[i];
                same = __syncthreads_or(diff) == 0;
            }
            __syncthreads();
            for (int i = tid; i < n_g; i += RT) sh.cur[i] = sh.nxt[i];
            n = n_g;
            if (same) {
                res.status = SAS_REFINE_CONVERGED;
                break;
            }
            res.status = SAS_REFINE_MAX_ROUNDS;
        }
        __syncthreads();
        res.n_gathered = n_g;
        if (res.rounds > 0 && a.gathered) {
            const int m = min(n_g, min(kMaxPoints, a.gather_cap));
            for (int i = tid; i < m; i += RT) a.gathered[cl * (int64_t)a.gather_cap + i] = sh.cur[i];
        }
        if (tid == 0) a.out[cl] = res;
    }
}

}  // namespace

hipError_t launch_refine_clusters(const RefineArgs &a, hipStream_t stream) {
    if (a.n_clusters <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(a.n_clusters < 4096 ? a.n_clusters : 4096);
    hipLaunchKernelGGL(k_refine_clusters, dim3(grid), dim3(RT), 0, stream, a);
    return hipGetLastError();
}

}  // namespace sas

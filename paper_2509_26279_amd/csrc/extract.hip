// Greedy cluster extraction (Step 3 of Sec. 2.1) on the GPU.
//
// The vote reports every (velocity, bin) at or above N_min.  Step 3 takes
// the maximum cell, calls the points that contributed to it a cluster,
// removes them from every cell they counted in, and repeats while the
// maximum still reaches N_min.  Counts only fall, so the loop runs over the
// reported cells; ties of the maximum go to the smaller (v_idx, by, bx).
//
//   1. k_contrib: one wave per reported cell gathers its contributors (the
//      detections whose exact Step-2 bin at the cell's velocity is the
//      cell) through the window index, as the vote does: lanes take epochs,
//      a wave scan places each lane's contributors.  A first pass counts,
//      a scan lays the cells' lists out, a second pass writes the sorted
//      positions of the contributors and their epochs.
//   2. an inverse index (detection -> cells that hold it) by counting sort,
//      and every cell's count (one wave per cell: distinct epochs through a
//      256-bit mask in LDS, or the number of live contributors);
//   3. parallel rounds: a cell whose key (count, then the tie rule) beats
//      every open cell sharing a live detection with it is taken by the
//      sequential loop too, with exactly its current contributors - counts
//      only fall, so no neighbour can overtake it, and what is taken
//      elsewhere meanwhile shares none of its detections.  Each round takes
//      all such local maxima at once (every detection keeps the best open
//      cell holding it; a cell is a local maximum when it is the best of all
//      its live detections), removes their detections and recounts;
//   4. k_greedy: one workgroup finishes whatever the rounds left, one take at
//      a time.  Each step a block reduction finds the maximum of the stored
//      counts under the tie rule (cells below N_min close), the maximum's
//      live contributors are taken and every open cell that held one of
//      them is queued; only the queued cells are recounted (one wave each);
//   5. the keys taken by the sequential loop strictly increase (counts only
//      fall and the tie rule is total), so ranking the clusters by key
//      restores its order; the owners are renumbered to that order.
#include <algorithm>

#include "internal.h"

namespace sas {
namespace {

constexpr int CT = 256;    // threads per gather block (4 cells at a time)
constexpr int GT = 1024;   // threads of the greedy workgroup
constexpr int GW = GT / 64;

__device__ inline int32_t shift_q8(int32_t v, int32_t d) {
    return (int32_t)(((int64_t)v * (int64_t)d + 65535) >> 16);
}

__device__ inline bool cell_span(int64_t lo, int64_t hi, int32_t f0, int32_t f1, int cl, int *c0,
                                 int *c1) {
    if (hi <= f0 || lo >= f1) return false;
    *c0 = (int)((max(lo, (int64_t)f0) - f0) >> cl);
    *c1 = (int)((min(hi, (int64_t)f1) - 1 - f0) >> cl);
    return true;
}

__device__ inline int32_t wave_excl(int32_t v, int32_t *total) {
    const int lane = __lane_id();
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    *total = __shfl(incl, 63, 64);
    return incl - v;
}

// Contributors of cell k in the lane's epochs e = lane, lane + 64, ...:
// counted (WRITE = false) or written from position at (WRITE = true).
template <bool WRITE>
__device__ int32_t lane_contributors(const ExtractArgs &a, const sas_candidate &cd,
                                     int32_t cell, int32_t at) {
    const PreparedCatalog &c = a.cat;
    const int lane = __lane_id();
    const int lb = a.log2b;
    const int32_t vx = a.vel[2 * (int64_t)cd.v_idx], vy = a.vel[2 * (int64_t)cd.v_idx + 1];
    int32_t n = 0;
    for (int e = lane; e < c.n_epochs; e += 64) {
        const int32_t d = c.dt[e];
        if (d < 0) continue;
        const int64_t xlo = ((int64_t)cd.bx << lb) + shift_q8(vx, d);
        const int64_t ylo = ((int64_t)cd.by << lb) + shift_q8(vy, d);
        const int64_t xhi = xlo + ((int64_t)1 << lb), yhi = ylo + ((int64_t)1 << lb);
        int cx0, cx1, cy0, cy1;
        if (!cell_span(xlo, xhi, c.x0, c.x1, c.cell_log2, &cx0, &cx1) ||
            !cell_span(ylo, yhi, c.y0, c.y1, c.cell_log2, &cy0, &cy1))
            continue;
        for (int cy = cy0; cy <= cy1; ++cy) {
            const int64_t base = ((int64_t)e * c.ncy + cy) * c.ncx;
            const int32_t j1 = c.off[base + cx1 + 1];
            for (int32_t j = c.off[base + cx0]; j < j1; ++j) {
                const int2 p = c.sxy[j];
                if (p.x < xlo || p.x >= xhi || p.y < ylo || p.y >= yhi) continue;
                if (WRITE) {
                    a.member[at + n] = j;
                    a.member_epoch[at + n] = (uint8_t)e;
                    a.member_cell[at + n] = cell;
                }
                ++n;
            }
        }
    }
    return n;
}

__global__ void __launch_bounds__(CT) k_contrib(ExtractArgs a, int write) {
    const int lane = __lane_id();
    const int64_t wave_id = ((int64_t)blockIdx.x * CT + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * CT) >> 6;
    for (int64_t k = wave_id; k < a.n_cand; k += n_waves) {
        const sas_candidate cd = a.cand[k];
        if (!write) {
            int32_t total;
            wave_excl(lane_contributors<false>(a, cd, (int32_t)k, 0), &total);
            if (lane == 0) a.first[k] = total;  // scanned into offsets afterwards
        } else {
            const int32_t mine = lane_contributors<false>(a, cd, (int32_t)k, 0);
            int32_t total;
            const int32_t pre = wave_excl(mine, &total);
            const int64_t at = a.first[k] + pre;
            if (a.first[a.n_cand] <= a.member_cap)  // all lists fit
                lane_contributors<true>(a, cd, (int32_t)k, (int32_t)at);
        }
    }
}

// (count, v_idx, by, bx) order of the maximum: larger count, then smaller
// v_idx, by, bx.
struct Best {
    int32_t count, k;
    uint32_t v;
    int32_t by, bx;
};

__device__ inline bool better(const Best &p, const Best &q) {
    if (p.k < 0) return false;
    if (q.k < 0) return true;
    if (p.count != q.count) return p.count > q.count;
    if (p.v != q.v) return p.v < q.v;
    if (p.by != q.by) return p.by < q.by;
    return p.bx < q.bx;
}

__device__ inline Best shfl_best(const Best &b, int src) {
    Best o;
    o.count = __shfl(b.count, src, 64);
    o.k = __shfl(b.k, src, 64);
    o.v = (uint32_t)__shfl((int32_t)b.v, src, 64);
    o.by = __shfl(b.by, src, 64);
    o.bx = __shfl(b.bx, src, 64);
    return o;
}

// Whether the contributor lists fit (all kernels after the lists read it).
__device__ inline bool lists_fit(const ExtractArgs &a) {
    return a.first[a.n_cand] <= a.member_cap;
}

// Per-detection state and the inverse index counts, cleared.
__global__ void k_inv_init(ExtractArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = t0; j <= a.n; j += stride) a.inv_first[j] = 0;
    for (int64_t j = t0; j < a.n; j += stride) {
        a.inv_cursor[j] = 0;
        a.live[j] = 1;
        a.best[j] = -1;
        a.cluster_of[j] = -1;
    }
    if (t0 < kExtractCounters) a.counters[t0] = 0;
    for (int64_t k = t0; k < a.n_cand; k += stride) {
        a.open[k] = 1;
        a.dirty[k] = 0;
    }
}

__global__ void k_inv_count(ExtractArgs a) {
    if (!lists_fit(a)) return;
    const int64_t n_members = a.first[a.n_cand];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < n_members; m += stride)
        atomicAdd(&a.inv_first[a.member[m]], 1);
}

__global__ void k_inv_fill(ExtractArgs a) {
    if (!lists_fit(a)) return;
    const int64_t n_members = a.first[a.n_cand];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < n_members; m += stride) {
        const int32_t j = a.member[m];
        a.inv[a.inv_first[j] + atomicAdd(&a.inv_cursor[j], 1)] = a.member_cell[m];
    }
}

// Count of cell k over its live contributors, by one wave (wave uniform);
// wmask: 8 words of LDS for this wave.
__device__ int32_t recount(const ExtractArgs &a, int64_t k, uint32_t *wmask) {
    const int lane = __lane_id();
    if (lane < kSlotWords) wmask[lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t f = a.first[k], l = a.first[k + 1];
    int32_t n = 0;
    for (int32_t m = f + lane; m < l; m += 64) {
        if (!a.live[a.member[m]]) continue;
        if (a.mode_epochs) {
            const uint32_t e = a.member_epoch[m];
            atomicOr(&wmask[e >> 5], 1u << (e & 31));
        } else {
            ++n;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (a.mode_epochs) n = lane < kSlotWords ? __popc(wmask[lane]) : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    return n;
}

__global__ void __launch_bounds__(CT) k_count_all(ExtractArgs a) {
    __shared__ uint32_t wmask[CT / 64][kSlotWords];
    if (!lists_fit(a)) return;
    const int wave = threadIdx.x >> 6;
    const int64_t wave_id = ((int64_t)blockIdx.x * CT + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * CT) >> 6;
    for (int64_t k = wave_id; k < a.n_cand; k += n_waves) {
        const int32_t n = recount(a, k, wmask[wave]);
        if (__lane_id() == 0) {
            a.count[k] = n;
            if (n < a.n_min)
                a.open[k] = 0;
            else
                atomicAdd(&a.counters[2], 1);
        }
    }
}

// Whether cell k beats cell c (c < 0: no cell) under the order of the
// maximum: larger count, then smaller v_idx, by, bx.
__device__ inline bool cell_better(const ExtractArgs &a, int32_t k, int32_t c) {
    if (c < 0) return true;
    const int32_t ck = a.count[k], cc = a.count[c];
    if (ck != cc) return ck > cc;
    const sas_candidate &p = a.cand[k], &q = a.cand[c];
    if (p.v_idx != q.v_idx) return p.v_idx < q.v_idx;
    if (p.by != q.by) return p.by < q.by;
    return p.bx < q.bx;
}

// A parallel round may run: the lists fit and the previous round left an
// open cell.
__device__ inline bool round_active(const ExtractArgs &a, int r) {
    return lists_fit(a) && a.counters[2 + r - 1] > 0;
}

#define FOR_CELLS(k)                                                                    \
    const int64_t wave_id = ((int64_t)blockIdx.x * CT + threadIdx.x) >> 6;             \
    const int64_t n_waves = ((int64_t)gridDim.x * CT) >> 6;                              \
    for (int64_t k = wave_id; k < a.n_cand; k += n_waves)

// Round r, step 1: every live detection of an open cell keeps the best
// open cell holding it (compare-and-swap until it holds the better one).
__global__ void __launch_bounds__(CT) k_round_best(ExtractArgs a, int r) {
    if (!round_active(a, r)) return;
    FOR_CELLS(k) {
        if (a.open[k] != 1) continue;  // wave uniform
        for (int32_t m = a.first[k] + __lane_id(); m < a.first[k + 1]; m += 64) {
            const int32_t j = a.member[m];
            if (!a.live[j]) continue;
            int32_t cur = a.best[j];
            while (cell_better(a, (int32_t)k, cur)) {
                const int32_t old = atomicCAS(&a.best[j], cur, (int32_t)k);
                if (old == cur) break;
                cur = old;
            }
        }
    }
}

// Step 2: a cell that is the best of all its live detections is taken.
__global__ void __launch_bounds__(CT) k_round_take(ExtractArgs a, int r) {
    if (!round_active(a, r)) return;
    FOR_CELLS(k) {
        if (a.open[k] != 1) continue;
        bool mine = true;
        for (int32_t m = a.first[k] + __lane_id(); m < a.first[k + 1]; m += 64) {
            const int32_t j = a.member[m];
            if (a.live[j] && a.best[j] != (int32_t)k) mine = false;
        }
        if (__all(mine) && __lane_id() == 0) {
            const int32_t s = atomicAdd(&a.counters[0], 1);
            a.slot[k] = s;
            a.taken[s] = (int32_t)k;
            a.open[k] = 2;
        }
    }
}

// Step 3: the taken cells' live detections leave (their live sets are
// disjoint: a detection has one best cell).
__global__ void __launch_bounds__(CT) k_round_kill(ExtractArgs a, int r) {
    if (!round_active(a, r)) return;
    FOR_CELLS(k) {
        if (a.open[k] != 2) continue;
        const int32_t s = a.slot[k];
        for (int32_t m = a.first[k] + __lane_id(); m < a.first[k + 1]; m += 64) {
            const int32_t j = a.member[m];
            if (!a.live[j]) continue;
            a.cluster_of[a.cat.sidx[j]] = s;
            a.live[j] = 0;
        }
        if (__lane_id() == 0) a.open[k] = 0;
    }
}

// Step 4: recount the open cells, close those below N_min, count the rest,
// and clear the best cell of their live detections for the next round.
__global__ void __launch_bounds__(CT) k_round_recount(ExtractArgs a, int r) {
    __shared__ uint32_t wmask[CT / 64][kSlotWords];
    if (!round_active(a, r)) return;
    const int wave = threadIdx.x >> 6;
    FOR_CELLS(k) {
        if (a.open[k] != 1) continue;
        const int32_t n = recount(a, k, wmask[wave]);
        if (__lane_id() == 0) {
            a.count[k] = n;
            if (n < a.n_min)
                a.open[k] = 0;
            else
                atomicAdd(&a.counters[2 + r], 1);
        }
        for (int32_t m = a.first[k] + __lane_id(); m < a.first[k + 1]; m += 64)
            a.best[a.member[m]] = -1;
    }
}

constexpr int kQueueCap = 4096;  // cells recounted after one take

__global__ void __launch_bounds__(GT) k_greedy(ExtractArgs a) {
    __shared__ uint32_t wmask[GW][kSlotWords];
    __shared__ int32_t queue[kQueueCap];
    __shared__ int32_t queue_n;
    __shared__ Best wbest[GW];
    __shared__ Best best_all;
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    if (!lists_fit(a)) return;  // reported by k_finish
    int32_t n_out = a.counters[0];  // clusters taken by the parallel rounds
    for (;;) {
        // the maximum of the stored counts; cells below N_min close
        Best mine{0, -1, 0, 0, 0};
        for (int64_t k = tid; k < a.n_cand; k += GT) {
            if (!a.open[k]) continue;
            const int32_t cnt = a.count[k];
            if (cnt < a.n_min) {
                a.open[k] = 0;
                continue;
            }
            if (cnt < mine.count) continue;
            const sas_candidate cd = a.cand[k];
            const Best b{cnt, (int32_t)k, cd.v_idx, cd.by, cd.bx};
            if (better(b, mine)) mine = b;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const Best other = shfl_best(mine, lane ^ o);
            if (better(other, mine)) mine = other;
        }
        if (lane == 0) wbest[wave] = mine;
        __syncthreads();
        if (tid == 0) {
            Best b = wbest[0];
            for (int w = 1; w < GW; ++w)
                if (better(wbest[w], b)) b = wbest[w];
            best_all = b;
            queue_n = 0;
        }
        __syncthreads();
        const Best b = best_all;
        if (b.k < 0) break;  // block uniform
        if (tid == 0) {
            a.taken[n_out] = b.k;
            a.open[b.k] = 0;
        }
        // take its live contributors; queue the open cells that held them
        const int32_t f = a.first[b.k], l = a.first[b.k + 1];
        for (int32_t m = f + tid; m < l; m += GT) {
            const int32_t j = a.member[m];
            if (!a.live[j]) continue;
            a.cluster_of[a.cat.sidx[j]] = (int32_t)n_out;
            for (int32_t i = a.inv_first[j]; i < a.inv_first[j + 1]; ++i) {
                const int32_t c = a.inv[i];
                if (c == b.k || !a.open[c]) continue;
                if (atomicExch(&a.dirty[c], 1u) == 0u) {
                    const int32_t q = atomicAdd(&queue_n, 1);
                    if (q < kQueueCap) queue[q] = c;
                }
            }
        }
        __syncthreads();  // every mark reads live before it drops
        for (int32_t m = f + tid; m < l; m += GT) a.live[a.member[m]] = 0;
        __syncthreads();
        // recount the queued cells (all open cells if the queue overflowed)
        const int32_t nq = queue_n;
        if (nq <= kQueueCap) {
            for (int32_t q = wave; q < nq; q += GW) {
                const int32_t c = queue[q];
                const int32_t n = recount(a, c, wmask[wave]);
                if (lane == 0) {
                    a.count[c] = n;
                    a.dirty[c] = 0;
                }
            }
        } else {
            for (int64_t c = wave; c < a.n_cand; c += GW) {
                if (!a.open[c]) continue;  // wave uniform
                const int32_t n = recount(a, c, wmask[wave]);
                if (lane == 0) {
                    a.count[c] = n;
                    a.dirty[c] = 0;
                }
            }
        }
        ++n_out;
        __syncthreads();
    }
    if (tid == 0) a.counters[1] = n_out;
}

// Key of a taken cell for the extraction order: (count at the take, v_idx,
// by, bx); a beats b when its count is larger, then its v_idx, by, bx smaller.
struct Key {
    int32_t count;
    uint32_t v;
    int32_t by, bx;
};

__device__ inline Key key_of(const ExtractArgs &a, int32_t k) {
    const sas_candidate cd = a.cand[k];
    return Key{a.count[k], cd.v_idx, cd.by, cd.bx};
}

__device__ inline bool key_before(const Key &p, const Key &q) {
    if (p.count != q.count) return p.count > q.count;
    if (p.v != q.v) return p.v < q.v;
    if (p.by != q.by) return p.by < q.by;
    return p.bx < q.bx;
}

constexpr int kRankTile = 1024;  // keys staged in LDS at a time

// Extraction order: the rank of each cluster's key among all clusters (keys
// are distinct); the records in that order.  The keys are walked in tiles
// staged in LDS.
__global__ void __launch_bounds__(256) k_rank(ExtractArgs a) {
    __shared__ Key tile[kRankTile];
    if (!lists_fit(a)) return;
    const int32_t total = a.counters[1];
    const uint32_t sat = (uint32_t)a.count_sat;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x; c0 < total; c0 += stride) {
        const int64_t c = c0 + threadIdx.x;  // block uniform loop, per-thread cluster
        const int32_t k = c < total ? a.taken[c] : 0;
        const Key mine = key_of(a, k);
        int32_t r = 0;
        for (int32_t d0 = 0; d0 < total; d0 += kRankTile) {
            const int32_t nd = min(kRankTile, total - d0);
            __syncthreads();
            for (int32_t i = threadIdx.x; i < nd; i += blockDim.x) tile[i] = key_of(a, a.taken[d0 + i]);
            __syncthreads();
            for (int32_t i = 0; i < nd; ++i) r += key_before(tile[i], mine) ? 1 : 0;
        }
        if (c >= total) continue;
        a.perm[c] = r;
        if (r < a.cluster_cap) {
            const sas_candidate cd = a.cand[k];
            const uint32_t cnt = (uint32_t)a.count[k];  // its count when taken
            uint4 rec;
            rec.x = cd.v_idx;
            rec.y = (uint32_t)cd.bx;
            rec.z = (uint32_t)cd.by;
            rec.w = (cnt > sat ? sat : cnt) | ((cnt > sat ? 1u : 0u) << 16);
            *(uint4 *)(a.clusters + r) = rec;
        }
    }
}

__global__ void k_renumber(ExtractArgs a) {
    if (!lists_fit(a)) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const int32_t c = a.cluster_of[i];
        if (c >= 0) a.cluster_of[i] = a.perm[c];
    }
}

__global__ void k_finish(ExtractArgs a) {
    const int64_t n_members = a.first[a.n_cand];
    if (n_members > a.member_cap) {  // the lists did not fit: nothing was extracted
        a.res->n_clusters = 0;
        a.res->n_members = n_members;
        a.res->status = SAS_EXTRACT_MEMBERS_FULL;
        return;
    }
    const int32_t total = a.counters[1];
    a.res->n_clusters = total;
    a.res->n_members = n_members;
    a.res->status = total > a.cluster_cap ? SAS_EXTRACT_CLUSTERS_FULL : 0;
}

__global__ void k_contrib_tail(int32_t *first, int64_t n_cand) { first[n_cand] = 0; }

}  // namespace

hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream) {
    const unsigned init_blocks = (unsigned)std::min<int64_t>(
        (std::max(a.n + 1, a.n_cand) + 255) / 256, 4096);
    hipLaunchKernelGGL(k_inv_init, dim3(init_blocks), dim3(256), 0, stream, a);
    const unsigned cell_blocks =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.n_cand + CT / 64 - 1) / (CT / 64),
                                                         65536));
    if (a.n_cand > 0)
        hipLaunchKernelGGL(k_contrib, dim3(cell_blocks), dim3(CT), 0, stream, a, 0);
    // first[n_cand] must read 0 before the scan turns counts into offsets
    hipLaunchKernelGGL(k_contrib_tail, dim3(1), dim3(1), 0, stream, a.first, a.n_cand);
    hipError_t e = launch_scan_exclusive(a.first, a.n_cand + 1, a.scan_blocksum, stream);
    if (e != hipSuccess) return e;
    if (a.n_cand > 0) {
        hipLaunchKernelGGL(k_contrib, dim3(cell_blocks), dim3(CT), 0, stream, a, 1);
        hipLaunchKernelGGL(k_inv_count, dim3(2048), dim3(256), 0, stream, a);
        e = launch_scan_exclusive(a.inv_first, a.n + 1, a.inv_blocksum, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_inv_fill, dim3(2048), dim3(256), 0, stream, a);
        hipLaunchKernelGGL(k_count_all, dim3(cell_blocks), dim3(CT), 0, stream, a);
        for (int r = 1; r <= a.rounds; ++r) {
            hipLaunchKernelGGL(k_round_best, dim3(cell_blocks), dim3(CT), 0, stream, a, r);
            hipLaunchKernelGGL(k_round_take, dim3(cell_blocks), dim3(CT), 0, stream, a, r);
            hipLaunchKernelGGL(k_round_kill, dim3(cell_blocks), dim3(CT), 0, stream, a, r);
            hipLaunchKernelGGL(k_round_recount, dim3(cell_blocks), dim3(CT), 0, stream, a, r);
        }
    }
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(GT), 0, stream, a);
    const unsigned rank_blocks =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>((a.n_cand + 255) / 256, 4096));
    hipLaunchKernelGGL(k_rank, dim3(rank_blocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_renumber, dim3(init_blocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, stream, a);
    return hipGetLastError();
}

}  // namespace sas

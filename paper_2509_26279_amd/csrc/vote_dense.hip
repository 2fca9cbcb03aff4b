// Dense LDS voting path for gfx950.
//
// Steps 1-2 of Sec. 2.1 (Project, Cluster) with the Step-3 threshold, for one
// work item = (velocity block, spatial tile of TX x TY bins).  A workgroup
//   1. computes, per epoch, the window of the original frame whose
//      detections can project into its tile for some velocity of its block
//      (the shift v * (t_e - t0) of every block member lies between the
//      block's extreme velocities), and gathers those detections from the
//      window index into registers (up to kVoteKmax per thread);
//   2. for every velocity of the block, projects each detection to the
//      reference epoch and bins it (bx = floor(X / (65536 b)) with X the
//      exact Q24 position), votes into an LDS tile with one atomic per
//      vote, and uses the atomic's return value to find the unique vote that
//      lifts a bin to N_min (no scan of the tile is needed);
//   3. emits the lifted bins with a wavefront ballot and one global atomic
//      per wave, then clears what it wrote.
//
// Tile variants:
//   kMask32  - EPOCHS with E <= 32: each bin is an epoch bitmask (atomic OR);
//              the lifting vote is the one that sets the N_min-th bit.
//   kCountDet - DETECTIONS: each bin is a counter (atomic add).
//   kCountEpo - EPOCHS with E > 32: a counter per bin flags every bin that
//              holds >= N_min detections (a superset of the answer); the
//              flagged bins are then tagged and the detections voting into
//              them OR their epochs into per-bin masks, giving the exact
//              number of distinct epochs.
// Detections beyond the register capacity are processed in chunks that are
// reloaded per velocity (correct for any catalog, slower).
#include "internal.h"

namespace sas {
namespace {

constexpr int T = kVoteThreads;
constexpr int K = kVoteKmax;
constexpr int kSlotWords = kMaxEpochs / 32;

struct Shared {
    int32_t prefix[kMaxEpochs + 1];
    int32_t rows[kMaxEpochs];  // cy0 | cy1 << 16   (cy0 > cy1: empty)
    int32_t cols[kMaxEpochs];  // cx0 | cx1 << 16
    int32_t dt[kMaxEpochs];
    int32_t wsum[T / 64];
    int32_t nflag;
};

__device__ inline int32_t bin_of(int32_t rel_q8, int32_t v, int32_t d, int sh) {
    const int64_t p = ((int64_t)rel_q8 << 16) - (int64_t)v * (int64_t)d;
    return (int32_t)(p >> sh);
}

// One candidate per participating lane; all lanes of the wave must call.
__device__ inline void emit(bool ok, uint32_t v_idx, int32_t bx, int32_t by, uint32_t cnt,
                            const DenseArgs &a) {
    const uint64_t mask = __ballot(ok);
    if (mask == 0) return;
    const int lane = __lane_id();
    unsigned long long base = 0;
    if (lane == 0)
        base = atomicAdd((unsigned long long *)&a.res->n_cand, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, 64);
    if (ok) {
        const uint32_t pre = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const int64_t idx = (int64_t)base + pre;
        if (idx < a.cand_cap) {
            const uint32_t sat = (uint32_t)a.count_sat;
            uint4 rec;
            rec.x = v_idx;
            rec.y = (uint32_t)bx;
            rec.z = (uint32_t)by;
            rec.w = (cnt > sat ? sat : cnt) | ((cnt > sat ? 1u : 0u) << 16);
            *(uint4 *)(a.cand + idx) = rec;
        }
    }
}

// Exclusive scan over the T threads of the block.
__device__ inline int32_t scan_block(int32_t v, int32_t *total, Shared &sh) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) sh.wsum[wave] = incl;
    __syncthreads();
    int32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) {
        const int32_t s = sh.wsum[w];
        off += (w < wave) ? s : 0;
        tot += s;
    }
    *total = tot;
    return off + incl - v;
}

// Registers holding the detections of one chunk of the item's window.
struct Held {
    int32_t xr[K];  // x - tile origin, Q8
    int32_t yr[K];
    int32_t d[K];   // t_e - t0, Q16 h
    int32_t e[K];
    int32_t cnt;
};

__device__ inline void load_chunk(int q, int32_t M, const PreparedCatalog &c, const Shared &sh,
                                  int64_t ox, int64_t oy, Held &h) {
    const int32_t mq = min(kVoteCap, M - q * kVoteCap);
    const int32_t per = (mq + T - 1) / T;
    const int32_t p0 = q * kVoteCap + (int32_t)threadIdx.x * per;
    const int32_t p1 = min(q * kVoteCap + mq, p0 + per);
    h.cnt = max(0, p1 - p0);
    if (h.cnt == 0) return;
    const int E = c.n_epochs;
    // epoch holding element p0: the last e with prefix[e] <= p0
    int lo = 0, hi = E - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.prefix[mid] <= p0) lo = mid; else hi = mid - 1;
    }
    int e = lo;
    int32_t r = p0 - sh.prefix[e];
    int cy = sh.rows[e] & 0xffff, cy1 = sh.rows[e] >> 16;
    int cx0 = sh.cols[e] & 0xffff, cx1 = sh.cols[e] >> 16;
    int64_t base = ((int64_t)e * c.ncy + cy) * c.ncx;
    int32_t pos = c.off[base + cx0], rend = c.off[base + cx1 + 1];
    while (r >= rend - pos && cy < cy1) {
        r -= rend - pos;
        ++cy;
        base = ((int64_t)e * c.ncy + cy) * c.ncx;
        pos = c.off[base + cx0];
        rend = c.off[base + cx1 + 1];
    }
    pos += r;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k < h.cnt) {
            while (pos >= rend) {  // next non-empty row of the window
                ++cy;
                while (cy > cy1 && e < E - 1) {
                    ++e;
                    cy = sh.rows[e] & 0xffff;
                    cy1 = sh.rows[e] >> 16;
                    cx0 = sh.cols[e] & 0xffff;
                    cx1 = sh.cols[e] >> 16;
                }
                if (cy > cy1) { h.cnt = k; break; }  // unreachable for consistent tables
                base = ((int64_t)e * c.ncy + cy) * c.ncx;
                pos = c.off[base + cx0];
                rend = c.off[base + cx1 + 1];
            }
            if (k < h.cnt) {
                h.xr[k] = (int32_t)((int64_t)c.sx[pos] - ox);
                h.yr[k] = (int32_t)((int64_t)c.sy[pos] - oy);
                h.d[k] = sh.dt[e];
                h.e[k] = e;
                ++pos;
            }
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(T) k_vote_dense(DenseArgs a) {
    extern __shared__ uint32_t smem[];
    __shared__ Shared sh;
    const int TX = a.tile_x, TY = a.tile_y, TB = TX * TY;
    uint32_t *tile = smem;
    int32_t *flags = (int32_t *)(smem + TB);
    uint32_t *slots = smem + 2 * TB;
    const int tid = threadIdx.x;
    const PreparedCatalog &c = a.cat;
    const int E = c.n_epochs;
    const int shf = a.shift;

    const int64_t item = blockIdx.x;
    const int32_t blk = a.items[3 * item];
    const int32_t tx0 = a.items[3 * item + 1];
    const int32_t ty0 = a.items[3 * item + 2];
    const int32_t vx_lo = a.block_vr[4 * blk], vx_hi = a.block_vr[4 * blk + 1];
    const int32_t vy_lo = a.block_vr[4 * blk + 2], vy_hi = a.block_vr[4 * blk + 3];
    const int64_t B = (int64_t)1 << shf;          // bin width in Q24
    const int64_t ox = ((int64_t)tx0 * B) >> 16;  // tile origin in Q8 (exact: B is a multiple of 2^16)
    const int64_t oy = ((int64_t)ty0 * B) >> 16;

    for (int i = tid; i < TB / 4; i += T) ((uint4 *)tile)[i] = make_uint4(0, 0, 0, 0);
    if (tid == 0) sh.nflag = 0;

    // 1. per-epoch windows in the original frame
    int32_t cnt_e = 0;
    if (tid < E) {
        const int32_t d = c.dt[tid];
        sh.dt[tid] = d;
        const int64_t sx_a = (int64_t)vx_lo * d, sx_b = (int64_t)vx_hi * d;
        const int64_t sy_a = (int64_t)vy_lo * d, sy_b = (int64_t)vy_hi * d;
        const int64_t xlo = ((int64_t)tx0 * B + min(sx_a, sx_b)) >> 16;
        const int64_t xhi = (((int64_t)(tx0 + TX) * B + max(sx_a, sx_b)) >> 16) + 1;
        const int64_t ylo = ((int64_t)ty0 * B + min(sy_a, sy_b)) >> 16;
        const int64_t yhi = (((int64_t)(ty0 + TY) * B + max(sy_a, sy_b)) >> 16) + 1;
        int32_t rows = 1, cols = 0;  // empty
        if (xhi > c.x0 && xlo < c.x1 && yhi > c.y0 && ylo < c.y1) {
            const int cx0 = (int)((max(xlo, (int64_t)c.x0) - c.x0) >> c.cell_log2);
            const int cx1 = min(c.ncx - 1, (int)((min(xhi, (int64_t)c.x1) - 1 - c.x0) >> c.cell_log2));
            const int cy0 = (int)((max(ylo, (int64_t)c.y0) - c.y0) >> c.cell_log2);
            const int cy1 = min(c.ncy - 1, (int)((min(yhi, (int64_t)c.y1) - 1 - c.y0) >> c.cell_log2));
            if (cx0 <= cx1 && cy0 <= cy1) {
                for (int cy = cy0; cy <= cy1; ++cy) {
                    const int64_t base = ((int64_t)tid * c.ncy + cy) * c.ncx;
                    cnt_e += c.off[base + cx1 + 1] - c.off[base + cx0];
                }
                rows = cy0 | (cy1 << 16);
                cols = cx0 | (cx1 << 16);
            }
        }
        sh.rows[tid] = rows;
        sh.cols[tid] = cols;
    }
    int32_t M;
    const int32_t ex = scan_block(cnt_e, &M, sh);
    if (tid < E) sh.prefix[tid] = ex;
    if (tid == 0) sh.prefix[E] = M;
    __syncthreads();
    if (M == 0) return;

    const int nchunks = (M + kVoteCap - 1) / kVoteCap;
    const bool sparse_clear = (nchunks == 1) && (2 * M < TB);
    Held h;
    h.cnt = 0;
    if (nchunks == 1) load_chunk(0, M, c, sh, ox, oy, h);

    const int32_t m0 = a.block_start[blk], m1 = a.block_start[blk + 1];
    const uint32_t nmin = (uint32_t)a.n_min;
    for (int m = m0; m < m1; ++m) {
        const int32_t v = a.members[m];
        const int32_t vx = a.vel[2 * v], vy = a.vel[2 * v + 1];

        // 2. vote
        for (int q = 0; q < nchunks; ++q) {
            if (nchunks > 1) load_chunk(q, M, c, sh, ox, oy, h);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < h.cnt) {
                    const int32_t bx = bin_of(h.xr[k], vx, h.d[k], shf);
                    const int32_t by = bin_of(h.yr[k], vy, h.d[k], shf);
                    if ((uint32_t)bx < (uint32_t)TX && (uint32_t)by < (uint32_t)TY) {
                        const int addr = by * TX + bx;
                        bool lifted;
                        if (MODE == kMask32) {
                            const uint32_t bit = 1u << h.e[k];
                            const uint32_t old = atomicOr(&tile[addr], bit);
                            lifted = !(old & bit) && (uint32_t)__popc(old | bit) == nmin;
                        } else {
                            const uint32_t old = atomicAdd(&tile[addr], 1u);
                            lifted = old == nmin - 1;
                        }
                        if (lifted) {
                            const int f = atomicAdd(&sh.nflag, 1);
                            if (f < TB) flags[f] = addr;  // a bin is lifted at most once
                        }
                    }
                }
            }
        }
        __syncthreads();

        // 3. emit the lifted bins
        const int nflag = min(sh.nflag, TB);
        if (nflag > 0) {
            if (MODE != kCountEpo) {
                for (int f0 = 0; f0 < nflag; f0 += T) {
                    const int f = f0 + tid;
                    const bool ok = f < nflag;
                    const int addr = ok ? flags[f] : 0;
                    const uint32_t w = tile[addr];
                    const uint32_t cnt = (MODE == kMask32) ? (uint32_t)__popc(w) : w;
                    emit(ok, (uint32_t)v, tx0 + addr % TX, ty0 + addr / TX, cnt, a);
                }
            } else {
                const int W = (E + 31) >> 5;
                for (int r0 = 0; r0 < nflag; r0 += kSlots) {
                    const int nr = min(kSlots, nflag - r0);
                    for (int s = tid; s < nr; s += T) {
                        tile[flags[r0 + s]] = kTag | (uint32_t)(r0 + s);
                        for (int w = 0; w < kSlotWords; ++w) slots[s * kSlotWords + w] = 0;
                    }
                    __syncthreads();
                    for (int q = 0; q < nchunks; ++q) {
                        if (nchunks > 1) load_chunk(q, M, c, sh, ox, oy, h);
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            if (k < h.cnt) {
                                const int32_t bx = bin_of(h.xr[k], vx, h.d[k], shf);
                                const int32_t by = bin_of(h.yr[k], vy, h.d[k], shf);
                                if ((uint32_t)bx < (uint32_t)TX && (uint32_t)by < (uint32_t)TY) {
                                    const uint32_t w = tile[by * TX + bx];
                                    const int32_t idx = (int32_t)(w & ~kTag);
                                    if ((w & kTag) && idx >= r0 && idx < r0 + nr)
                                        atomicOr(&slots[(idx - r0) * kSlotWords + (h.e[k] >> 5)],
                                                 1u << (h.e[k] & 31));
                                }
                            }
                        }
                    }
                    __syncthreads();
                    for (int s0 = 0; s0 < nr; s0 += T) {
                        const int s = s0 + tid;
                        uint32_t cnt = 0;
                        int addr = 0;
                        if (s < nr) {
                            for (int w = 0; w < W; ++w) cnt += __popc(slots[s * kSlotWords + w]);
                            addr = flags[r0 + s];
                        }
                        emit(s < nr && cnt >= nmin, (uint32_t)v, tx0 + addr % TX,
                             ty0 + addr / TX, cnt, a);
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
        }

        // 4. clear what this velocity wrote
        if (sparse_clear) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < h.cnt) {
                    const int32_t bx = bin_of(h.xr[k], vx, h.d[k], shf);
                    const int32_t by = bin_of(h.yr[k], vy, h.d[k], shf);
                    if ((uint32_t)bx < (uint32_t)TX && (uint32_t)by < (uint32_t)TY)
                        tile[by * TX + bx] = 0;
                }
            }
        } else {
            for (int i = tid; i < TB / 4; i += T) ((uint4 *)tile)[i] = make_uint4(0, 0, 0, 0);
        }
        if (tid == 0) sh.nflag = 0;
        __syncthreads();
    }
}

}  // namespace

size_t dense_lds_bytes(int mode, int tile_x, int tile_y) {
    size_t b = (size_t)2 * tile_x * tile_y * sizeof(uint32_t);
    if (mode == kCountEpo) b += (size_t)kSlots * kSlotWords * sizeof(uint32_t);
    return b;
}

hipError_t launch_vote_dense(int mode, const DenseArgs &a, hipStream_t stream) {
    if (a.n_items <= 0) return hipSuccess;
    const size_t lds = dense_lds_bytes(mode, a.tile_x, a.tile_y);
    const dim3 grid((unsigned)a.n_items), block(T);
    switch (mode) {
    case kMask32:
        hipLaunchKernelGGL(k_vote_dense<kMask32>, grid, block, lds, stream, a);
        break;
    case kCountDet:
        hipLaunchKernelGGL(k_vote_dense<kCountDet>, grid, block, lds, stream, a);
        break;
    default:
        hipLaunchKernelGGL(k_vote_dense<kCountEpo>, grid, block, lds, stream, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace sas

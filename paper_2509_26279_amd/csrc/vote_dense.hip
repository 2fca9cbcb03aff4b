// Dense LDS voting path for gfx950.
//
// Steps 1-2 of Sec. 2.1 (Project, Cluster) with the Step-3 threshold.  The
// velocity grid is cut into segments of up to 32 velocities (8 x 4 lattice
// blocks).  A workgroup takes a (segment, tile of TX x TY bins) and keeps
// an LDS histogram of every (bin, velocity) cell, laid out [bin][32]:
//   1. per epoch, the window of the original frame whose detections can land
//      in the tile for some velocity of the segment is looked up in the window
//      index and staged in LDS (tile-relative Q8 coordinates, epoch order);
//   2. each wave takes epochs; lanes 0-31 and 32-63 carry the segment's 32
//      velocities and vote two staged detections per instruction.  With
//      d = t_e - t0 and S(v) = ceil(v d / 65536), the exact bin of Step 2
//      floor((65536 x - v d) / (65536 b)) equals (x - S(v)) >> log2(b): one
//      32-bit subtract and shift per axis; S is computed once per (lane,
//      epoch).  A bin's 32 velocities are 32 consecutive words, so an atomic
//      of a wave touches every LDS bank exactly twice;
//   3. the atomic's return value identifies the unique vote that lifts a cell
//      to N_min; lifted cells are emitted with a wavefront ballot and one
//      global atomic per wave, or queued for refinement (below).
// Cell variants:
//   kMask32  - EPOCHS with E <= 32: epoch bitmask per cell, emitted directly;
//   kCountDet - DETECTIONS: counter per cell, emitted directly;
//   kCountRef - counter of detections per cell as a filter: a bin can hold
//               N_min distinct epochs (or detections) only if its cell holds
//               N_min detections.  Used for EPOCHS with E > 32 and for coarse
//               cells of 2^m x 2^m bins (sparse catalogs: far fewer cells per
//               vote); lifted cells go to a list that k_refine resolves into
//               exact bins.
#include "internal.h"

namespace sas {
namespace {

constexpr int T = kVoteThreads;

struct Shared {
    int32_t dt[kMaxEpochs];
    int32_t sp[kMaxEpochs + 1];  // first window index of each epoch
    int32_t rows[kMaxEpochs];    // cy0 | cy1 << 16   (cy0 > cy1: empty)
    int32_t cols[kMaxEpochs];    // cx0 | cx1 << 16
    int32_t wsum[T / 64];
    int32_t sv[kLanes];          // segment: v_idx of each lane (-1: unused)
    int32_t svx[kLanes];         // segment: velocity of each lane
    int32_t svy[kLanes];
    int32_t nflag;
    int32_t max_rows;
};

// ceil(v * d / 65536) for d >= 0: the shift v (t_e - t0) in Q8 pixels,
// rounded so that the floor of the shifted position is exact.
__device__ inline int32_t shift_q8(int32_t v, int32_t d) {
    return (int32_t)(((int64_t)v * (int64_t)d + 65535) >> 16);
}

__device__ inline void write_cand(sas_candidate *cand, int64_t idx, uint32_t v_idx, int32_t bx,
                                  int32_t by, uint32_t cnt, uint32_t sat) {
    uint4 rec;
    rec.x = v_idx;
    rec.y = (uint32_t)bx;
    rec.z = (uint32_t)by;
    rec.w = (cnt > sat ? sat : cnt) | ((cnt > sat ? 1u : 0u) << 16);
    *(uint4 *)(cand + idx) = rec;
}

// Wave-aggregated append: one global atomic per wave; returns the slot of
// this lane (valid when ok).  All lanes of the wave must call.
__device__ inline int64_t wave_append(bool ok, unsigned long long *counter, bool *any) {
    const uint64_t mask = __ballot(ok);
    *any = mask != 0;
    if (mask == 0) return 0;
    unsigned long long base = 0;
    if (__lane_id() == 0) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, 64);
    const uint32_t pre = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    return (int64_t)base + pre;
}

__device__ inline void emit(bool ok, uint32_t v_idx, int32_t bx, int32_t by, uint32_t cnt,
                            sas_candidate *cand, int64_t cap, sas_vote_result *res, int count_sat) {
    bool any;
    const int64_t idx = wave_append(ok, (unsigned long long *)&res->n_cand, &any);
    if (ok && idx < cap) write_cand(cand, idx, v_idx, bx, by, cnt, (uint32_t)count_sat);
}

// Exclusive scan over the T threads of the block; *total gets the sum.
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

struct Tile {
    int32_t tx0, ty0;  // first cell-bin
    int64_t ox, oy;    // origin, Q8
    int32_t vx_lo, vx_hi, vy_lo, vy_hi;
};

// Cell rows/columns of the window index that an axis interval [lo, hi) of
// Q8 positions touches, clamped to the footprint; false when none.
__device__ inline bool cell_span(int64_t lo, int64_t hi, int32_t f0, int32_t f1, int cl, int *c0,
                                 int *c1) {
    if (hi <= f0 || lo >= f1) return false;
    *c0 = (int)((max(lo, (int64_t)f0) - f0) >> cl);
    *c1 = (int)((min(hi, (int64_t)f1) - 1 - f0) >> cl);
    return true;
}

// Per-epoch windows of the tile in the original frame: cell rows and
// columns, window prefix sh.sp, and the total M (returned, block uniform).
// Ends with a barrier.
__device__ int32_t tile_windows(const DenseArgs &a, const Tile &t, Shared &sh) {
    const PreparedCatalog &c = a.cat;
    const int tid = threadIdx.x;
    const int E = c.n_epochs;
    int32_t cnt_e = 0;
    if (tid == 0) sh.max_rows = 0;
    if (tid < E) {
        const int32_t d = c.dt[tid];
        sh.dt[tid] = d;
        int32_t rows = 1, cols = 0;  // empty
        if (d >= 0) {
            const int kc = a.log2b + a.coarse_log2;
            const int64_t wx = (int64_t)a.tile_x << kc, wy = (int64_t)a.tile_y << kc;
            const int64_t xlo = t.ox + shift_q8(t.vx_lo, d);
            const int64_t xhi = t.ox + shift_q8(t.vx_hi, d) + wx;  // exclusive
            const int64_t ylo = t.oy + shift_q8(t.vy_lo, d);
            const int64_t yhi = t.oy + shift_q8(t.vy_hi, d) + wy;
            int cx0, cx1, cy0, cy1;
            if (cell_span(xlo, xhi, c.x0, c.x1, c.cell_log2, &cx0, &cx1) &&
                cell_span(ylo, yhi, c.y0, c.y1, c.cell_log2, &cy0, &cy1)) {
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
    __syncthreads();
    if (tid < E) {
        const int nr = (sh.rows[tid] >> 16) - (sh.rows[tid] & 0xffff) + 1;
        if (nr > 0) atomicMax(&sh.max_rows, nr);
    }
    int32_t M;
    const int32_t ex = scan_block(cnt_e, &M, sh);
    if (tid < E) sh.sp[tid] = ex;
    if (tid == 0) sh.sp[E] = M;
    __syncthreads();
    return M;
}

// Copy window elements [c0, c1) (epoch order) into the stage as
// tile-relative coordinates.  One thread per (epoch, cell row).
__device__ void stage_chunk(const DenseArgs &a, const Shared &sh, const Tile &t, int2 *stage,
                            int32_t c0, int32_t c1) {
    const PreparedCatalog &c = a.cat;
    const int E = c.n_epochs;
    const int R = sh.max_rows;
    for (int pr = threadIdx.x; pr < E * R; pr += T) {
        const int e = pr / R, r = pr - (pr / R) * R;
        const int cy0 = sh.rows[e] & 0xffff, cy1 = sh.rows[e] >> 16;
        if (cy0 + r > cy1 || sh.sp[e + 1] <= c0 || sh.sp[e] >= c1) continue;
        const int cx0 = sh.cols[e] & 0xffff, cx1 = sh.cols[e] >> 16;
        int32_t dst = sh.sp[e];
        for (int rr = 0; rr < r; ++rr) {
            const int64_t b2 = ((int64_t)e * c.ncy + cy0 + rr) * c.ncx;
            dst += c.off[b2 + cx1 + 1] - c.off[b2 + cx0];
        }
        const int64_t base = ((int64_t)e * c.ncy + cy0 + r) * c.ncx;
        const int32_t src = c.off[base + cx0];
        const int32_t len = c.off[base + cx1 + 1] - src;
        const int32_t j0 = max(0, c0 - dst), j1 = min(len, c1 - dst);
#pragma unroll 4
        for (int32_t j = j0; j < j1; ++j) {
            const int2 p = c.sxy[src + j];
            stage[dst + j - c0] = make_int2((int32_t)(p.x - t.ox), (int32_t)(p.y - t.oy));
        }
    }
}

// Value of a lane's trash word: out-of-tile votes go there instead of being
// masked off, and the value makes sure no such vote ever looks lifted.
template <int MODE>
__device__ inline uint32_t trash_value() {
    return MODE == kMask32 ? 0xffffffffu : 0x7fffffffu;
}

// Vote every staged detection of the window with every lane velocity.  For
// each epoch a wave takes, lanes compute the shifts of their velocity once;
// then batches of kBatch iterations load 2 * kBatch staged detections, bin
// them, issue all atomics, and only then look at the returned values.
template <int MODE>
__device__ void vote_window(const DenseArgs &a, Shared &sh, const Tile &t, int2 *stage,
                            uint32_t *cells, int32_t *flags, int32_t M, int32_t my_vx,
                            int32_t my_vy, bool lane_ok) {
    const int E = a.cat.n_epochs;
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    const int half = lane >> 5, l32 = lane & (kLanes - 1);
    const uint32_t TX = (uint32_t)a.tile_x, TY = (uint32_t)a.tile_y;
    const int lTX = a.log2_tile_x, kc = a.log2b + a.coarse_log2;
    const uint32_t trash = (uint32_t)(a.tile_x * a.tile_y * kLanes + lane);
    const uint32_t nmin = (uint32_t)a.n_min;
    const int nch = (M + kStageCap - 1) / kStageCap;
    for (int ch = 0; ch < nch; ++ch) {
        const int32_t c0 = ch * kStageCap, c1 = min(M, c0 + kStageCap);
        __syncthreads();  // the previous chunk (or tile) is no longer read
        stage_chunk(a, sh, t, stage, c0, c1);
        __syncthreads();
        for (int e = wave; e < E; e += T / 64) {
            const int32_t p0 = max(sh.sp[e], c0) - c0, p1 = min(sh.sp[e + 1], c1) - c0;
            if (p0 >= p1) continue;
            const int32_t d = sh.dt[e];
            // an unused lane's shift puts every detection far outside the tile
            const int32_t sx = lane_ok ? shift_q8(my_vx, d) : 0x40000000;
            const int32_t sy = shift_q8(my_vy, d);
            const uint32_t val = MODE == kMask32 ? (1u << e) : 1u;
            for (int32_t i0 = p0 + half; i0 < p1; i0 += 2 * kBatch) {
                int2 q[kBatch];
#pragma unroll
                for (int b = 0; b < kBatch; ++b) q[b] = stage[i0 + 2 * b];  // padded stage
                uint32_t cell[kBatch];
#pragma unroll
                for (int b = 0; b < kBatch; ++b) {
                    const int32_t bx = (q[b].x - sx) >> kc, by = (q[b].y - sy) >> kc;
                    const bool ok = (i0 + 2 * b < p1) & ((uint32_t)bx < TX) & ((uint32_t)by < TY);
                    const uint32_t c = ((((uint32_t)by << lTX) | (uint32_t)bx) << 5) | (uint32_t)l32;
                    cell[b] = ok ? c : trash;
                }
                uint32_t old[kBatch];
#pragma unroll
                for (int b = 0; b < kBatch; ++b)
                    old[b] = MODE == kMask32 ? atomicOr(&cells[cell[b]], val)
                                             : atomicAdd(&cells[cell[b]], val);
                bool any = false;
#pragma unroll
                for (int b = 0; b < kBatch; ++b) {
                    const bool lifted = MODE == kMask32
                                            ? (!(old[b] & val) && (uint32_t)__popc(old[b] | val) == nmin)
                                            : old[b] == nmin - 1;
                    any |= lifted;
                }
                if (any) {  // rare: record the lifted cells
#pragma unroll
                    for (int b = 0; b < kBatch; ++b) {
                        const bool lifted =
                            MODE == kMask32
                                ? (!(old[b] & val) && (uint32_t)__popc(old[b] | val) == nmin)
                                : old[b] == nmin - 1;
                        if (lifted) {
                            const int f = atomicAdd(&sh.nflag, 1);
                            if (f < kFlagCap) flags[f] = (int32_t)cell[b];
                        }
                    }
                }
            }
        }
    }
}

template <int MODE>
__device__ inline uint32_t cell_count(uint32_t w) {
    return MODE == kMask32 ? (uint32_t)__popc(w) : w;
}

template <int MODE>
__global__ void __launch_bounds__(T) k_vote_dense(DenseArgs a) {
    extern __shared__ uint32_t smem[];
    __shared__ Shared sh;
    const int TX = a.tile_x, TY = a.tile_y;
    const int ncell = TX * TY * kLanes;
    uint32_t *cells = smem;
    int32_t *flags = (int32_t *)(smem + ncell + 64);  // after the 64 trash words
    int2 *stage = (int2 *)(smem + ncell + 64 + kFlagCap);
    const int tid = threadIdx.x;
    const int l32 = __lane_id() & (kLanes - 1);
    const uint32_t nmin = (uint32_t)a.n_min;

    for (int i = tid; i < ncell / 4; i += T) ((uint4 *)cells)[i] = make_uint4(0, 0, 0, 0);
    if (tid < 64) cells[ncell + tid] = trash_value<MODE>();
    for (int i = tid; i < kStagePad; i += T)  // padding past the stage: far outside any tile
        stage[kStageCap + i] = make_int2(0x40000000, 0x40000000);
    for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
        const int32_t sg = a.items[4 * item], ty0 = a.items[4 * item + 1];
        const int32_t txf = a.items[4 * item + 2], ntiles = a.items[4 * item + 3];
        __syncthreads();  // the previous item no longer reads the segment
        if (tid < kLanes) {
            const int64_t o = (int64_t)sg * kLanes + tid;
            sh.sv[tid] = a.seg_v[o];
            sh.svx[tid] = a.seg_vel[2 * o];
            sh.svy[tid] = a.seg_vel[2 * o + 1];
        }
        Tile t;
        t.ty0 = ty0;
        t.vx_lo = a.seg[4 * sg];
        t.vx_hi = a.seg[4 * sg + 1];
        t.vy_lo = a.seg[4 * sg + 2];
        t.vy_hi = a.seg[4 * sg + 3];
        const int kc = a.log2b + a.coarse_log2;
        t.oy = (int64_t)ty0 * ((int64_t)1 << kc);
        __syncthreads();
        const int32_t my_v = sh.sv[l32];
        const bool lane_ok = my_v >= 0;
        const int32_t my_vx = sh.svx[l32], my_vy = sh.svy[l32];

        for (int32_t ti = 0; ti < ntiles; ++ti) {
            t.tx0 = txf + ti * TX;
            t.ox = (int64_t)t.tx0 * ((int64_t)1 << kc);
            if (tid == 0) sh.nflag = 0;
            const int32_t M = tile_windows(a, t, sh);  // ends with a barrier
            if (M == 0) continue;
            if (M > kStageCap && tid == 0) atomicAdd(&a.res->n_spilled, 1);

            vote_window<MODE>(a, sh, t, stage, cells, flags, M, my_vx, my_vy, lane_ok);
            __syncthreads();

            // emit (or queue) the lifted cells; with an overflowed list, scan
            const int nflag = sh.nflag;
            if (nflag > 0) {
                const bool scan = nflag > kFlagCap;
                const int n = scan ? ncell : nflag;
                for (int f0 = 0; f0 < n; f0 += T) {
                    const int f = f0 + tid;
                    int cell = 0;
                    bool ok = false;
                    uint32_t cnt = 0;
                    if (f < n) {
                        cell = scan ? f : flags[f];
                        cnt = cell_count<MODE>(cells[cell]);
                        ok = cnt >= nmin;
                    }
                    const int bin = cell >> 5;
                    const uint32_t v = (uint32_t)sh.sv[cell & (kLanes - 1)];
                    const int32_t bx = t.tx0 + bin % TX, by = t.ty0 + bin / TX;
                    if (MODE == kCountRef) {
                        bool any;
                        const int64_t idx = wave_append(ok, (unsigned long long *)a.refine_count,
                                                        &any);
                        if (ok && idx < a.refine_cap)
                            a.refine[idx] = make_int4((int32_t)v, bx, by, 0);
                    } else {
                        emit(ok, v, bx, by, cnt, a.cand, a.cand_cap, a.res, a.count_sat);
                    }
                }
            }

            // clear the histogram (and reset the trash words) for the next tile
            __syncthreads();
            for (int i = tid; i < ncell / 4; i += T) ((uint4 *)cells)[i] = make_uint4(0, 0, 0, 0);
            if (tid < 64) cells[ncell + tid] = trash_value<MODE>();
        }
    }
}

// Exact bins of a queued cell: for velocity v and the cell's 2^m x 2^m
// bins, gather the detections that project into it (window index, one
// epoch per lane), count distinct epochs (or detections) per bin, emit the
// bins at or above N_min.  One wave per queued cell.
constexpr int kRefineBins = 64;  // up to 8 x 8 bins per cell

__global__ void __launch_bounds__(T) k_refine(DenseArgs a) {
    __shared__ uint32_t masks[T / 64][kRefineBins * kSlotWords];
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    uint32_t *mk = masks[wave];
    const PreparedCatalog &c = a.cat;
    const int E = c.n_epochs;
    const int m = a.coarse_log2, cw = 1 << m, nb = cw * cw;
    const int k = a.log2b;
    const int64_t n_all = (int64_t)*a.refine_count;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_all > a.refine_cap)
        atomicOr(&a.res->status, SAS_DATA_REFINE_FULL);
    const int64_t n_q = min(n_all, a.refine_cap);
    for (int64_t qi = (int64_t)blockIdx.x * (T / 64) + wave; qi < n_q;
         qi += (int64_t)gridDim.x * (T / 64)) {
        const int4 q = a.refine[qi];
        const int32_t v = q.x;
        const int32_t vx = a.vel[2 * (int64_t)v], vy = a.vel[2 * (int64_t)v + 1];
        const int32_t fbx0 = q.y * cw, fby0 = q.z * cw;  // first bin of the cell
        for (int i = lane; i < kRefineBins * kSlotWords; i += 64) mk[i] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < E; e += 64) {
            const int32_t d = c.dt[e];
            if (d < 0) continue;
            const int32_t sx = shift_q8(vx, d), sy = shift_q8(vy, d);
            const int64_t xlo = ((int64_t)fbx0 << k) + sx, ylo = ((int64_t)fby0 << k) + sy;
            int cx0, cx1, cy0, cy1;
            if (!cell_span(xlo, xlo + ((int64_t)cw << k), c.x0, c.x1, c.cell_log2, &cx0, &cx1) ||
                !cell_span(ylo, ylo + ((int64_t)cw << k), c.y0, c.y1, c.cell_log2, &cy0, &cy1))
                continue;
            for (int cy = cy0; cy <= cy1; ++cy) {
                const int64_t base = ((int64_t)e * c.ncy + cy) * c.ncx;
                const int32_t j1 = c.off[base + cx1 + 1];
                for (int32_t j = c.off[base + cx0]; j < j1; ++j) {
                    const int2 p = c.sxy[j];
                    const int32_t bx = ((p.x - sx) >> k) - fbx0, by = ((p.y - sy) >> k) - fby0;
                    if ((uint32_t)bx < (uint32_t)cw && (uint32_t)by < (uint32_t)cw) {
                        const int bin = by * cw + bx;
                        if (a.mode_epochs)
                            atomicOr(&mk[bin * kSlotWords + (e >> 5)], 1u << (e & 31));
                        else
                            atomicAdd(&mk[bin * kSlotWords], 1u);
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        uint32_t cnt = 0;
        if (lane < nb) {
            if (a.mode_epochs) {
                for (int w = 0; w < kSlotWords; ++w) cnt += __popc(mk[lane * kSlotWords + w]);
            } else {
                cnt = mk[lane * kSlotWords];
            }
        }
        emit(lane < nb && cnt >= (uint32_t)a.n_min, (uint32_t)v, fbx0 + (lane % cw),
             fby0 + (lane / cw), cnt, a.cand, a.cand_cap, a.res, a.count_sat);
        __builtin_amdgcn_wave_barrier();
    }
}

template <int MODE>
hipError_t launch_mode(const DenseArgs &a, size_t lds, hipStream_t stream) {
    const dim3 grid((unsigned)(a.n_items < kMaxVoteGrid ? a.n_items : kMaxVoteGrid)), block(T);
    hipLaunchKernelGGL(k_vote_dense<MODE>, grid, block, lds, stream, a);
    if (MODE == kCountRef)
        hipLaunchKernelGGL(k_refine, dim3(kRefineGrid), block, 0, stream, a);
    return hipGetLastError();
}

}  // namespace

size_t dense_lds_bytes(int mode, int tile_x, int tile_y) {
    (void)mode;
    size_t b = (size_t)tile_x * tile_y * kLanes * sizeof(uint32_t);  // histogram
    b += 64 * sizeof(uint32_t);                                      // trash words
    b += (size_t)kFlagCap * sizeof(int32_t);                         // lifted cells
    b += (size_t)(kStageCap + kStagePad) * sizeof(int2);             // staged window
    return b;
}

hipError_t launch_vote_dense(int mode, const DenseArgs &a, hipStream_t stream) {
    if (a.n_items <= 0) return hipSuccess;
    const size_t lds = dense_lds_bytes(mode, a.tile_x, a.tile_y);
    static bool attr_set[3] = {false, false, false};
    if (lds > 65536 && !attr_set[mode]) {
        const void *fn = mode == kMask32 ? (const void *)k_vote_dense<kMask32>
                         : mode == kCountDet ? (const void *)k_vote_dense<kCountDet>
                                             : (const void *)k_vote_dense<kCountRef>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_set[mode] = true;
    }
    switch (mode) {
    case kMask32: return launch_mode<kMask32>(a, lds, stream);
    case kCountDet: return launch_mode<kCountDet>(a, lds, stream);
    default: return launch_mode<kCountRef>(a, lds, stream);
    }
}

}  // namespace sas

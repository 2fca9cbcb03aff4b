// Sort-by-bin-key voting path for gfx950.
//
// Steps 1-2 of Sec. 2.1 with the Step-3 threshold, as a sort instead of a
// histogram: for a block of trial velocities, every (velocity j, detection i)
// vote becomes one 64-bit key
//     key = ((j * nby + (by - by0)) * nbx + (bx - bx0)) << 8 | epoch
// with (bx, by) the exact bin of Step 2 (floor((x - S(v)) / b), S(v) =
// ceil(v d / 65536)).  An LSD radix sort (8-bit digits, stable, only over the
// bits above the epoch byte) brings the votes of each (velocity, bin)
// together; one thread per run then counts its distinct epochs (or its
// length) and emits the run when the count reaches N_min.  The cost is in
// HBM: one key write, then per radix pass one read for the digit histogram
// and one read and one write for the scatter, then one read to count.
#include "internal.h"

namespace sas {
namespace {

constexpr int T = 256;                  // threads per block
constexpr int NWV = T / 64;             // waves per block
constexpr int kKeys = kSortKeysPerTile / T;  // keys per thread in a radix tile
constexpr uint64_t kNoKey = ~(uint64_t)0;    // invalid detections sort last and are ignored

__device__ inline int32_t shift_q8(int32_t v, int32_t d) {
    return (int32_t)(((int64_t)v * (int64_t)d + 65535) >> 16);
}

__global__ void __launch_bounds__(T) k_sort_keygen(SortArgs a, SortBlock blk) {
    const int64_t total = (int64_t)blk.nv * a.n;
    const int64_t stride = (int64_t)gridDim.x * T;
    const uint64_t limit = (uint64_t)1 << blk.key_bits;
    for (int64_t t = (int64_t)blockIdx.x * T + threadIdx.x; t < total; t += stride) {
        const int64_t j = t / a.n, i = t - j * a.n;
        const int e = a.epoch[i];
        uint64_t key = kNoKey;
        if (e < a.n_epochs) {
            const int32_t d = a.dt[e];
            const int32_t vx = a.vel[2 * (blk.v_off + j)], vy = a.vel[2 * (blk.v_off + j) + 1];
            // arithmetic shifts: floor for negative positions too
            const int64_t bx = (int64_t)(a.x[i] - shift_q8(vx, d)) >> a.log2b;
            const int64_t by = (int64_t)(a.y[i] - shift_q8(vy, d)) >> a.log2b;
            const int64_t rx = bx - blk.bx0, ry = by - blk.by0;
            if (rx >= 0 && rx < blk.nbx && ry >= 0 && ry < blk.nby) {
                const uint64_t bin = ((uint64_t)j * blk.nby + (uint64_t)ry) * blk.nbx + (uint64_t)rx;
                if (bin < limit) key = bin << 8 | (uint64_t)e;
            }
        }
        a.keys[t] = key;
    }
}

// Digit counts of one radix tile: hist[digit * n_tiles + tile].
__global__ void __launch_bounds__(T) k_rs_hist(const uint64_t *__restrict__ in, int64_t m,
                                                int shift, int32_t *__restrict__ hist,
                                                int64_t n_tiles) {
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kSortKeysPerTile;
#pragma unroll
    for (int k = 0; k < kKeys; ++k) {
        const int64_t i = t0 + k * T + threadIdx.x;
        if (i < m) atomicAdd(&cnt[(int)((in[i] >> shift) & 255)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one radix tile.  The tile is taken in rounds of T
// consecutive keys; within a round, a key's rank among the keys of its wave
// with the same digit comes from eight ballots (one per digit bit), and the
// waves' counts per digit are combined in LDS, so equal digits keep their
// input order.
__global__ void __launch_bounds__(T) k_rs_scatter(const uint64_t *__restrict__ in,
                                                   uint64_t *__restrict__ out, int64_t m,
                                                   int shift, const int32_t *__restrict__ hist,
                                                   int64_t n_tiles) {
    __shared__ int32_t base[256];
    __shared__ int32_t wcnt[NWV][256];
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kSortKeysPerTile;
    base[tid] = hist[(int64_t)tid * n_tiles + blockIdx.x];
    const uint64_t lt = lane ? (~(uint64_t)0 >> (64 - lane)) : 0;  // lanes below this one
    for (int r = 0; r < kKeys; ++r) {
#pragma unroll
        for (int w = 0; w < NWV; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = t0 + (int64_t)r * T + tid;
        const bool valid = i < m;
        const uint64_t key = valid ? in[i] : 0;
        const int d = (int)((key >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t mb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? mb : ~mb;
        }
        const int rank = __popcll(peers & lt);
        if (valid && (peers & lt) == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t pos = base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            out[pos] = key;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) add += wcnt[w][tid];
        base[tid] += add;
    }
}

// Wave-aggregated append: one global atomic per wave.  All lanes must call.
__device__ inline int64_t wave_append(bool ok, unsigned long long *counter) {
    const uint64_t mask = __ballot(ok);
    if (mask == 0) return 0;
    unsigned long long b = 0;
    if (__lane_id() == 0) b = atomicAdd(counter, (unsigned long long)__popcll(mask));
    b = __shfl(b, 0, 64);
    const uint32_t pre = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    return (int64_t)b + pre;
}

// One thread per run head: count the run's distinct epochs (or its length).
__global__ void __launch_bounds__(T) k_sort_count(SortArgs a, SortBlock blk,
                                                   const uint64_t *__restrict__ keys, int64_t m) {
    __shared__ uint32_t masks[T][kSlotWords + 1];
    uint32_t *mk = masks[threadIdx.x];
    const int64_t stride = (int64_t)gridDim.x * T;
    for (int64_t i0 = (int64_t)blockIdx.x * T; i0 < m; i0 += stride) {
        const int64_t i = i0 + threadIdx.x;
        bool ok = false;
        uint32_t cnt = 0;
        uint64_t bin = 0;
        if (i < m) {
            const uint64_t key = keys[i];
            bin = key >> 8;
            const bool head = key != kNoKey && (i == 0 || (keys[i - 1] >> 8) != bin);
            if (head) {
                if (a.mode_epochs) {
#pragma unroll
                    for (int w = 0; w < kSlotWords; ++w) mk[w] = 0;
                    for (int64_t k = i; k < m && (keys[k] >> 8) == bin; ++k) {
                        const uint32_t e = (uint32_t)(keys[k] & 255);
                        mk[e >> 5] |= 1u << (e & 31);
                    }
#pragma unroll
                    for (int w = 0; w < kSlotWords; ++w) cnt += __popc(mk[w]);
                } else {
                    int64_t k = i;
                    while (k < m && (keys[k] >> 8) == bin) ++k;
                    cnt = (uint32_t)(k - i);
                }
                ok = cnt >= (uint32_t)a.n_min;
            }
        }
        const int64_t idx = wave_append(ok, (unsigned long long *)&a.res->n_cand);
        if (ok && idx < a.cand_cap) {
            const uint64_t plane = (uint64_t)blk.nbx * (uint64_t)blk.nby;
            const int64_t j = (int64_t)(bin / plane);
            const uint64_t rem = bin - (uint64_t)j * plane;
            const int32_t by = blk.by0 + (int32_t)(rem / (uint64_t)blk.nbx);
            const int32_t bx = blk.bx0 + (int32_t)(rem % (uint64_t)blk.nbx);
            const uint32_t sat = (uint32_t)a.count_sat;
            uint4 rec;
            rec.x = (uint32_t)a.v_idx[blk.v_off + j];
            rec.y = (uint32_t)bx;
            rec.z = (uint32_t)by;
            rec.w = (cnt > sat ? sat : cnt) | ((cnt > sat ? 1u : 0u) << 16);
            *(uint4 *)(a.cand + idx) = rec;
        }
    }
}

inline unsigned grid_for(int64_t n, int64_t cap) {
    const int64_t b = (n + T - 1) / T;
    return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

}  // namespace

hipError_t launch_radix_sort_u64(uint64_t *keys, uint64_t *alt, int64_t m, int lo_bit, int hi_bit,
                                 int32_t *hist, int32_t *hist_blocksum, hipStream_t stream,
                                 uint64_t **sorted) {
    const int64_t n_tiles = (m + kSortKeysPerTile - 1) / kSortKeysPerTile;
    uint64_t *in = keys, *out = alt;
    for (int shift = lo_bit; shift < hi_bit && m > 0; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)n_tiles), dim3(T), 0, stream, in, m, shift,
                           hist, n_tiles);
        hipError_t e = launch_scan_exclusive(hist, 256 * n_tiles, hist_blocksum, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)n_tiles), dim3(T), 0, stream, in, out, m,
                           shift, hist, n_tiles);
        uint64_t *tmp = in;
        in = out;
        out = tmp;
    }
    *sorted = in;
    return hipGetLastError();
}

hipError_t launch_vote_sort_block(const SortArgs &a, const SortBlock &blk, hipStream_t stream) {
    const int64_t m = (int64_t)blk.nv * a.n;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort_keygen, dim3(grid_for(m, 1 << 16)), dim3(T), 0, stream, a, blk);
    uint64_t *in = nullptr;
    hipError_t e = launch_radix_sort_u64(a.keys, a.keys_alt, m, 8, 8 + blk.key_bits, a.hist,
                                         a.hist_blocksum, stream, &in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_count, dim3(grid_for(m, 1 << 15)), dim3(T), 0, stream, a, blk,
                       (const uint64_t *)in, m);
    return hipGetLastError();
}

}  // namespace sas

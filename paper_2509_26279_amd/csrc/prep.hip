// Catalog preparation for the voting transform.
//
//   * the reference epoch of Step 1 (Sec. 2.1): t0 is the earliest time at
//     which the catalog holds a detection, and every epoch that holds one gets
//     d_e = t_e - t0 (the others get -1);
//   * a window index: detections are grouped by (epoch, cell row, cell
//     column) with a counting sort, so that a workgroup can fetch the
//     detections that can land in its tile with one contiguous range per
//     (epoch, cell row);
//   * validation of the catalog (epoch < E, detection inside the footprint),
//     recorded as flags in the vote result.
#include "internal.h"

namespace sas {
namespace {

__device__ inline int wave_lane() { return __lane_id(); }

// Exclusive scan of one value per thread over the block (waves of 64,
// blockDim.x a multiple of 64, at most kScanThreads).  *total receives the
// block sum.  Ends with a barrier so that it may be called again.
__device__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t wave_off[kScanThreads / 64];
    __shared__ int32_t block_total;
    const int lane = wave_lane();
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wave_off[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const int32_t s = lane < nw ? wave_off[lane] : 0;
        int32_t si = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(si, d, 64);
            if (lane >= d) si += o;
        }
        if (lane < nw) wave_off[lane] = si - s;
        if (lane == nw - 1) block_total = si;
    }
    __syncthreads();
    const int32_t r = wave_off[wave] + incl - v;
    *total = block_total;
    __syncthreads();
    return r;
}

__global__ void k_prep_zero(int32_t *count, int64_t n_count, int32_t *present, int32_t n_epochs,
                            sas_vote_result *res, unsigned long long *refine_count,
                            unsigned long long *item_queue) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_count; i += stride)
        count[i] = 0;
    if (blockIdx.x == 0) {
        for (int e = threadIdx.x; e < n_epochs; e += blockDim.x) present[e] = 0;
        if (threadIdx.x == 0) {
            res->n_cand = 0;
            res->status = 0;
            res->n_spilled = 0;
            *refine_count = 0;
        }
        if (threadIdx.x < kXcds) item_queue[threadIdx.x] = 0;
    }
}

__global__ void k_prep_count(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                             const uint8_t *__restrict__ epoch, int64_t n, int32_t n_epochs,
                             int32_t ncx, int32_t ncy, int32_t cell_log2, int32_t x0, int32_t x1,
                             int32_t y0, int32_t y1, int32_t *__restrict__ count,
                             int32_t *__restrict__ cellid, int32_t *__restrict__ rank,
                             int32_t *__restrict__ present, sas_vote_result *res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e = epoch[i];
    const int32_t xi = x[i], yi = y[i];
    int32_t c = -1;
    if (e >= n_epochs) {
        atomicOr(&res->status, SAS_DATA_BAD_EPOCH);
    } else if (xi < x0 || xi >= x1 || yi < y0 || yi >= y1) {
        atomicOr(&res->status, SAS_DATA_OUTSIDE);
    } else {
        const int32_t cx = (xi - x0) >> cell_log2;
        const int32_t cy = (yi - y0) >> cell_log2;
        c = (e * ncy + cy) * ncx + cx;
        rank[i] = atomicAdd(&count[c], 1);
        present[e] = 1;
    }
    cellid[i] = c;
}

// Per-tile exclusive scan in place; tile totals to blocksum.
__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(int32_t *data, int64_t n, int32_t *blocksum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    int32_t v[kScanPerThread];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = (base + k < n) ? data[base + k] : 0;
        s += v[k];
    }
    int32_t total;
    int32_t run = block_exclusive_scan(s, &total);
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < n) data[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}

// Exclusive scan of the tile totals (one block, any count).
__global__ void __launch_bounds__(kScanThreads)
k_scan_blocksums(int32_t *blocksum, int64_t nb) {
    int32_t carry = 0;
    for (int64_t start = 0; start < nb; start += kScanThreads) {
        const int64_t i = start + threadIdx.x;
        const int32_t v = i < nb ? blocksum[i] : 0;
        int32_t total;
        const int32_t ex = block_exclusive_scan(v, &total);
        if (i < nb) blocksum[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

__global__ void k_scan_add(int32_t *data, int64_t n, const int32_t *blocksum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) data[i] += blocksum[i / kScanTile];
}

// Reference epoch (Step 1): t0 = min over epochs that hold a detection.
__global__ void k_prep_reftime(const int64_t *t, const int32_t *present, int32_t n_epochs,
                               int32_t *dt) {
    __shared__ long long red[kMaxEpochs];
    const int e = threadIdx.x;
    long long v = (e < n_epochs && present[e]) ? (long long)t[e] : LLONG_MAX;
    red[e] = v;
    __syncthreads();
    for (int s = kMaxEpochs / 2; s > 0; s >>= 1) {
        if (e < s) red[e] = red[e] < red[e + s] ? red[e] : red[e + s];
        __syncthreads();
    }
    const long long t0 = red[0];
    // epochs without detections get -1: nothing of theirs is ever projected
    if (e < n_epochs) dt[e] = (present[e] && t0 != LLONG_MAX) ? (int32_t)(t[e] - t0) : -1;
}

// Offsets by column: offT[(e (ncx + 1) + cx) ncy + cy] = off[(e ncy + cy) ncx + cx]
// for cx in [0, ncx] (cx = ncx reads the start of the next row, the end of
// row cy).  Threads run over offT in order, so its writes are coalesced.
__global__ void k_prep_offsets_by_column(const int32_t *__restrict__ off, int32_t *__restrict__ offT,
                                         int32_t n_epochs, int32_t ncx, int32_t ncy) {
    const int64_t total = (int64_t)n_epochs * (ncx + 1) * ncy;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t cy = i % ncy, rest = i / ncy;
        const int64_t cx = rest % (ncx + 1), e = rest / (ncx + 1);
        offT[i] = off[(e * ncy + cy) * ncx + cx];
    }
}

__global__ void k_prep_scatter(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                               const uint8_t *__restrict__ weight, int64_t n,
                               const int32_t *__restrict__ cellid,
                               const int32_t *__restrict__ rank, const int32_t *__restrict__ off,
                               int2 *__restrict__ sxy, int32_t *__restrict__ sidx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cellid[i];
    if (c < 0) return;
    const int32_t pos = off[c] + rank[i];
    // with weights the index keeps 256 x + w (|x| < 2^23 for weighted plans)
    sxy[pos] = make_int2(weight ? (int32_t)(((uint32_t)x[i] << 8) | weight[i]) : x[i], y[i]);
    sidx[pos] = (int32_t)i;  // position in the caller's catalog (candidate features)
}

inline unsigned blocks_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

hipError_t launch_scan_exclusive(int32_t *data, int64_t n, int32_t *blocksum, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, data, n,
                       blocksum);
    hipLaunchKernelGGL(k_scan_blocksums, dim3(1), dim3(kScanThreads), 0, stream, blocksum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n, 256)), dim3(256), 0, stream, data, n,
                       blocksum);
    return hipGetLastError();
}

hipError_t launch_prep(const int32_t *x, const int32_t *y, const uint8_t *epoch,
                       const uint8_t *weight, int64_t n,
                       const int64_t *t_dev, int32_t n_epochs, int32_t ncx, int32_t ncy,
                       int32_t cell_log2, const int32_t ext[4], int64_t n_cells,
                       const PrepBuffers &pb, sas_vote_result *res, hipStream_t stream) {
    const int64_t n_count = n_cells + 1;
    unsigned zb = blocks_for(n_count, 256);
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(k_prep_zero, dim3(zb), dim3(256), 0, stream, pb.count, n_count,
                       pb.present, n_epochs, res, pb.refine_count, pb.item_queue);
    if (n > 0) {
        hipLaunchKernelGGL(k_prep_count, dim3(blocks_for(n, 256)), dim3(256), 0, stream, x, y,
                           epoch, n, n_epochs, ncx, ncy, cell_log2, ext[0], ext[1], ext[2],
                           ext[3], pb.count, pb.cellid, pb.rank, pb.present, res);
    }
    const int64_t nb = (n_count + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, pb.count,
                       n_count, pb.blocksum);
    hipLaunchKernelGGL(k_scan_blocksums, dim3(1), dim3(kScanThreads), 0, stream, pb.blocksum, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n_count, 256)), dim3(256), 0, stream,
                       pb.count, n_count, pb.blocksum);
    {
        const int64_t total = (int64_t)n_epochs * (ncx + 1) * ncy;
        unsigned tb = blocks_for(total, 256);
        if (tb > 4096) tb = 4096;
        if (tb > 0)
            hipLaunchKernelGGL(k_prep_offsets_by_column, dim3(tb), dim3(256), 0, stream,
                               pb.count, pb.offT, n_epochs, ncx, ncy);
    }
    hipLaunchKernelGGL(k_prep_reftime, dim3(1), dim3(kMaxEpochs), 0, stream, t_dev, pb.present,
                       n_epochs, pb.dt);
    if (n > 0) {
        hipLaunchKernelGGL(k_prep_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, stream, x, y,
                           weight, n, pb.cellid, pb.rank, pb.count, pb.sxy, pb.sidx);
    }
    return hipGetLastError();
}

}  // namespace sas

// Internal declarations shared by the host code and the kernels of libsas.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sas.h"

namespace sas {

constexpr int kMaxEpochs = 256;
constexpr int kVoteThreads = 256;   // threads per dense-vote workgroup
constexpr int kVoteKmax = 16;       // detections held in registers per thread
constexpr int kVoteCap = kVoteThreads * kVoteKmax;
constexpr int kSlots = 256;         // exact-epoch slots per tag round (EPOCHS with E > 32)
constexpr uint32_t kTag = 0x80000000u;

// Dense-path kernel variants.
enum DenseMode : int {
    kMask32 = 0,    // EPOCHS, E <= 32: one epoch bitmask word per bin
    kCountDet = 1,  // DETECTIONS: one counter per bin
    kCountEpo = 2,  // EPOCHS, E > 32: counter per bin filters, tags give exact epochs
};

// Catalog after preparation: detections grouped by (epoch, cell row, cell column).
struct PreparedCatalog {
    const int32_t *sx;    // [n_valid] x, Q8
    const int32_t *sy;    // [n_valid] y, Q8
    const int32_t *off;   // [n_cells + 1] CSR offsets; cell = (e * ncy + cy) * ncx + cx
    const int32_t *dt;    // [E] t[e] - t0, Q16 h (0 for epochs without detections)
    int32_t n_epochs;
    int32_t ncx, ncy, cell_log2;
    int32_t x0, x1, y0, y1;
};

struct DenseArgs {
    PreparedCatalog cat;
    int32_t shift;        // 16 + log2(binw_q8): Q24 -> bin index
    int32_t tile_x, tile_y;
    int32_t n_min, count_sat;
    const int32_t *vel;         // [n_v][2]
    const int32_t *members;     // v_idx, grouped by block
    const int32_t *block_start; // [n_blocks + 1]
    const int32_t *block_vr;    // [n_blocks][4] vx_lo, vx_hi, vy_lo, vy_hi
    const int32_t *items;       // [n_items][3] block, tx0, ty0
    int64_t n_items;
    sas_candidate *cand;
    int64_t cand_cap;
    sas_vote_result *res;
};

// Workspace carve-up for the preparation stage.
struct PrepBuffers {
    int32_t *count;     // [n_cells + 1] -> offsets after the scan
    int32_t *blocksum;  // [scan blocks]
    int32_t *cellid;    // [n]
    int32_t *rank;      // [n]
    int32_t *sx, *sy;   // [n]
    int32_t *present;   // [E]
    int32_t *dt;        // [E]
};

constexpr int kScanThreads = 1024;
constexpr int kScanPerThread = 8;
constexpr int64_t kScanTile = (int64_t)kScanThreads * kScanPerThread;

hipError_t launch_prep(const int32_t *x, const int32_t *y, const uint8_t *epoch, int64_t n,
                       const int64_t *t_dev, int32_t n_epochs, int32_t ncx, int32_t ncy,
                       int32_t cell_log2, const int32_t ext[4], int64_t n_cells,
                       const PrepBuffers &pb, sas_vote_result *res, hipStream_t stream);

hipError_t launch_vote_dense(int mode, const DenseArgs &a, hipStream_t stream);
size_t dense_lds_bytes(int mode, int tile_x, int tile_y);

}  // namespace sas

// Internal declarations shared by the host code and the kernels of libsas.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sas.h"

namespace sas {

constexpr int kMaxEpochs = 256;
constexpr int kVoteThreads = 512;          // threads per vote workgroup
constexpr int kVoteWaves = kVoteThreads / 64;
constexpr int kMaxWavePairs = 128;         // (epoch, index row) pairs of one wave's windows
constexpr int kSlotWords = kMaxEpochs / 32;
constexpr int kLdsPerCU = 160 * 1024;      // gfx950
constexpr int kXcds = 8;                   // MI355X: accelerator dies, one L2 each

constexpr int kRefineGrid = 2048;          // workgroups of the refinement launch

// Detections of a window-index run that the refinement kernel loads at a
// time (each load bounded by the run's end).
constexpr int kCopyAhead = 4;

// Histogram variants of the dense path.
enum DenseMode : int {
    kMask32 = 0,    // EPOCHS, E <= 32, single bins: epoch bitmask per cell, emitted directly
    kCountDet = 1,  // DETECTIONS, single bins: counter per cell, emitted directly
    kCountRef = 2,  // counter of detections as a filter; lifted cells are refined
    kWeightDet = 3, // WEIGHTED_DETECTIONS, single bins: sum of weights, emitted directly
    kWeightRef = 4, // sum of weights as a filter (weighted modes); lifted cells are refined
};

// Catalog after preparation: detections grouped by (epoch, cell row, cell column).
struct PreparedCatalog {
    const int2 *sxy;      // [n_valid] (x, y), Q8; weighted plans: (256 x + w, y)
    const int32_t *sidx;  // [n_valid] catalog index of each detection
    const int32_t *off;   // [n_cells + 1] CSR offsets; cell = (e * ncy + cy) * ncx + cx
    const int32_t *offT;  // [E][ncx + 1][ncy] the same offsets by column:
                          // offT[(e * (ncx + 1) + cx) * ncy + cy] = off[(e * ncy + cy) * ncx + cx]
                          // (cx = ncx: the end of row cy), so that consecutive rows of one
                          // column are adjacent
    const int32_t *dt;    // [E] t[e] - t0, Q16 h; -1 for epochs without detections
    int32_t n_epochs;
    int32_t ncx, ncy, cell_log2;
    int32_t x0, x1, y0, y1;
};

struct DenseArgs {
    PreparedCatalog cat;
    int32_t log2b;            // bin width = 2^log2b Q8 px
    int32_t coarse_log2;      // histogram cells of 2^m x 2^m bins (kCountRef only)
    int32_t tile_x, tile_y;   // interior cells per tile
    int32_t hx, hy;           // histogram cells per tile, guards included
    int32_t stage_cap;        // detections staged in LDS at a time
    int32_t rows;             // index rows a tile window can touch (planner bound)
    int32_t rows_log2;        // run rows per epoch: 2^rows_log2 >= rows
    int32_t packed;           // 1: packed 16-bit votes (stage entries of 4 bytes)
    int32_t halves;           // 16-bit counts, lanes j and j + NV / 2 share a word: 1, two
                              // histograms of hx * hy * NV / 2 words alternate by tile;
                              // 2, one such histogram (its LDS is half a 32-bit one)
    int32_t n_min, count_sat;
    int32_t mode_epochs;      // 1: count distinct epochs, 0: count detections
    int32_t weighted;         // 0, or SAS_MODE_WEIGHTED_EPOCHS / _DETECTIONS
    const int32_t *vel;       // [n_v][2] velocities, Q8 px/h
    const int32_t *seg;       // [n_seg][4] vx_lo, vx_hi, vy_lo, vy_hi (Q8 px/h)
    const int32_t *seg_v;     // [n_seg][NV] v_idx of each lane (-1: unused)
    const int32_t *seg_vel;   // [n_seg][NV][2] velocity of each lane
    const int32_t *seg_guard; // [n_seg][NV] left guard cells gx | gy << 16
    const int32_t *items;     // [n_items][4] segment, ty0, first tx0, number of tiles
    int64_t n_items;
    int64_t n_items_kept;     // items [0, n_items_kept) suffice when epoch e_first (the
    int32_t e_first;          // earliest scheduled) holds a detection; the rest hold only
                              // tiles that fewer than N_min epochs can reach from it
    int4 *refine;             // [refine_cap] queued (v_idx, cell x, cell y, 0)
    unsigned long long *refine_count;
    int64_t refine_cap;
    unsigned long long *item_queue;  // [kXcds] items taken from each XCD's range (zeroed
                                     // by the preparation)
    sas_candidate *cand;
    int64_t cand_cap;
    sas_vote_result *res;
    unsigned long long *atomics;  // or null: adds the LDS atomic vote instructions issued
};

// Workspace carve-up for the preparation stage.
struct PrepBuffers {
    int32_t *count;     // [n_cells + 1] -> offsets after the scan
    int32_t *offT;      // [E][ncx + 1][ncy] offsets by column (PreparedCatalog::offT)
    int32_t *blocksum;  // [scan blocks]
    int32_t *cellid;    // [n]
    int32_t *rank;      // [n]
    int2 *sxy;          // [n]; with weights: (256 x + w, y)
    int32_t *sidx;      // [n] catalog index of each sorted detection
    int32_t *present;   // [E]
    int32_t *dt;        // [E]
    unsigned long long *refine_count;
    unsigned long long *item_queue;  // [kXcds]
};

constexpr int kScanThreads = 1024;
constexpr int kScanPerThread = 8;
constexpr int64_t kScanTile = (int64_t)kScanThreads * kScanPerThread;

hipError_t launch_prep(const int32_t *x, const int32_t *y, const uint8_t *epoch,
                       const uint8_t *weight, int64_t n,
                       const int64_t *t_dev, int32_t n_epochs, int32_t ncx, int32_t ncy,
                       int32_t cell_log2, const int32_t ext[4], int64_t n_cells,
                       const PrepBuffers &pb, sas_vote_result *res, hipStream_t stream);

// Exclusive scan of n int32 in place (blocksum: (n + kScanTile - 1) / kScanTile).
hipError_t launch_scan_exclusive(int32_t *data, int64_t n, int32_t *blocksum, hipStream_t stream);

// Sort-by-bin-key path.  A sort block is a run of velocities whose keys are
// generated, radix sorted and counted together.
struct SortBlock {
    int32_t v_off, nv;        // velocities [v_off, v_off + nv) of the block tables
    int32_t bx0, by0;         // smallest bin any (velocity, detection) of the block reaches
    int32_t nbx, nby;         // bin extent
    int32_t key_bits;         // bits of (velocity, by, bx) in the key above the epoch byte
    int32_t reserved;
};

struct SortArgs {
    const int32_t *x, *y;
    const uint8_t *epoch;
    int64_t n;
    const int32_t *dt;        // [E] d_e, -1 for epochs without detections
    int32_t n_epochs;
    int32_t log2b;
    int32_t n_min, count_sat, mode_epochs;
    const int32_t *vel;       // [n_v][2] velocities in block order
    const int32_t *v_idx;     // [n_v] v_idx in block order
    uint64_t *keys, *keys_alt;
    int32_t *hist, *hist_blocksum;
    sas_candidate *cand;
    int64_t cand_cap;
    sas_vote_result *res;
};

constexpr int kSortKeysPerTile = 4096;  // radix tile: 256 threads x 16 keys

// Stable LSD radix sort of m keys on bits [lo_bit, hi_bit) (8-bit digits);
// *sorted is keys or alt, whichever holds the result.  hist: 256 x tiles.
hipError_t launch_radix_sort_u64(uint64_t *keys, uint64_t *alt, int64_t m, int lo_bit, int hi_bit,
                                 int32_t *hist, int32_t *hist_blocksum, hipStream_t stream,
                                 uint64_t **sorted);

// Keys, radix sort and count of one sort block (blk: host copy of its table row).
hipError_t launch_vote_sort_block(const SortArgs &a, const SortBlock &blk, hipStream_t stream);

// Candidate features for learned vetting.
constexpr int kFeatures = 32;
struct FeatureArgs {
    PreparedCatalog cat;       // window index of the voted catalog
    int32_t log2b;
    int64_t span;              // Delta t of the plan, Q16 h (>= 1)
    double vmax;               // largest |v| of the plan's grid, Q8 px/h
    const int32_t *vel;        // [n_v][2]
    const float *snr;          // [n] by catalog index, or null
    const sas_candidate *cand;
    int64_t n_cand;
    float *feat;               // [n_cand][kFeatures]
    int32_t spacing;           // lattice spacing of the grid (0: no neighbour features)
    uint64_t *keys, *keys_alt; // [n_cand] neighbour keys (scratch)
    int32_t *hist, *hist_blocksum;
};
// Neighbour keys of the candidates, their sort, then the features.
hipError_t launch_features(const FeatureArgs &a, hipStream_t stream);

// ---- greedy cluster extraction (Step 3)
struct ExtractArgs {
    PreparedCatalog cat;
    int32_t log2b;
    int32_t n_min, mode_epochs, count_sat;
    const int32_t *vel;        // [n_v][2]
    const sas_candidate *cand;  // the cells the vote reported
    int64_t n_cand;
    int64_t n;                 // detections
    int32_t *first;            // [n_cand + 1] contributor counts, then offsets
    int32_t *scan_blocksum;
    int32_t *member;           // [member_cap] sorted positions of the contributors
    uint8_t *member_epoch;     // [member_cap] their epochs
    int32_t *member_cell;      // [member_cap] the cell of each entry
    int64_t member_cap;
    int32_t *inv_first;        // [n + 1] cells holding a detection: counts, then offsets
    int32_t *inv_blocksum;
    int32_t *inv_cursor;       // [n]
    int32_t *inv;              // [member_cap] the cells, grouped by detection
    int32_t *count;            // [n_cand] current count of each cell
    uint32_t *dirty;           // [n_cand] queued for a recount
    uint8_t *live;             // [n] by sorted position: not yet in a cluster
    uint8_t *open;             // [n_cand] 0 closed, 1 open, 2 taken in this round
    int32_t *best;             // [n] by sorted position: the best open cell holding it, -1
    int32_t *slot;             // [n_cand] provisional cluster of a cell taken in a round
    int32_t *taken;            // [n_cand] the cell of each cluster, by provisional index
    int32_t *perm;             // [n_cand] provisional index -> extraction order
    int32_t *counters;         // [2 + kExtractRounds + 1] taken so far, total, open after round r
    int32_t rounds;            // parallel rounds before the sequential finish (<= kExtractRounds)
    sas_candidate *clusters;   // [cluster_cap] in extraction order
    int64_t cluster_cap;
    int32_t *cluster_of;       // [n] by catalog index: cluster or -1
    sas_extract_result *res;
};
constexpr int kExtractRounds = 12;  // most parallel rounds before the sequential finish
constexpr int kExtractDefaultRounds = 4;
constexpr int kExtractCounters = 2 + kExtractRounds + 1;
hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream);

// Vetting MLP 32 -> 128 -> 128 -> 1; parameters packed W1 (32 x 128),
// b1, W2 (128 x 128), b2, W3 (128), b3.
constexpr int kMlpIn = 32, kMlpHidden = 128;
constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpIn * kMlpHidden;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpHidden;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpHidden * kMlpHidden;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpHidden;
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpHidden;
constexpr int kMlpParams = kMlpOffB3 + 1;  // 20865
constexpr int kMlpSplitK = 512;            // batch rows per weight-gradient partial

struct MlpWeights {        // bf16 working copies of the weights
    uint16_t *w1;          // [32][128]
    uint16_t *w2;          // [128][128]
    uint16_t *w3;          // [128][16], column 0 = W3, the rest 0
    float *b3pad;          // [16], element 0 = b3, the rest 0
};

struct MlpBuffers {
    float *p, *m, *v, *grad;   // FP32 master parameters, AdamW moments, gradient
    MlpWeights w;
    float *mu, *sd;            // [32] input standardisation
    uint16_t *a0;              // [max_batch][32]
    uint16_t *h1, *h2;         // [max_batch][128]
    uint16_t *d1, *d2;         // [max_batch][128]
    float *z16;                // [max_batch][16], column 0 = logits
    uint16_t *g3;              // [max_batch][16]
    float *row_loss;           // [max_batch]
    float *part;               // [max_batch / kMlpSplitK + 1][128][128]
};

hipError_t mlp_forward(const MlpBuffers &b, const float *x, int64_t n, hipStream_t s);
hipError_t mlp_logits(const MlpBuffers &b, const float *x, int64_t n, float *out, hipStream_t s);
hipError_t mlp_grad(const MlpBuffers &b, const float *x, const float *y, int64_t B, float pw,
                    float *loss, float *grad, hipStream_t s);
hipError_t mlp_adamw(const MlpBuffers &b, const float *grad, float lr, float b1, float b2,
                     float eps, float wd, float c1, float c2, hipStream_t s);
hipError_t mlp_refresh(const MlpBuffers &b, hipStream_t s);

// groups: lane groups G (1, 2 or 4); segments hold 64 / G velocities.
// ev0 / ev1 (optional) are recorded on the stream around the vote kernel.
hipError_t launch_vote_dense(int mode, int groups, const DenseArgs &a, hipStream_t stream,
                             hipEvent_t ev0, hipEvent_t ev1);
// One persistent launch over the merged items (chip, segment, ty0, txf,
// ntiles) of many chips of one kernel class: every chip's kept items first
// (n_kept of them), then the tiles skipped by coverage.  queue: kXcds device
// counters of this launch's own, zeroed on the stream before the vote kernel.
hipError_t launch_vote_dense_batch(int mode, int groups, int packed, const DenseArgs *chips_dev,
                                   int32_t n_chips, const int32_t *items5_dev, int64_t n_items,
                                   int64_t n_kept, int32_t hist_words_max, size_t lds,
                                   unsigned long long *queue, unsigned long long *atomics,
                                   hipStream_t stream);
hipError_t launch_refine(const DenseArgs &a, hipStream_t stream);
size_t dense_lds_bytes(int groups, int hx, int hy, int stage_cap, int packed, int halves);
size_t dense_static_lds_bytes();

// Refine / Gather / iterate (Steps 4-6) per cluster.
constexpr int kMaxRefineStarts = SAS_REFINE_MAX_STARTS;
struct RefineArgs {
    PreparedCatalog cat;       // window index of the voted catalog
    int32_t weighted;          // the index holds 256 x + w
    const int32_t *x, *y;      // [n] caller's catalog, Q8
    const uint8_t *epoch;      // [n]
    int64_t n;
    const int32_t *first;      // [n_clusters + 1] CSR over members
    const int32_t *members;    // [n_members] catalog indices
    int64_t n_members, n_clusters;
    const uint32_t *starts;    // [n_starts][4] random draws of the FAST-MCD starts
    int32_t n_starts;
    double radius_px;          // gather radius
    sas_refined *out;          // [n_clusters]
    int32_t *gathered;         // [n_clusters][gather_cap] or null
    int32_t gather_cap;
    int32_t *subset;           // [subset_clusters][SAS_REFINE_MAX_POINTS] or null
    int64_t subset_clusters;
};
hipError_t launch_refine_clusters(const RefineArgs &a, hipStream_t stream);

}  // namespace sas

/*
 * sas.h - C ABI of the catalog shift-and-stack voting transform on MI355X.
 *
 * The method (Stetzler et al., "An Efficient Shift-and-Stack Algorithm
 * Applied to Detection Catalogs", Sec. 2.1) takes a detection catalog
 * C = [x_i, y_i, t_i], a set of trial velocities V, a cluster size Delta x
 * and a minimum count N_min, and:
 *   Step 1 (Project) moves every detection back to the reference epoch t0,
 *          the earliest observation time in the catalog, along each trial
 *          velocity (linear motion, eqs. 1-2);
 *   Step 2 (Cluster) histograms the projected positions of each velocity with
 *          square bins of side Delta x;
 *   Step 3 (Find clusters) stops at bins whose count is below N_min.
 * This library computes Steps 1-2 exactly and reports every bin whose count
 * reaches N_min (the Step-3 threshold, without the greedy removal loop).
 *
 * Number formats (integers only cross the ABI):
 *   positions   Q8 pixels          int32   x_q8 = floor(256 * x_px)
 *   velocities  Q8 pixels / hour   int32
 *   times       Q16 hours          int64   any origin
 *   bin width   Q8 pixels          int32   (a power of two on the GPU path)
 * With d = t[e] - t0 (Q16 h), the projected position is the exact Q24 value
 *   X = 65536 * x - vx * d,  and the bin is bx = floor(X / (65536 * binw)),
 * the same for y.  Bins are anchored at 0 and half open: [k b, (k+1) b).
 * Count of a bin: the number of distinct epochs among its detections
 * (SAS_MODE_EPOCHS) or the number of its detections (SAS_MODE_DETECTIONS).
 * Weighted counts accumulate a per-detection weight w_i in [0, 255] (for
 * example a quantised detection likelihood) in place of the indicator, as
 * the Conclusions suggest: per epoch the largest weight among the bin's
 * detections of that epoch, summed over epochs (SAS_MODE_WEIGHTED_EPOCHS),
 * or the sum of all their weights (SAS_MODE_WEIGHTED_DETECTIONS).  N_min is
 * then the threshold on that score.  Weights of 1 give the indicator modes.
 *
 * Memory: "host" pointers are ordinary CPU memory, "device" pointers are
 * HIP device memory (hipMalloc or a framework's allocator) of the GPU that
 * is current when the call is made.  The caller owns every buffer passed
 * in; the library never frees them.  Plans own the device memory they
 * allocate until sas_plan_destroy.
 *
 * Streams: `stream` arguments are hipStream_t values passed as void*;
 * NULL means the default stream.  Asynchronous calls only enqueue work.
 *
 * Errors: every call returns a sas_status.  Argument errors are detected on
 * the host before anything is enqueued.  Data errors found on the device
 * (an epoch index >= E, a detection outside the declared footprint) are
 * recorded in the sas_vote_result and reported by sas_peaks.  A failing
 * HIP call returns SAS_E_DEVICE.  sas_last_error() gives a thread-local
 * message describing the last failure of the calling thread.
 */
#ifndef SAS_H
#define SAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sas_status;
#define SAS_OK 0
#define SAS_E_INVALID (-1)     /* bad argument or bad catalog data */
#define SAS_E_NOMEM (-2)       /* device or host allocation failed */
#define SAS_E_OVERFLOW (-3)    /* an output buffer is too small; the needed size is reported */
#define SAS_E_DEVICE (-4)      /* a HIP call failed, or no usable GPU */
#define SAS_E_UNSUPPORTED (-5) /* valid request outside what the GPU path implements */
#define SAS_E_WORKSPACE (-6)   /* workspace smaller than sas_vote_workspace_size() */

/* Device-side data errors (bits of sas_vote_result.status). */
#define SAS_DATA_BAD_EPOCH 1   /* an epoch index >= n_epochs */
#define SAS_DATA_OUTSIDE 2     /* a detection outside the plan's footprint */
#define SAS_DATA_REFINE_FULL 4 /* more flagged cells than the plan's refinement list holds */
#define SAS_DATA_INTERNAL 8    /* a tile window exceeded the plan's run table or guard cells
                                  (a library bug; the votes concerned were skipped) */

const char *sas_status_string(sas_status s);
/* Message of the calling thread's last failing call ("" if none). */
const char *sas_last_error(void);
/* Library version string. */
const char *sas_version(void);

/* ------------------------------------------------------------------------
 * Velocity grid (Sec. 2: the residuals of an object stay inside one cluster
 * of size Delta x when each velocity component is off by at most
 * Delta x / Delta t; eq. v_size counts the resulting set).
 * ---------------------------------------------------------------------- */
#define SAS_GRID_BOX 0     /* vx in [vmin, vmax], vy in [vy_min, vy_max]       */
#define SAS_GRID_DISK 1    /* |v| <= vmax                                       */
#define SAS_GRID_ANNULUS 2 /* vmin <= |v| <= vmax                               */
#define SAS_GRID_SECTOR 3  /* annulus and direction within angle +- half_width   */

typedef struct {
    int32_t shape;          /* SAS_GRID_* */
    double vmin, vmax;      /* px/h: box vx range, or speed range */
    double vy_min, vy_max;  /* px/h: box only */
    double angle_deg;       /* sector: centre direction (deg, from +x toward +y) */
    double half_width_deg;  /* sector: half opening, in (0, 90) */
    int32_t binw_q8;        /* Delta x, Q8 px (> 0) */
    int64_t span_q16;       /* Delta t, Q16 h (> 0): last minus first epoch */
    int32_t spacing_q8;     /* 0: floor(binw_q8 * 65536 / span_q16); else this value */
} sas_grid_spec;

/* Lattice spacing floor(binw_q8 * 65536 / span_q16) in Q8 px/h (>= 1). */
sas_status sas_grid_spacing(int32_t binw_q8, int64_t span_q16, int32_t *spacing_out);

/*
 * sas_build_grid: lattice points (i s, j s) whose closed cell
 * [p - s/2, p + s/2]^2 meets the region, written to v_out_host as
 * (vx, vy) int32 pairs in row-major (vy, vx) order.  That order defines
 * v_idx.  Two-call protocol: *n_out always receives the full count; if cap
 * is smaller, only the first cap points are written and SAS_E_OVERFLOW is
 * returned.  v_out_host == NULL with cap == 0 is a pure count query (SAS_OK).
 * Host only; no device is touched.
 */
sas_status sas_build_grid(const sas_grid_spec *spec, int32_t *v_out_host, int64_t cap,
                          int64_t *n_out);

/*
 * sas_threshold_n_min: the threshold rule of Sec. 2.2.  With mu noise
 * detections per bin per epoch (Poisson), a pure-noise bin holds a noise
 * detection in an epoch with probability 1 - exp(-mu); its distinct epochs
 * are Binomial(E, 1 - exp(-mu)) (SAS_MODE_EPOCHS) and its detections
 * Poisson(E mu) (SAS_MODE_DETECTIONS).  *n_min_out receives the smallest
 * N_min with n_stacks * P(count >= N_min) <= n_false, n_stacks being the
 * number of independent stacks of eq. (N_stacks), |V| Omega / Delta x^2.
 * Host only.  Errors: SAS_E_INVALID (arguments, or no N_min <= E reaches
 * n_false in EPOCHS mode).
 */
sas_status sas_threshold_n_min(int32_t n_epochs, double mu, double n_stacks, double n_false,
                               int32_t mode, int32_t *n_min_out);

/* ------------------------------------------------------------------------
 * Candidates and results
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t v_idx;  /* index of the trial velocity in the plan's velocity set */
    int32_t bx, by;  /* bin of the projected positions, anchored at 0 */
    uint16_t count;  /* the bin's count or weighted score, capped at count_sat */
    uint16_t flags;  /* bit 0: the true count exceeded count_sat */
} sas_candidate;     /* 16 bytes */

typedef struct {
    int64_t n_cand;  /* total candidates found; may exceed the buffer capacity */
    int32_t status;  /* SAS_DATA_* bits, 0 when the catalog was valid */
    int32_t n_spilled; /* diagnostic: tiles whose detection window exceeded the LDS
                          staging capacity and were processed in chunks (same result) */
} sas_vote_result;   /* 16 bytes, device resident, written by sas_vote */

#define SAS_MODE_EPOCHS 0
#define SAS_MODE_DETECTIONS 1
#define SAS_MODE_WEIGHTED_EPOCHS 2     /* dense path; voted with sas_vote_weighted */
#define SAS_MODE_WEIGHTED_DETECTIONS 3 /* dense path; voted with sas_vote_weighted */

#define SAS_PATH_AUTO 0
#define SAS_PATH_DENSE 1   /* LDS-resident count tiles (velocity block x spatial tile) */
#define SAS_PATH_SORT 2    /* sort-by-bin-key in HBM */

/* Launch shape of the dense path; zeros select the built-in defaults. */
typedef struct {
    int32_t tile_x, tile_y;     /* interior histogram cells per tile (>= 1; the histogram with
                                   its guard cells and the stage must fit in LDS) */
    int32_t vblock_x, vblock_y; /* velocity segment in lattice steps; the product is at most
                                   64 / groups */
    int32_t groups;             /* lane groups G in {1, 2, 4}: a wave votes G detections per
                                   instruction for 64 / G velocities */
    int32_t stage_cap;          /* detections staged in LDS at a time (larger windows are
                                   processed in chunks) */
    int32_t cell_log2;          /* log2 of the window-index cell size in Q8 px */
    int32_t sort_vblock;        /* velocities per sort-path block */
    int32_t n_det_hint;         /* expected detections per catalog: chooses the cell size */
    int32_t coarse_log2;        /* histogram cells of 2^m x 2^m bins, m in [0, 3]; -1: single
                                   bins; 0: chosen from n_det_hint */
    int32_t refine_cap;         /* capacity of the list of flagged cells (0: chosen by the plan) */
    int32_t packed;             /* 0: packed 16-bit votes wherever the tile allows them (a
                                   histogram row and column span at most 2^16 Q8 px); -1: never */
    int32_t weight_hint;        /* weighted plans: typical weight of a detection (1..255); with
                                   n_det_hint it lets coarse_log2 = 0 choose coarse cells.
                                   0: weighted plans use single bins unless coarse_log2 > 0 */
    int32_t half_counts;        /* 16-bit histogram counts (dense plans that count detections,
                                   more than 32 epochs, or coarse cells): velocity lanes j and
                                   j + NV / 2 of a block of NV = 64 / groups share a word.
                                   One lane group with 32-bit votes: two histograms alternate
                                   by tile, and a tile whose window entries reach 2^16 is voted
                                   with 32-bit counts; otherwise one histogram in half the LDS
                                   (larger tiles, or three workgroups per CU for one lane group
                                   with packed votes), and such a tile is voted in two passes
                                   of half the lanes each with 32-bit counts.  0: on wherever
                                   the plan allows it; 1: on, and an error (SAS_E_INVALID) where
                                   the plan does not; -1: off */
    int32_t prune;              /* SAS_MODE_EPOCHS plans: 0 skips the tiles of a velocity block
                                   where fewer than N_min epochs can reach any bin (the window
                                   of every other epoch misses the footprint), which cannot
                                   hold a candidate; the output is unchanged.  -1: vote every
                                   tile.  Other modes never skip tiles. */
} sas_tuning;

/* ------------------------------------------------------------------------
 * Plans: host analysis of (velocity set, epochs, parameters, footprint).
 * A plan fixes the work decomposition and holds its tables in device
 * memory, so that sas_vote itself allocates nothing, never synchronises
 * and can be captured into a HIP graph.
 * ---------------------------------------------------------------------- */
typedef struct {
    const int32_t *v_host;  /* host [n_v][2] Q8 px/h; row j is velocity v_idx = j */
    int64_t n_v;            /* >= 0 */
    int32_t n_epochs;       /* E in [1, 256] */
    const int64_t *t_q16;   /* host [E] epoch times, Q16 h; max - min < 2^31 */
    int32_t binw_q8;        /* Delta x in Q8 px: a power of two in [1, 2^20] */
    int32_t n_min;          /* >= 1 */
    int32_t mode;           /* SAS_MODE_* */
    int32_t count_sat;      /* 255 or 65535: largest reportable count */
    int32_t path;           /* SAS_PATH_* */
    int32_t extent_q8[4];   /* footprint x0, x1, y0, y1 (Q8): every detection must
                               satisfy x0 <= x < x1 and y0 <= y < y1; |values| < 2^30 */
    const sas_tuning *tuning; /* NULL: defaults */
} sas_plan_desc;

typedef struct sas_plan sas_plan;

/*
 * sas_plan_create: validate the description, decompose the work and upload
 * the plan tables to the current device (allocates; synchronous).  The
 * velocity array is copied; the caller may free it on return.
 * Errors: SAS_E_INVALID (arguments; message in sas_last_error),
 * SAS_E_UNSUPPORTED (bin width not a power of two, |v| * Delta t too large
 * for 32-bit bins, a weighted mode on the sort path, a weighted tile row of
 * 2^24 Q8 px or more, a weighted plan whose footprint plus largest shift
 * reaches 2^23 Q8 px), SAS_E_NOMEM, SAS_E_DEVICE.
 * Weighted plans choose coarse cells only with tuning.weight_hint (or an
 * explicit coarse_log2 > 0), and never use the packed 16-bit votes.
 */
sas_status sas_plan_create(const sas_plan_desc *desc, sas_plan **plan_out);
sas_status sas_plan_destroy(sas_plan *plan);
/* Work-decomposition facts: items, velocity blocks, path chosen. */
typedef struct {
    int64_t n_items;   /* (velocity block, tile row) work items */
    int64_t n_tiles;   /* (velocity block, tile) pairs */
    int64_t n_blocks;
    int32_t path;
    int32_t tile_x, tile_y;
    int32_t vblock_x, vblock_y;
    int32_t cell_log2;
    int32_t coarse_log2;   /* histogram cells of 2^m x 2^m bins */
    int32_t mode_variant;  /* 0 epoch masks, 1 detection counts, 2 counts + refinement,
                              3 weight sums, 4 weight sums + refinement */
    int64_t n_v;
    int32_t groups;        /* lane groups G */
    int32_t hist_x, hist_y; /* histogram cells per tile, guard cells included */
    int32_t stage_cap;
    int32_t lds_bytes;     /* LDS per vote workgroup */
    int32_t packed;        /* 1: votes use packed 16-bit arithmetic */
    int32_t half_counts;   /* 16-bit histogram counts: 1, two histograms by tile (one lane
                              group, 32-bit votes); 2, one histogram; 0, 32-bit counts */
    int64_t n_tiles_kept;  /* tiles voted when the catalog's earliest epoch holds a detection
                              (the rest reach fewer than N_min epochs; tuning.prune) */
    int64_t n_items_kept;  /* their work items */
} sas_plan_info;
sas_status sas_plan_get_info(const sas_plan *plan, sas_plan_info *info);

/*
 * sas_plan_set_probe: measurement hook.  Later sas_vote calls with this plan
 * record the two hipEvent_t handles on their stream immediately before and
 * after the vote kernel (preparation and refinement excluded), so that the
 * caller can time that kernel alone.  NULL handles switch the hook off.  The
 * events stay owned by the caller.
 */
sas_status sas_plan_set_probe(sas_plan *plan, void *ev_before, void *ev_after);

/*
 * sas_plan_set_counter: measurement hook.  Later sas_vote calls with this
 * plan add to *counter_dev (a device uint64 the caller owns and clears) the
 * number of 64-lane LDS atomic instructions their vote kernel issues to
 * cast votes (a run of n staged detections of one epoch takes
 * ceil(n / groups) of them).  With the kernel time this gives the rate of
 * the LDS atomic unit.  NULL switches it off.
 */
sas_status sas_plan_set_counter(sas_plan *plan, uint64_t *counter_dev);

/* ------------------------------------------------------------------------
 * Autotuner of the dense path's launch shape (no paper passage: the paper's
 * implementation runs on CPUs).  A launch shape changes the time of a vote,
 * never its candidate list; the tuner checks that.
 * ---------------------------------------------------------------------- */
typedef struct {
    sas_tuning tuning;  /* the candidate tried */
    float ms;           /* median time of its vote kernel, -1 when its plan does not fit */
    int32_t status;     /* SAS_OK, or the sas_plan_create error of this shape */
} sas_autotune_trial;

/*
 * sas_autotune_default_candidates: the built-in candidate list around the
 * planner's choice for desc (its tuning field is the base every candidate
 * starts from): the planner default, each lane-group count, window-index
 * cells one step finer and coarser, and five tile shapes per lane-group
 * count.  *n_out receives the count; SAS_E_OVERFLOW when cap is smaller.
 * Creates (and destroys) a plan on the current device.
 */
sas_status sas_autotune_default_candidates(const sas_plan_desc *desc, sas_tuning *out,
                                           int32_t cap, int32_t *n_out);

/*
 * sas_autotune: time each candidate tuning on one catalog and return the
 * fastest in *best_out.  For every candidate: a plan (desc with that
 * tuning), one vote whose list is collected in canonical order, then `reps`
 * votes timed with events around the vote kernel (the median is kept).
 *   x_q8, y_q8, epoch: device [n]; cands: host [n_cands]; trials_out: host
 *   [n_cands].
 * Candidates whose plan does not fit (SAS_E_INVALID or SAS_E_UNSUPPORTED
 * from sas_plan_create) get ms = -1 and are skipped.  Every other candidate
 * must give the candidate list of the first one that fits; a difference is
 * a library bug and returns SAS_E_DEVICE naming the shape.  Allocates
 * device memory and synchronises `stream`: an offline call.
 * Errors: SAS_E_INVALID (arguments, no shape fits), SAS_E_UNSUPPORTED
 * (sort-path or weighted plans), SAS_E_NOMEM, SAS_E_DEVICE, and those of
 * sas_vote and sas_peaks for the catalog.
 */
sas_status sas_autotune(const sas_plan_desc *desc, const int32_t *x_q8, const int32_t *y_q8,
                        const uint8_t *epoch, int64_t n, const sas_tuning *cands, int32_t n_cands,
                        int32_t reps, sas_autotune_trial *trials_out, sas_tuning *best_out,
                        void *stream);

/*
 * sas_autotune_key: the shape class of a catalog, the key of the tuning
 * cache: bin width, lattice spacing floor(binw * 65536 / span), and the
 * epoch count, detection count n and velocity count rounded down to powers
 * of two, and the mode ("b1024_s256_E64_n262144_V65536_m0").  Host only.
 */
sas_status sas_autotune_key(const sas_plan_desc *desc, int64_t n, char *key_out, int64_t cap);

/*
 * Tuning cache: a text file with one shape class per line,
 * "<key> name=value ..." (sas_tuning field names; absent fields are 0).
 * sas_autotune_cache_get sets *found to 1 and fills *out when the key is
 * present (a missing file is an empty cache); sas_autotune_cache_put adds
 * or replaces the key's line (lines kept sorted; written through a
 * temporary file).  Host only.
 */
sas_status sas_autotune_cache_get(const char *path, const char *key, sas_tuning *out,
                                  int32_t *found);
sas_status sas_autotune_cache_put(const char *path, const char *key, const sas_tuning *tuning);

/* ------------------------------------------------------------------------
 * Ceilings: rates of the units the dense vote uses, measured on the current
 * device (no paper passage; the roofline of the vote kernel is stated
 * against them).  Each figure is the best of a few launches of a kernel that
 * repeats one kind of instruction on every resident wave.
 * ---------------------------------------------------------------------- */
typedef struct {
    double lds_atomic_conflict_free; /* lane atomic adds per second, 64 consecutive words per
                                        wave instruction (no bank conflict) */
    double lds_atomic_lane_groups;   /* the same with 4 groups of 16 lanes each adding to the
                                        16 words of one random bin (the G = 4 vote pattern) */
    double valu_int32_ops;           /* 32-bit integer add / xor lane operations per second */
    double valu_int16x2_ops;         /* packed 16-bit integer half operations per second */
    double hbm_copy_bytes_per_s;     /* bytes read plus written per second, 1 GiB device copy */
} sas_ceilings;

/* Run the measurements on `stream` (allocates 2 GiB and more for its buffers,
 * frees them, synchronises).  Errors: SAS_E_INVALID, SAS_E_DEVICE. */
sas_status sas_measure_ceilings(sas_ceilings *out, void *stream);

/* Device workspace needed by sas_vote for a catalog of n detections. */
sas_status sas_vote_workspace_size(const sas_plan *plan, int64_t n, size_t *bytes);

/*
 * sas_vote: enqueue the voting transform of one catalog on `stream`.
 *   x_q8, y_q8, epoch: device [n]; epoch values in [0, n_epochs).
 *   cand_dev:  device [cand_cap] candidate records (unordered).
 *   res_dev:   device sas_vote_result; n_cand counts every candidate even
 *              past cand_cap (later ones are not written).
 *   workspace: device, >= sas_vote_workspace_size(plan, n) bytes,
 *              256-byte aligned; its contents are scratch.
 * Asynchronous: returns once the work is enqueued.  No allocation, no
 * synchronisation, no memset nodes: safe to capture in a HIP graph.  Calls
 * that share a workspace or a result must be ordered by the caller.
 * Errors (host side, nothing enqueued): SAS_E_INVALID (also for a plan in
 * a weighted mode), SAS_E_WORKSPACE.
 */
sas_status sas_vote(const sas_plan *plan, const int32_t *x_q8, const int32_t *y_q8,
                    const uint8_t *epoch, int64_t n, sas_candidate *cand_dev, int64_t cand_cap,
                    sas_vote_result *res_dev, void *workspace, size_t ws_bytes, void *stream);

/*
 * sas_vote_weighted: sas_vote for a plan in SAS_MODE_WEIGHTED_EPOCHS or
 * SAS_MODE_WEIGHTED_DETECTIONS (the weighted accumulation the Conclusions
 * propose in place of the detection indicator).
 *   weight: device [n] uint8, the weight of each detection (0..255).
 * Every other argument, the outputs and the asynchronous, allocation-free
 * behaviour are those of sas_vote; a candidate's count is its score capped
 * at count_sat.  Weighted plans are not accepted by sas_batch_create,
 * sas_features or sas_extract_clusters.
 * Errors (host side, nothing enqueued): SAS_E_INVALID (also for a plan in
 * an indicator mode, or a null weight array with n > 0), SAS_E_WORKSPACE.
 */
sas_status sas_vote_weighted(const sas_plan *plan, const int32_t *x_q8, const int32_t *y_q8,
                             const uint8_t *epoch, const uint8_t *weight, int64_t n,
                             sas_candidate *cand_dev, int64_t cand_cap, sas_vote_result *res_dev,
                             void *workspace, size_t ws_bytes, void *stream);

/*
 * sas_vote_static: sas_vote for callers that cannot allocate device memory
 * or take a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The scratch sas_vote keeps in the
 * caller's workspace lives instead in one static device array of
 * SAS_STATIC_SCRATCH_BYTES per GPU, owned by the library and held until the
 * process ends.  The caller still passes the catalog and the outputs, with
 * the meaning they have in sas_vote; no allocation is made.
 *   Every call on one GPU shares that GPU's array and leaves its contents
 *   behind; each call clears what it needs itself.  Calls that overlap on
 *   one GPU (concurrent streams or threads) race on the array: order them.
 *   Extraction, features and refinement read a vote's workspace and so need
 *   sas_vote, not this variant.
 * Errors (host side, nothing enqueued): those of sas_vote, and
 * SAS_E_WORKSPACE when sas_vote_workspace_size(plan, n) exceeds
 * SAS_STATIC_SCRATCH_BYTES (a plan with a smaller tuning.refine_cap may fit).
 */
#define SAS_STATIC_SCRATCH_BYTES (64 * 1024 * 1024)
sas_status sas_vote_static(const sas_plan *plan, const int32_t *x_q8, const int32_t *y_q8,
                           const uint8_t *epoch, int64_t n, sas_candidate *cand_dev,
                           int64_t cand_cap, sas_vote_result *res_dev, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many catalogs (e.g. the chips of one night, each with its own
 * plan: grid, epochs, threshold, footprint) voted by one persistent launch
 * per kernel class.  The chips' work items are merged into one list (largest
 * chips first) that the resident workgroups walk together, so chips of very
 * different sizes keep every CU busy.
 * ---------------------------------------------------------------------- */
typedef struct {
    const sas_plan *plan;           /* dense-path plan of this chip (kept alive by the caller) */
    const int32_t *x_q8, *y_q8;     /* device [n] */
    const uint8_t *epoch;           /* device [n] */
    int64_t n;
    sas_candidate *cand_dev;        /* device [cand_cap] */
    int64_t cand_cap;
    sas_vote_result *res_dev;       /* device */
} sas_batch_chip;

typedef struct sas_batch sas_batch;

/* Device workspace of a batch (all chips' workspaces plus the queues). */
sas_status sas_batch_workspace_size(const sas_batch_chip *chips, int32_t n_chips, size_t *bytes);

/*
 * sas_batch_create: bind n_chips catalogs, outputs and one workspace
 * (>= sas_batch_workspace_size, 256-byte aligned), merge the chips' work
 * items into one list per kernel class and upload the
 * tables (allocates; synchronous).  The bound buffers must stay valid while
 * the batch is used; their contents may change between votes.
 * Errors: SAS_E_INVALID (arguments, a plan that is not on the dense path),
 * SAS_E_WORKSPACE, SAS_E_NOMEM, SAS_E_DEVICE.
 */
sas_status sas_batch_create(const sas_batch_chip *chips, int32_t n_chips, void *workspace,
                            size_t ws_bytes, sas_batch **batch_out);
sas_status sas_batch_destroy(sas_batch *batch);

/*
 * sas_vote_batch: enqueue the voting transform of every bound chip on
 * `stream`; each chip's candidates and result go to its own buffers
 * (collect them with sas_peaks).  No allocation, no synchronisation, no
 * memset nodes: safe to capture in a HIP graph and replay.
 */
sas_status sas_vote_batch(const sas_batch *batch, void *stream);

/* Measurement hook: record ev_before / ev_after around the batch's vote
 * kernels (first class launch to last) on the call's stream; NULL, NULL off. */
sas_status sas_batch_set_probe(sas_batch *batch, void *ev_before, void *ev_after);
/* Measurement hook: later sas_vote_batch calls add their vote kernels' LDS
 * atomic vote instructions to *counter_dev (as sas_plan_set_counter). */
sas_status sas_batch_set_counter(sas_batch *batch, uint64_t *counter_dev);

/* ------------------------------------------------------------------------
 * Greedy cluster extraction (Step 3 of Sec. 2.1).
 * ---------------------------------------------------------------------- */
#define SAS_EXTRACT_MEMBERS_FULL 1  /* the contributor lists exceed member_cap */
#define SAS_EXTRACT_CLUSTERS_FULL 2 /* more clusters than cluster_cap (n_clusters is true) */

typedef struct {
    int64_t n_clusters; /* clusters extracted (may exceed cluster_cap) */
    int64_t n_members;  /* contributors of all reported cells (the lists' total size) */
    int32_t status;     /* SAS_EXTRACT_* bits */
    int32_t reserved;
} sas_extract_result;

/*
 * sas_extract_clusters: Step 3 of Sec. 2.1 over the cells a vote reported.
 * The loop takes the cell with the largest count (ties: smaller v_idx, then
 * by, then bx), reports it as a cluster, removes its contributing
 * detections (those whose exact bin at its velocity is the cell) from every
 * cell, recounts, and stops when no cell reaches the plan's N_min.  Counts
 * follow the plan's mode (distinct epochs or detections).  Counts only fall,
 * so cells below N_min at the start are never needed.
 *   workspace:   the workspace of the last sas_vote of this dense-path plan
 *                on this catalog (n detections): its window index is read.
 *   cand_dev:    device [n_cand] cells reported by that vote (any order).
 *                The list must be complete: a vote whose result reports a
 *                data error or more candidates than its buffer held (what
 *                sas_peaks refuses) gives a wrong extraction.
 *   member_cap:  capacity of the contributor lists (sum over the cells of
 *                their contributors); see res->n_members when exceeded.
 *   scratch:     device, >= sas_extract_scratch_size(n, n_cand, member_cap).
 *   clusters_dev: device [cluster_cap] clusters in extraction order, count =
 *                the count at extraction (saturated like the vote's).
 *   cluster_of_dev: device int32 [n] by catalog index: the cluster that took
 *                the detection, or -1.
 *   res_dev:     device sas_extract_result.
 *   rounds:      parallel rounds before the loop goes on one take at a time:
 *                each round takes every cell that beats all open cells
 *                sharing a live detection with it (the loop would take each
 *                of them, with the same detections); 0: the default (4),
 *                -1: none, 1..12.  The result does not depend on it.
 * Asynchronous, no allocation.  Errors: SAS_E_INVALID (arguments,
 * member_cap >= 2^31, rounds outside [-1, 12], not a dense-path plan),
 * SAS_E_UNSUPPORTED (a weighted plan), SAS_E_WORKSPACE.
 */
sas_status sas_extract_clusters(const sas_plan *plan, const void *workspace, size_t ws_bytes,
                                int64_t n, const sas_candidate *cand_dev, int64_t n_cand,
                                int64_t member_cap, void *scratch, size_t scratch_bytes,
                                sas_candidate *clusters_dev, int64_t cluster_cap,
                                int32_t *cluster_of_dev, sas_extract_result *res_dev,
                                int32_t rounds, void *stream);

/* Bytes of scratch sas_extract_clusters needs. */
sas_status sas_extract_scratch_size(int64_t n, int64_t n_cand, int64_t member_cap,
                                    size_t *bytes);

/* ------------------------------------------------------------------------
 * Learned vetting: candidate features.
 * ---------------------------------------------------------------------- */
#define SAS_N_FEATURES 32

/*
 * sas_features: 32 float features per candidate for vetting (no paper
 * definition exists; the list is in the library's documentation: coverage,
 * time extent, longest epoch run, velocity, SNR statistics, neighbouring
 * candidates in (velocity, bin), residuals of the projected positions inside
 * the bin with their per-time-slice means, their slope against time and
 * their scatter about the fitted line, time-slice fractions, shared epochs).
 *   workspace:  the workspace of the last sas_vote of this plan on this
 *               catalog (n detections): its window index is read.
 *   snr_dev:    device [n] float SNR by catalog index, or NULL (zeros).
 *   cand_dev:   device [n_cand] candidates of this plan (exact bins).
 *   spacing_q8: lattice spacing of the velocity grid (Q8 px/h; the
 *               sas_grid_spec spacing).  Velocities are placed on the lattice
 *               by rounding v / spacing half up; two candidates are
 *               neighbours when those indices and their bins differ by at
 *               most 1 per component.  0 leaves features 9 and 10 at zero.
 *   scratch:    device memory of sas_features_scratch_size(n_cand) bytes or
 *               more (neighbour keys and their sort); unused when
 *               spacing_q8 is 0 (may then be NULL).
 *   feat_dev:   device [n_cand][32] float, row-major.
 * Asynchronous, no allocation.  Errors: SAS_E_INVALID (n_cand >= 2^31,
 * negative spacing), SAS_E_WORKSPACE (workspace or scratch too small).
 */
sas_status sas_features(const sas_plan *plan, const void *workspace, size_t ws_bytes, int64_t n,
                        const float *snr_dev, const sas_candidate *cand_dev, int64_t n_cand,
                        int32_t spacing_q8, void *scratch, size_t scratch_bytes,
                        float *feat_dev, void *stream);

/* Bytes of scratch sas_features needs for n_cand candidates. */
sas_status sas_features_scratch_size(int64_t n_cand, size_t *bytes);

/*
 * Vetting MLP 32 -> 128 -> 128 -> 1 (ReLU), bf16 operands on the matrix
 * cores with FP32 accumulation, FP32 master weights.  Parameters are packed
 * W1 (32 x 128, row-major), b1 (128), W2 (128 x 128), b2 (128), W3 (128),
 * b3 (1): 20865 floats.  Inputs are [n][32] float rows on the device,
 * standardised inside as (x - mean) / std (std 0 counts as 1).  The loss is
 * the batch mean of binary cross-entropy with logits, positives weighted by
 * pos_weight; weight gradients are reduced over the batch in a fixed order,
 * so they are identical from run to run.  The optimiser is AdamW with
 * decoupled weight decay on every parameter.
 */
typedef struct sas_mlp sas_mlp;
#define SAS_MLP_PARAMS 20865

/* Allocate the network for batches of up to max_batch rows; He-uniform
 * weights (bound sqrt(6 / fan_in)) and zero biases from `seed`. */
sas_status sas_mlp_create(int64_t max_batch, uint64_t seed, sas_mlp **mlp_out);
sas_status sas_mlp_destroy(sas_mlp *mlp);
/* Host mean[32] and std[32] of the input standardisation (synchronous). */
sas_status sas_mlp_set_norm(sas_mlp *mlp, const float *mean_host, const float *std_host);
/* Copy the FP32 parameters out (cap >= 20865; *n_out = 20865), or in
 * (n = 20865; resets the optimiser state).  Synchronous. */
sas_status sas_mlp_get_params(const sas_mlp *mlp, float *host, int64_t cap, int64_t *n_out);
sas_status sas_mlp_set_params(sas_mlp *mlp, const float *host, int64_t n);
/*
 * Checkpoints (no paper passage): everything a resumed training needs, so
 * that training resumed from a checkpoint continues bit for bit as the
 * uninterrupted run would.  sas_mlp_save writes, to host memory, a 256-byte
 * text header (one JSON object padded with spaces and ending in a newline:
 * format "sas_mlp", version 1, parameter and input counts, the AdamW step
 * count and the creation seed) followed by float32 little-endian arrays:
 * the FP32 master parameters, the AdamW first and second moments (20865
 * each), and the input mean and std (32 each).  Two-call protocol: *n_out
 * receives the size; a smaller cap returns SAS_E_OVERFLOW.  sas_mlp_load
 * restores all of it (and the bf16 working weights) into a network of any
 * max_batch; SAS_E_INVALID for a wrong size or header.  Both synchronous.
 */
sas_status sas_mlp_save(const sas_mlp *mlp, void *host, int64_t cap, int64_t *n_out);
sas_status sas_mlp_load(sas_mlp *mlp, const void *host, int64_t n);
/* Logits of n rows (any n; processed max_batch rows at a time). */
sas_status sas_mlp_forward(const sas_mlp *mlp, const float *x_dev, int64_t n, float *logits_dev,
                           void *stream);
/* Mean loss (device float) and gradient (device [20865] float) of one batch
 * (1 <= batch <= max_batch), without updating the parameters. */
sas_status sas_mlp_grad(const sas_mlp *mlp, const float *x_dev, const float *y_dev, int64_t batch,
                        float pos_weight, float *loss_dev, float *grad_dev, void *stream);
/* One AdamW training step on a batch; *loss_dev receives its mean loss. */
sas_status sas_mlp_train_step(sas_mlp *mlp, const float *x_dev, const float *y_dev, int64_t batch,
                              float pos_weight, float lr, float beta1, float beta2, float eps,
                              float weight_decay, float *loss_dev, void *stream);

/* ------------------------------------------------------------------------
 * Peaks: collect the candidates of a finished vote in a deterministic order.
 * ---------------------------------------------------------------------- */
#define SAS_ORDER_CANONICAL 0 /* (v_idx, by, bx) ascending */
#define SAS_ORDER_BY_COUNT 1  /* count descending, then (v_idx, by, bx) */

/*
 * sas_peaks: synchronise `stream`, read the result and copy the candidates
 * to out_host in the requested order; with top_k > 0 only the first top_k
 * of that order (the "first clusters with the highest number of
 * detections" of Sec. 3.3 when order is BY_COUNT).
 *   *n_out receives the number of records written.
 * Returns SAS_E_INVALID if the vote flagged bad catalog data (message
 * names the flag), SAS_E_OVERFLOW if the vote found more candidates than
 * cand_cap (then *n_out is the true total and the caller reruns with a
 * larger buffer) or if out_cap is too small (then *n_out is the needed
 * size).  The output is identical for every path, tuning and ordering of
 * the input catalog.
 */
sas_status sas_peaks(const sas_candidate *cand_dev, const sas_vote_result *res_dev,
                     int64_t cand_cap, int32_t order, int64_t top_k, sas_candidate *out_host,
                     int64_t out_cap, int64_t *n_out, void *stream);

/* ------------------------------------------------------------------------
 * Refine, Gather, iterate (Steps 4-6 of Sec. 2.1).
 *
 * Step 4 fits each cluster with the multivariate regression of Sec. 2
 * (independent variable t, responses x and y): slope B (the velocity),
 * intercept c (the position at the reference epoch t0) and error
 * covariance Sigma_eps, all from the mean and covariance of the Minimum
 * Covariance Determinant subset of the cluster's points (t, x, y) instead
 * of the sample ones, which tolerates up to half outliers.  FAST-MCD
 * (Rousseeuw and Van Driessen 1999) approximates that subset: h = (n + 4) / 2
 * points; from n_starts random 4-point starts two C-steps each, the 10
 * lowest determinants iterated until the subset stops changing (at most 30
 * C-steps), the lowest determinant wins.  Step 5 gathers the catalog
 * detections within the radius of the line c + B t (Euclidean, <=) at their
 * epoch's time; Step 6 refits on the gathered set and repeats until it no
 * longer changes (at most 10 rounds).
 * ---------------------------------------------------------------------- */
#define SAS_REFINE_MAX_POINTS 512   /* points of one set (cluster or gathered) */
#define SAS_REFINE_MAX_STARTS 1024

#define SAS_REFINE_CONVERGED 0   /* the gathered set equals the set fitted */
#define SAS_REFINE_MAX_ROUNDS 1  /* still changing after 10 rounds */
#define SAS_REFINE_TOO_SMALL 2   /* a set of fewer than 5 points */
#define SAS_REFINE_NO_START 3    /* every start repeated a point or was degenerate */
#define SAS_REFINE_TOO_LARGE 4   /* a set of more than SAS_REFINE_MAX_POINTS points */
#define SAS_REFINE_BAD_INPUT 5   /* the cluster's CSR range or a member index is invalid */

typedef struct {
    double vx, vy;          /* B: px/h */
    double x0, y0;          /* c: px at t0 (t0 = the earliest epoch holding a detection) */
    double sxx, sxy, syy;   /* Sigma_eps, px^2 */
    int32_t n_points;       /* h of the last fit */
    int32_t n_gathered;     /* detections gathered by the last fit */
    int32_t rounds;         /* fits made (0: none) */
    int32_t status;         /* SAS_REFINE_* */
} sas_refined;              /* 72 bytes */

/*
 * sas_refine_clusters: enqueue Steps 4-6 for n_clusters clusters of the
 * catalog last voted with this dense-path plan and workspace (its window
 * index serves the gather).
 *   x_q8, y_q8, epoch: device [n], the catalog that was voted.
 *   first_dev:   device [n_clusters + 1], CSR offsets into members_dev;
 *   members_dev: device [n_members] catalog indices of each cluster's
 *                detections (any order; for example from the owners that
 *                sas_extract_clusters writes).
 *   starts_dev:  device [n_starts][4] uint32, the random draws of the
 *                FAST-MCD starts (a start takes the points value mod n);
 *                1 <= n_starts <= SAS_REFINE_MAX_STARTS.
 *   radius_q8:   gather radius in Q8 px (0: the plan's bin width Delta x).
 *   out_dev:     device [n_clusters] results.
 *   gathered_dev: device [n_clusters][gather_cap] or NULL: the final
 *                gathered set, catalog indices ascending (the first
 *                min(n_gathered, gather_cap) of them).
 *   subset_dev:  device [n_clusters][SAS_REFINE_MAX_POINTS] or NULL: the
 *                MCD subset of the last fit, ascending (n_points of them).
 * Asynchronous, allocates nothing.  An invalid cluster gets status
 * SAS_REFINE_BAD_INPUT; the call itself checks the arguments on the host.
 * Errors: SAS_E_INVALID (arguments, a plan not on the dense path).
 */
sas_status sas_refine_clusters(const sas_plan *plan, const void *workspace, size_t ws_bytes,
                               const int32_t *x_q8, const int32_t *y_q8, const uint8_t *epoch,
                               int64_t n, const int32_t *first_dev, const int32_t *members_dev,
                               int64_t n_members, int64_t n_clusters, const uint32_t *starts_dev,
                               int32_t n_starts, int32_t radius_q8, sas_refined *out_dev,
                               int32_t *gathered_dev, int32_t gather_cap, int32_t *subset_dev,
                               void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SAS_H */

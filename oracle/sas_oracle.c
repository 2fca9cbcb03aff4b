/*
 * CPU oracle for the catalog shift-and-stack voting transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * What it computes is the plain definition of Steps 1-2 of the algorithm in
 * Sec. 2.1 (Project, Cluster), with the threshold of Step 3 read as "report
 * every histogram bin whose count is at least N_min":
 *
 *   t0      = min over detections i of t[e_i]          (Step 1: reference epoch)
 *   d_e     = t[e] - t0                                 (Q16 hours)
 *   X_ij    = 65536 * x_i - u_j * d_{e_i}               (Q24 px, exact: eqs. 1-2
 *                                                        solved for the position
 *                                                        at t0 under velocity j)
 *   bx_ij   = floor(X_ij / (65536 * b)),  same for y    (Step 2: 2-D histogram at
 *                                                        resolution b = Delta x)
 *   EPOCHS:      c_j(bx,by) = |{ e_i : (bx_ij,by_ij) = (bx,by) }|
 *   DETECTIONS:  c_j(bx,by) = |{ i   : (bx_ij,by_ij) = (bx,by) }|
 *   output: every (j, bx, by, c) with c >= N_min, ordered by (j, by, bx).
 *
 * Weighted counts (the accumulation of a per-detection likelihood instead
 * of an indicator, suggested in the Conclusions): every detection carries
 * an integer weight w_i in [0, 255], and
 *   WEIGHTED_EPOCHS:     c_j(bx,by) = sum over epochs e of the largest w_i
 *                        among the detections of epoch e in the bin,
 *   WEIGHTED_DETECTIONS: c_j(bx,by) = sum of w_i over the bin's detections,
 * with N_min the threshold on that score.  All weights 1 give EPOCHS and
 * DETECTIONS back.
 *
 * Products are formed in 128-bit integers and divided with an explicit floor
 * division (not shifts), so no range assumption is needed here.  Each
 * velocity is handled by sorting its (by, bx, e) triples and walking the runs:
 * slow and plain on purpose.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint32_t v_idx;
    int32_t bx;
    int32_t by;
    uint16_t count;
    uint16_t flags; /* bit 0: count saturated at the reported maximum */
} oracle_cand;

typedef struct {
    int64_t by, bx;
    int32_t e;
    int32_t w;
} triple;

static __int128 floor_div128(__int128 a, __int128 b) /* b > 0 */
{
    __int128 q = a / b; /* C division truncates toward zero */
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

static int cmp_triple(const void *pa, const void *pb)
{
    const triple *a = (const triple *)pa, *b = (const triple *)pb;
    if (a->by != b->by) return a->by < b->by ? -1 : 1;
    if (a->bx != b->bx) return a->bx < b->bx ? -1 : 1;
    if (a->e != b->e) return a->e < b->e ? -1 : 1;
    return 0;
}

/* Reference epoch of Step 1: the earliest time at which the catalog holds a
 * detection.  Returns 0 and leaves *t0 untouched when n == 0. */
static int reference_time(int64_t n, const uint8_t *epoch, const int64_t *t, int64_t *t0)
{
    if (n <= 0) return 0;
    int64_t best = t[epoch[0]];
    for (int64_t i = 1; i < n; ++i)
        if (t[epoch[i]] < best) best = t[epoch[i]];
    *t0 = best;
    return 1;
}

#define MODE_EPOCHS 0
#define MODE_DETECTIONS 1
#define MODE_WEIGHTED_EPOCHS 2
#define MODE_WEIGHTED_DETECTIONS 3

/* Count of the bin held by the sorted run r[0, len) (one epoch after
 * another, by the sort order) in the given mode. */
static int64_t run_count(const triple *r, int64_t len, int32_t mode)
{
    int64_t count = 0, best = 0;
    for (int64_t k = 0; k < len; ++k) {
        const int new_epoch = k == 0 || r[k].e != r[k - 1].e;
        switch (mode) {
        case MODE_EPOCHS:
            if (new_epoch) count += 1;                   /* a new epoch in this bin */
            break;
        case MODE_DETECTIONS:
            count += 1;                                  /* every detection */
            break;
        case MODE_WEIGHTED_EPOCHS:
            if (new_epoch) {                             /* close the previous epoch */
                count += best;
                best = 0;
            }
            if (r[k].w > best) best = r[k].w;            /* largest weight of this epoch */
            break;
        default:
            count += r[k].w;                             /* every detection's weight */
        }
    }
    return count + best;
}

/* One velocity: fills `out` (capacity n) with this velocity's candidates in
 * (by, bx) order and returns how many there are. */
static int64_t one_velocity(int64_t n, const int32_t *x, const int32_t *y, const uint8_t *epoch,
                            const uint8_t *weight, const int64_t *dt, int64_t u, int64_t w,
                            int64_t binw,
                            int32_t n_min, int32_t mode, int32_t count_sat, uint32_t j,
                            triple *scratch, oracle_cand *out)
{
    const __int128 denom = (__int128)binw * 65536;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t d = dt[epoch[i]];
        const __int128 X = (__int128)x[i] * 65536 - (__int128)u * d;
        const __int128 Y = (__int128)y[i] * 65536 - (__int128)w * d;
        scratch[i].bx = (int64_t)floor_div128(X, denom);
        scratch[i].by = (int64_t)floor_div128(Y, denom);
        scratch[i].e = epoch[i];
        scratch[i].w = weight ? weight[i] : 1;
    }
    qsort(scratch, (size_t)n, sizeof(triple), cmp_triple);

    int64_t n_out = 0;
    int64_t i = 0;
    while (i < n) {
        int64_t k = i;
        while (k < n && scratch[k].by == scratch[i].by && scratch[k].bx == scratch[i].bx) ++k;
        const int64_t count = run_count(scratch + i, k - i, mode);
        if (count >= n_min) {
            oracle_cand c;
            c.v_idx = j;
            c.bx = (int32_t)scratch[i].bx;
            c.by = (int32_t)scratch[i].by;
            c.count = (uint16_t)(count > count_sat ? count_sat : count);
            c.flags = (uint16_t)(count > count_sat ? 1 : 0);
            out[n_out++] = c;
        }
        i = k;
    }
    return n_out;
}

/*
 * oracle_vote: candidates of the whole velocity set.
 *   x, y      [n] int32 Q8 px;   epoch [n] in [0, n_epochs)
 *   t_q16     [n_epochs] int64 Q16 h (any origin)
 *   v         [n_v][2] int32 Q8 px/h
 *   binw      bin width, Q8 px (> 0)
 *   weight    [n] in [0, 255] for the weighted modes, NULL otherwise
 *   mode      0 = distinct epochs, 1 = detections, 2 = weighted epochs,
 *             3 = weighted detections
 *   count_sat largest reportable count (255 or 65535)
 *   out/cap   caller buffer; the return value is the total number of
 *             candidates (out holds the first min(total, cap) of them).
 * Returns -1 on invalid arguments or allocation failure.
 */
int64_t oracle_vote(int64_t n, const int32_t *x, const int32_t *y, const uint8_t *epoch,
                    const uint8_t *weight, int32_t n_epochs, const int64_t *t_q16, int64_t n_v,
                    const int32_t *v, int64_t binw, int32_t n_min, int32_t mode,
                    int32_t count_sat, int32_t n_threads, oracle_cand *out, int64_t cap)
{
    if (n < 0 || n_v < 0 || binw <= 0 || n_min < 1 || n_epochs < 1 || mode < 0 || mode > 3 ||
        (mode >= MODE_WEIGHTED_EPOCHS) != (weight != NULL))
        return -1;
    for (int64_t i = 0; i < n; ++i)
        if (epoch[i] >= n_epochs) return -1;
    int64_t t0 = 0;
    if (!reference_time(n, epoch, t_q16, &t0) || n_v == 0) return 0;

    int64_t *dt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_epochs);
    int64_t *per_v = (int64_t *)calloc((size_t)n_v, sizeof(int64_t));
    oracle_cand **res = (oracle_cand **)calloc((size_t)n_v, sizeof(oracle_cand *));
    if (!dt || !per_v || !res) { free(dt); free(per_v); free(res); return -1; }
    for (int32_t e = 0; e < n_epochs; ++e) dt[e] = t_q16[e] - t0;

    int failed = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        triple *scratch = (triple *)malloc(sizeof(triple) * (size_t)(n > 0 ? n : 1));
        oracle_cand *tmp = (oracle_cand *)malloc(sizeof(oracle_cand) * (size_t)(n > 0 ? n : 1));
        if (!scratch || !tmp) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = 0; j < n_v; ++j) {
            if (!scratch || !tmp) continue;
            int64_t k = one_velocity(n, x, y, epoch, weight, dt, v[2 * j], v[2 * j + 1], binw,
                                     n_min, mode, count_sat, (uint32_t)j, scratch, tmp);
            per_v[j] = k;
            if (k > 0) {
                res[j] = (oracle_cand *)malloc(sizeof(oracle_cand) * (size_t)k);
                if (!res[j]) {
#pragma omp atomic write
                    failed = 1;
                } else {
                    memcpy(res[j], tmp, sizeof(oracle_cand) * (size_t)k);
                }
            }
        }
        free(scratch);
        free(tmp);
    }

    int64_t total = 0;
    for (int64_t j = 0; j < n_v; ++j) {
        for (int64_t k = 0; k < per_v[j] && res[j]; ++k) {
            if (total < cap) out[total] = res[j][k];
            ++total;
        }
        free(res[j]);
    }
    free(res);
    free(per_v);
    free(dt);
    return failed ? -1 : total;
}

/*
 * oracle_histogram: the full 2-D histogram of one velocity over a window of
 * bins [bx0, bx0+nbx) x [by0, by0+nby), row-major by (by, bx).  Used by the
 * invariant tests (sum over bins, v = 0 against a library histogram).
 * Detections outside the window are counted into *outside.
 */
int oracle_histogram(int64_t n, const int32_t *x, const int32_t *y, const uint8_t *epoch,
                     const uint8_t *weight, int32_t n_epochs, const int64_t *t_q16, int32_t u,
                     int32_t w, int64_t binw, int32_t mode, int64_t bx0, int64_t by0,
                     int64_t nbx, int64_t nby, int64_t *hist, int64_t *outside)
{
    if (n < 0 || binw <= 0 || n_epochs < 1 || nbx < 0 || nby < 0 || mode < 0 || mode > 3 ||
        (mode >= MODE_WEIGHTED_EPOCHS) != (weight != NULL))
        return -1;
    for (int64_t i = 0; i < n; ++i)
        if (epoch[i] >= n_epochs) return -1;
    memset(hist, 0, sizeof(int64_t) * (size_t)(nbx * nby));
    *outside = 0;
    int64_t t0 = 0;
    if (!reference_time(n, epoch, t_q16, &t0)) return 0;
    /* per bin, a record of which epochs were seen (n_epochs <= 256); in
     * WEIGHTED_EPOCHS, the largest weight (+1) seen per (bin, epoch) */
    uint8_t *seen = NULL;
    int32_t *best = NULL;
    if (mode == MODE_EPOCHS) {
        seen = (uint8_t *)calloc((size_t)(nbx * nby) * 256, 1);
        if (!seen) return -1;
    } else if (mode == MODE_WEIGHTED_EPOCHS) {
        best = (int32_t *)calloc((size_t)(nbx * nby) * 256, sizeof(int32_t));
        if (!best) return -1;
    }
    const __int128 denom = (__int128)binw * 65536;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t d = t_q16[epoch[i]] - t0;
        const __int128 X = (__int128)x[i] * 65536 - (__int128)u * d;
        const __int128 Y = (__int128)y[i] * 65536 - (__int128)w * d;
        const int64_t bx = (int64_t)floor_div128(X, denom) - bx0;
        const int64_t by = (int64_t)floor_div128(Y, denom) - by0;
        if (bx < 0 || bx >= nbx || by < 0 || by >= nby) { *outside += 1; continue; }
        const int64_t cell = by * nbx + bx;
        if (mode == MODE_DETECTIONS) {
            hist[cell] += 1;
        } else if (mode == MODE_WEIGHTED_DETECTIONS) {
            hist[cell] += weight[i];
        } else if (mode == MODE_WEIGHTED_EPOCHS) {
            /* replace this epoch's contribution when a heavier detection comes */
            int32_t *b = &best[cell * 256 + epoch[i]];
            if (weight[i] > *b) {
                hist[cell] += weight[i] - *b;
                *b = weight[i];
            }
        } else if (!seen[cell * 256 + epoch[i]]) {
            seen[cell * 256 + epoch[i]] = 1;
            hist[cell] += 1;
        }
    }
    free(seen);
    free(best);
    return 0;
}

// Host side of libsas: argument validation, work decomposition (plans),
// workspace layout, launches and candidate collection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <cstdio>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "peaks_sort.h"

namespace sas {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

sas_status fail(sas_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

sas_status hip_fail(hipError_t e, const char *what) {
    return fail(SAS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t floor_div(__int128 a, __int128 b) {  // b > 0
    __int128 q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return (int64_t)q;
}

int ilog2_exact(int64_t v) {  // -1 unless v is a power of two
    if (v <= 0 || (v & (v - 1))) return -1;
    int k = 0;
    while ((int64_t(1) << k) < v) ++k;
    return k;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

using Pt = std::pair<__int128, __int128>;

__int128 cross(const Pt &o, const Pt &a, const Pt &b) {
    return (a.first - o.first) * (b.second - o.second) - (a.second - o.second) * (b.first - o.first);
}

// Convex hull (monotone chain), counter-clockwise, exact integer predicates.
std::vector<Pt> convex_hull(std::vector<Pt> p) {
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
    if (p.size() < 3) return p;
    std::vector<Pt> h(2 * p.size());
    size_t k = 0;
    for (size_t i = 0; i < p.size(); ++i) {
        while (k >= 2 && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    for (size_t i = p.size() - 1, t = k + 1; i > 0; --i) {
        while (k >= t && cross(h[k - 2], h[k - 1], p[i - 1]) <= 0) --k;
        h[k++] = p[i - 1];
    }
    h.resize(k - 1);
    return h;
}

// x range of the hull within the band ylo <= y <= yhi (false when empty).
// Approximate in the last bits; callers widen the result.
bool hull_x_range(const std::vector<Pt> &h, long double ylo, long double yhi, long double *xlo,
                  long double *xhi) {
    bool any = false;
    long double lo = 0, hi = 0;
    auto take = [&](long double x) {
        if (!any) { lo = hi = x; any = true; }
        lo = std::min(lo, x);
        hi = std::max(hi, x);
    };
    const size_t n = h.size();
    for (size_t i = 0; i < n; ++i) {
        const long double px = (long double)h[i].first, py = (long double)h[i].second;
        if (py >= ylo && py <= yhi) take(px);
        const Pt &q = h[(i + 1) % n];
        const long double qx = (long double)q.first, qy = (long double)q.second;
        for (long double yl : {ylo, yhi}) {
            if ((py - yl) * (qy - yl) <= 0 && py != qy) take(px + (yl - py) * (qx - px) / (qy - py));
        }
    }
    *xlo = lo;
    *xhi = hi;
    return any;
}

}  // namespace
}  // namespace sas

using namespace sas;

struct sas_plan {
    int device = 0;
    int32_t n_epochs = 0;
    std::vector<int64_t> t;
    int64_t span = 0;
    int32_t binw = 0, log2b = 0, n_min = 1, mode = 0, count_sat = 65535, path = 0;
    int32_t ext[4] = {0, 0, 0, 0};
    int64_t n_v = 0;
    int dense_mode = 0;
    int32_t tile_x = 16, tile_y = 16, vbx = 8, vby = 8, groups = 1, cell_log2 = 11;
    int32_t coarse_log2 = 0, hx = 0, hy = 0, stage_cap = 0, rows = 0, rows_log2 = 0;
    int32_t packed = 0;  // packed 16-bit votes
    int32_t halves = 0;  // 16-bit histogram counts, two histograms by tile
    int32_t ncx = 1, ncy = 1;
    int64_t n_cells = 0, n_items = 0, n_segments = 0, n_tiles = 0, refine_cap = 0;
    // items [0, n_items_kept) are the tiles that can hold a candidate when the
    // earliest epoch e_first holds a detection; the rest are voted otherwise
    int64_t n_items_kept = 0, n_tiles_kept = 0;
    int32_t e_first = 0;
    size_t lds_bytes = 0;
    int32_t *d_vel = nullptr, *d_seg = nullptr, *d_seg_v = nullptr, *d_seg_vel = nullptr;
    int32_t *d_seg_guard = nullptr, *d_items = nullptr;
    std::vector<int32_t> h_items;  // host copy of the work items
    double footprint_cells = 1.0;  // cells of the footprint (batch cost estimates)
    double vmax = 0.0;             // largest |v| of the grid, Q8 px/h
    // sort path
    std::vector<SortBlock> sort_blocks;
    int64_t sort_max_nv = 0;
    int32_t sort_vblock = 0;
    int32_t *d_sort_vel = nullptr, *d_sort_vidx = nullptr;
    hipEvent_t probe[2] = {nullptr, nullptr};
    unsigned long long *counter = nullptr;  // device: LDS atomic vote instructions (probe)
    int64_t *d_t = nullptr;
    std::vector<void *> allocs;
};

namespace {

template <typename T>
sas_status upload(sas_plan *p, T **dst, const std::vector<T> &src) {
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(SAS_E_NOMEM, std::string("plan upload: ") + hipGetErrorString(e));
    p->allocs.push_back(d);
    if (!src.empty()) {
        e = hipMemcpy(d, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "plan upload");
    }
    *dst = (T *)d;
    return SAS_OK;
}

bool is_weighted(int32_t mode) {
    return mode == SAS_MODE_WEIGHTED_EPOCHS || mode == SAS_MODE_WEIGHTED_DETECTIONS;
}

bool refines(int dense_mode) { return dense_mode == kCountRef || dense_mode == kWeightRef; }

struct WsLayout {
    size_t count, offT, blocksum, cellid, rank, sxy, sidx, present, dt, refine_count, item_queue,
        refine;
    size_t keys, keys_alt, hist, hist_blocksum;  // sort path
    size_t total;
};

WsLayout ws_layout(const sas_plan *p, int64_t n) {
    WsLayout L{};
    size_t o = 0;
    const int64_t n_count = p->n_cells + 1;
    const int64_t nb = (n_count + kScanTile - 1) / kScanTile;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    L.count = o; o = align_up(o + sizeof(int32_t) * n_count);
    L.offT = o; o = align_up(o + sizeof(int32_t) * (size_t)p->n_epochs * (p->ncx + 1) * p->ncy);
    L.blocksum = o; o = align_up(o + sizeof(int32_t) * nb);
    L.cellid = o; o = align_up(o + sizeof(int32_t) * nn);
    L.rank = o; o = align_up(o + sizeof(int32_t) * nn);
    L.sxy = o; o = align_up(o + 2 * sizeof(int32_t) * nn);
    L.sidx = o; o = align_up(o + sizeof(int32_t) * nn);
    L.present = o; o = align_up(o + sizeof(int32_t) * kMaxEpochs);
    L.dt = o; o = align_up(o + sizeof(int32_t) * kMaxEpochs);
    L.refine_count = o; o = align_up(o + sizeof(unsigned long long));
    L.item_queue = o; o = align_up(o + sizeof(unsigned long long) * kXcds);
    L.refine = o;
    o = align_up(o + sizeof(int4) * (p->path == SAS_PATH_DENSE && refines(p->dense_mode)
                                         ? p->refine_cap : 1));
    const int64_t keys = p->path == SAS_PATH_SORT ? p->sort_max_nv * std::max<int64_t>(n, 1) : 1;
    const int64_t tiles = (keys + kSortKeysPerTile - 1) / kSortKeysPerTile;
    const int64_t hist = 256 * tiles;
    L.keys = o; o = align_up(o + sizeof(uint64_t) * keys);
    L.keys_alt = o; o = align_up(o + sizeof(uint64_t) * keys);
    L.hist = o; o = align_up(o + sizeof(int32_t) * hist);
    L.hist_blocksum = o; o = align_up(o + sizeof(int32_t) * ((hist + kScanTile - 1) / kScanTile));
    L.total = o;
    return L;
}

PrepBuffers prep_buffers(const WsLayout &L, char *w) {
    PrepBuffers pb;
    pb.count = (int32_t *)(w + L.count);
    pb.offT = (int32_t *)(w + L.offT);
    pb.blocksum = (int32_t *)(w + L.blocksum);
    pb.cellid = (int32_t *)(w + L.cellid);
    pb.rank = (int32_t *)(w + L.rank);
    pb.sxy = (int2 *)(w + L.sxy);
    pb.sidx = (int32_t *)(w + L.sidx);
    pb.present = (int32_t *)(w + L.present);
    pb.dt = (int32_t *)(w + L.dt);
    pb.refine_count = (unsigned long long *)(w + L.refine_count);
    pb.item_queue = (unsigned long long *)(w + L.item_queue);
    return pb;
}

DenseArgs dense_args(const sas_plan *p, const WsLayout &L, char *w, const PrepBuffers &pb,
                     sas_candidate *cand, int64_t cand_cap, sas_vote_result *res) {
    DenseArgs a{};
    a.cat.sxy = pb.sxy;
    a.cat.sidx = pb.sidx;
    a.cat.off = pb.count;
    a.cat.offT = pb.offT;
    a.cat.dt = pb.dt;
    a.cat.n_epochs = p->n_epochs;
    a.cat.ncx = p->ncx;
    a.cat.ncy = p->ncy;
    a.cat.cell_log2 = p->cell_log2;
    a.cat.x0 = p->ext[0];
    a.cat.x1 = p->ext[1];
    a.cat.y0 = p->ext[2];
    a.cat.y1 = p->ext[3];
    a.log2b = p->log2b;
    a.coarse_log2 = p->coarse_log2;
    a.tile_x = p->tile_x;
    a.tile_y = p->tile_y;
    a.hx = p->hx;
    a.hy = p->hy;
    a.stage_cap = p->stage_cap;
    a.rows = p->rows;
    a.rows_log2 = p->rows_log2;
    a.packed = p->packed;
    a.halves = p->halves;
    a.n_min = p->n_min;
    a.count_sat = p->count_sat;
    a.mode_epochs = p->mode == SAS_MODE_EPOCHS ? 1 : 0;
    a.weighted = is_weighted(p->mode) ? p->mode : 0;
    a.vel = p->d_vel;
    a.seg = p->d_seg;
    a.seg_v = p->d_seg_v;
    a.seg_vel = p->d_seg_vel;
    a.seg_guard = p->d_seg_guard;
    a.items = p->d_items;
    a.n_items = p->n_items;
    a.n_items_kept = p->n_items_kept;
    a.e_first = p->e_first;
    a.refine = (int4 *)(w + L.refine);
    a.refine_count = pb.refine_count;
    a.item_queue = pb.item_queue;
    a.refine_cap = refines(p->dense_mode) ? p->refine_cap : 0;
    a.cand = cand;
    a.cand_cap = cand_cap;
    a.res = res;
    a.atomics = p->counter;
    return a;
}

}  // namespace

extern "C" {

const char *sas_status_string(sas_status s) {
    switch (s) {
    case SAS_OK: return "SAS_OK";
    case SAS_E_INVALID: return "SAS_E_INVALID";
    case SAS_E_NOMEM: return "SAS_E_NOMEM";
    case SAS_E_OVERFLOW: return "SAS_E_OVERFLOW";
    case SAS_E_DEVICE: return "SAS_E_DEVICE";
    case SAS_E_UNSUPPORTED: return "SAS_E_UNSUPPORTED";
    case SAS_E_WORKSPACE: return "SAS_E_WORKSPACE";
    default: return "SAS_E_UNKNOWN";
    }
}

const char *sas_last_error(void) { return g_last_error.c_str(); }

const char *sas_version(void) { return "sas-mi355x 0.1 (gfx950)"; }

sas_status sas_plan_create(const sas_plan_desc *d, sas_plan **plan_out) {
    if (!d || !plan_out) return fail(SAS_E_INVALID, "sas_plan_create: null argument");
    *plan_out = nullptr;
    if (d->n_v < 0 || d->n_v >= ((int64_t)1 << 31))
        return fail(SAS_E_INVALID, "sas_plan_create: n_v must be in [0, 2^31)");
    if (d->n_v > 0 && !d->v_host) return fail(SAS_E_INVALID, "sas_plan_create: v_host is null");
    if (d->n_epochs < 1 || d->n_epochs > kMaxEpochs)
        return fail(SAS_E_INVALID, "sas_plan_create: n_epochs must be in [1, 256]");
    if (!d->t_q16) return fail(SAS_E_INVALID, "sas_plan_create: t_q16 is null");
    if (d->binw_q8 <= 0) return fail(SAS_E_INVALID, "sas_plan_create: binw_q8 must be > 0");
    if (d->n_min < 1) return fail(SAS_E_INVALID, "sas_plan_create: n_min must be >= 1");
    if (d->mode < SAS_MODE_EPOCHS || d->mode > SAS_MODE_WEIGHTED_DETECTIONS)
        return fail(SAS_E_INVALID, "sas_plan_create: unknown mode");
    const bool weighted = is_weighted(d->mode);
    if (weighted && d->path == SAS_PATH_SORT)
        return fail(SAS_E_UNSUPPORTED, "sas_plan_create: weighted counts run on the dense path only");
    if (d->count_sat != 255 && d->count_sat != 65535)
        return fail(SAS_E_INVALID, "sas_plan_create: count_sat must be 255 or 65535");
    if (d->path < SAS_PATH_AUTO || d->path > SAS_PATH_SORT)
        return fail(SAS_E_INVALID, "sas_plan_create: unknown path");
    const int32_t *ex = d->extent_q8;
    for (int k = 0; k < 4; ++k)
        if (ex[k] <= -(1 << 30) || ex[k] >= (1 << 30))
            return fail(SAS_E_INVALID, "sas_plan_create: footprint values must satisfy |v| < 2^30");
    if (!(ex[0] < ex[1] && ex[2] < ex[3]))
        return fail(SAS_E_INVALID, "sas_plan_create: empty footprint");
    const int log2b = ilog2_exact(d->binw_q8);
    if (log2b < 0 || log2b > 20)
        return fail(SAS_E_UNSUPPORTED,
                    "sas_plan_create: the GPU path needs a power-of-two bin width <= 2^20 (Q8)");

    int64_t tmin = d->t_q16[0], tmax = d->t_q16[0];
    for (int e = 1; e < d->n_epochs; ++e) {
        tmin = std::min(tmin, d->t_q16[e]);
        tmax = std::max(tmax, d->t_q16[e]);
    }
    const __int128 span128 = (__int128)tmax - tmin;
    if (span128 >= ((__int128)1 << 31))
        return fail(SAS_E_INVALID, "sas_plan_create: epoch times must span less than 2^31 (Q16 h)");
    const int64_t span = (int64_t)span128;

    sas_tuning tu{};
    if (d->tuning) tu = *d->tuning;
    const int64_t n_v = d->n_v;
    const int64_t D = span;  // bound on every t_e - t0
    // natural lattice step Delta x / Delta t (Q8 px/h)
    const int64_t s_ref = span > 0 ? std::max<int64_t>(1, ((int64_t)d->binw_q8 * 65536) / span)
                                   : ((int64_t)1 << 30);
    if (tu.coarse_log2 < -1 || tu.coarse_log2 > 3)
        return fail(SAS_E_INVALID, "sas_plan_create: coarse_log2 must be in [-1, 3]");
    if (tu.refine_cap < 0) return fail(SAS_E_INVALID, "sas_plan_create: refine_cap must be >= 0");
    if (tu.weight_hint < 0 || tu.weight_hint > 255)
        return fail(SAS_E_INVALID, "sas_plan_create: weight_hint must be in [0, 255]");
    if (tu.half_counts < -1 || tu.half_counts > 1)
        return fail(SAS_E_INVALID, "sas_plan_create: half_counts must be -1, 0 or 1");
    if (tu.tile_x < 0 || tu.tile_y < 0 || tu.stage_cap < 0 || tu.vblock_x < 0 || tu.vblock_y < 0)
        return fail(SAS_E_INVALID, "sas_plan_create: negative tuning value");
    if (tu.prune < -1 || tu.prune > 0)
        return fail(SAS_E_INVALID, "sas_plan_create: prune must be 0 or -1");

    // Cell size of the histogram.  A cell of 2^m x 2^m bins counts the
    // detections of all its bins; only cells reaching N_min are refined into
    // exact bins.  Choose the largest m whose expected number of pure-noise
    // cells reaching N_min (Poisson counts at the catalog's mean density)
    // stays small, so that sparse catalogs use far fewer cells per vote.
    const double area = (double)((int64_t)ex[1] - ex[0]) * (double)((int64_t)ex[3] - ex[2]);
    double expected_flags = 0.0;
    int m = 0;
    if (tu.coarse_log2 > 0) {
        m = tu.coarse_log2;
    } else if (tu.coarse_log2 == 0 && tu.n_det_hint > 0 && n_v > 0 &&
               (!weighted || tu.weight_hint > 0)) {
        // A weighted threshold is read as a detection count through the
        // typical weight (the estimate only sizes the filter; a cell that
        // does lift is refined exactly either way).
        const int32_t n_eq = weighted ? std::max<int32_t>(1, (int32_t)std::floor(
                                            (double)d->n_min / tu.weight_hint))
                                      : d->n_min;
        const double lam1 = (double)tu.n_det_hint * (double)d->binw_q8 * d->binw_q8 / area;
        for (int mm = 3; mm >= 1; --mm) {
            const double lam = lam1 * (double)(1 << (2 * mm));
            // P(Poisson(lam) >= n_eq)
            double term = std::exp(-lam), cdf = 0.0;
            for (int k = 0; k < n_eq; ++k) {
                cdf += term;
                term *= lam / (k + 1);
            }
            const double tail = std::max(0.0, 1.0 - cdf);
            const double cells_per_v = area / ((double)d->binw_q8 * d->binw_q8 * (1 << (2 * mm)));
            const double flags = tail * cells_per_v * (double)n_v;
            if (lam < 0.5 * n_eq && flags < 2.0e5) {
                m = mm;
                expected_flags = flags;
                break;
            }
        }
    }
    const int kc = log2b + m;  // log2 of the cell width in Q8
    const int64_t cellw = (int64_t)1 << kc;

    // Lane groups and velocity blocks.  A block of k lattice steps spreads
    // the projections of one detection over about k bins at the last epoch;
    // the guard cells of a tile grow with that spread, so blocks are kept
    // near one cell of spread where possible.
    int G = tu.groups;
    if (G == 0) {
        const double spread8 = 7.0 * (double)d->binw_q8 / (double)cellw;  // 8 steps, in cells
        G = spread8 <= 2.0 ? 1 : 2;
    }
    if (G != 1 && G != 2 && G != 4)
        return fail(SAS_E_INVALID, "sas_plan_create: groups must be 1, 2 or 4");
    const int NV = 64 / G;
    const int32_t vbx = tu.vblock_x ? tu.vblock_x : (G == 4 ? 4 : 8);
    const int32_t vby = tu.vblock_y ? tu.vblock_y : (G == 1 ? 8 : 4);
    if (vbx < 1 || vby < 1 || vbx * vby > NV)
        return fail(SAS_E_INVALID, "sas_plan_create: vblock_x * vblock_y must be in [1, 64 / groups]");

    // velocities: range checks
    for (int64_t j = 0; j < n_v; ++j) {
        for (int a = 0; a < 2; ++a) {
            const int64_t v = d->v_host[2 * j + a];
            if ((__int128)(v < 0 ? -v : v) * span >= ((__int128)1 << 46))
                return fail(SAS_E_UNSUPPORTED, "sas_plan_create: |v| * span too large (>= 2^46 Q24)");
        }
    }

    // Segments: velocities bucketed by blocks of vbx x vby natural lattice
    // steps (row-major over blocks), at most NV per segment.
    const int32_t *V = d->v_host;
    int64_t vxmin = 0, vymin = 0;
    if (n_v > 0) {
        vxmin = V[0];
        vymin = V[1];
        for (int64_t j = 1; j < n_v; ++j) {
            vxmin = std::min<int64_t>(vxmin, V[2 * j]);
            vymin = std::min<int64_t>(vymin, V[2 * j + 1]);
        }
    }
    std::vector<int64_t> kx(n_v), ky(n_v);
    std::vector<int32_t> order(n_v);
    for (int64_t j = 0; j < n_v; ++j) {
        order[j] = (int32_t)j;
        kx[j] = ((int64_t)V[2 * j] - vxmin) / ((int64_t)vbx * s_ref);
        ky[j] = ((int64_t)V[2 * j + 1] - vymin) / ((int64_t)vby * s_ref);
    }
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (ky[a] != ky[b]) return ky[a] < ky[b];
        if (kx[a] != kx[b]) return kx[a] < kx[b];
        if (V[2 * a + 1] != V[2 * b + 1]) return V[2 * a + 1] < V[2 * b + 1];
        if (V[2 * a] != V[2 * b]) return V[2 * a] < V[2 * b];
        return a < b;
    });
    // ceil((dv * D) / 65536) for dv >= 0: a bound on S(v + dv) - S(v) over
    // every epoch, with S(v) = ceil(v d / 65536) and 0 <= d <= D.
    auto spread_q8 = [&](int64_t dv) -> int64_t {
        return (int64_t)(((__int128)dv * D + 65535) >> 16);
    };
    auto ceil_cells = [&](int64_t q8) -> int64_t { return (q8 + cellw - 1) >> kc; };
    std::vector<int32_t> seg, seg_v, seg_vel, seg_guard;
    std::vector<int64_t> seg_ky;  // velocity-block row of each segment
    int64_t guard_x = 0, guard_y = 0, spread_y_max = 0;
    double spread_x_sum = 0, spread_y_sum = 0;
    {
        int64_t i = 0;
        while (i < n_v) {
            int64_t k = i;
            while (k < n_v && k - i < NV && ky[order[k]] == ky[order[i]] &&
                   kx[order[k]] == kx[order[i]])
                ++k;
            int32_t vx_lo = INT32_MAX, vx_hi = INT32_MIN, vy_lo = INT32_MAX, vy_hi = INT32_MIN;
            for (int64_t q = i; q < k; ++q) {
                vx_lo = std::min(vx_lo, V[2 * order[q]]);
                vx_hi = std::max(vx_hi, V[2 * order[q]]);
                vy_lo = std::min(vy_lo, V[2 * order[q] + 1]);
                vy_hi = std::max(vy_hi, V[2 * order[q] + 1]);
            }
            seg.insert(seg.end(), {vx_lo, vx_hi, vy_lo, vy_hi});
            seg_ky.push_back(ky[order[i]]);
            spread_x_sum += (double)spread_q8((int64_t)vx_hi - vx_lo);
            spread_y_sum += (double)spread_q8((int64_t)vy_hi - vy_lo);
            spread_y_max = std::max(spread_y_max, spread_q8((int64_t)vy_hi - vy_lo));
            for (int l = 0; l < NV; ++l) {
                const bool used = i + l < k;
                const int32_t u = used ? V[2 * order[i + l]] : vx_lo;
                const int32_t w = used ? V[2 * order[i + l] + 1] : vy_lo;
                seg_v.push_back(used ? order[i + l] : -1);
                seg_vel.push_back(u);
                seg_vel.push_back(w);
                // left guard: room for S(u) - S(u_lo) plus one Q8 step (the
                // padding detection); right guard: S(u_hi) - S(u)
                const int64_t gx = ceil_cells(spread_q8((int64_t)u - vx_lo) + 1);
                const int64_t gy = ceil_cells(spread_q8((int64_t)w - vy_lo) + 1);
                const int64_t rx = ceil_cells(spread_q8((int64_t)vx_hi - u));
                const int64_t ry = ceil_cells(spread_q8((int64_t)vy_hi - w));
                if (gx >= 32768 || gy >= 32768 || gx + rx >= 32768 || gy + ry >= 32768)
                    return fail(SAS_E_UNSUPPORTED, "sas_plan_create: velocity block spreads over "
                                                   "too many cells; use a smaller vblock");
                seg_guard.push_back((int32_t)(gx | (gy << 16)));
                guard_x = std::max(guard_x, gx + rx);
                guard_y = std::max(guard_y, gy + ry);
            }
            i = k;
        }
    }
    const int64_t n_seg = (int64_t)seg.size() / 4;
    const double spread_x_avg = n_seg ? spread_x_sum / n_seg : 0.0;  // Q8, at the last epoch
    const double spread_y_avg = n_seg ? spread_y_sum / n_seg : 0.0;

    // LDS budget of one workgroup: two workgroups per CU, three for plans with
    // one lane group and packed votes (their kernels keep 80 registers, so
    // that six waves share a SIMD).
    const size_t lds_static = dense_static_lds_bytes();
    const size_t lds_cap = (size_t)kLdsPerCU - lds_static;
    const size_t lds_target2 = (size_t)kLdsPerCU / 2 - 2048 - lds_static;
    const size_t lds_target3 = (size_t)kLdsPerCU / 3 - 2048 - lds_static;
    int cl = tu.cell_log2;
    if (cl < 0 || cl > 30) return fail(SAS_E_INVALID, "sas_plan_create: cell_log2 out of range");
    auto ncells_of = [&](int c, int64_t lo, int64_t hi) { return ((hi - lo) + (1LL << c) - 1) >> c; };
    auto rows_bound = [&](int c, int64_t ty) {  // index rows one tile's window can touch
        return (int64_t)((ty * cellw + spread_y_max - 1) >> c) + 2;
    };
    auto log2_ceil = [](int64_t v) {
        int l = 0;
        while (((int64_t)1 << l) < v) ++l;
        return l;
    };
    // 16-bit histogram counts for the counting cell variants on the dense
    // path (a count never exceeds the window entries of its tile, and the
    // kernel votes a tile that reaches 2^16 with 32-bit counts): one
    // histogram in half the LDS of a 32-bit one (halves = 2), so that tiles
    // get larger or more workgroups fit; one lane group with 32-bit votes
    // instead keeps two histograms alternating by tile in that LDS
    // (halves = 1).
    const bool counts_mode =
        !weighted && (m > 0 || d->mode == SAS_MODE_DETECTIONS ||
                      (d->mode == SAS_MODE_EPOCHS && d->n_epochs > 32));
    const bool dense_path = d->path == SAS_PATH_AUTO || d->path == SAS_PATH_DENSE;
    if (tu.half_counts == 1 && !(counts_mode && dense_path))
        return fail(SAS_E_INVALID, "sas_plan_create: half_counts = 1 needs the dense path and a "
                                   "counting cell variant (detections, more than 32 epochs, or "
                                   "coarse cells)");
    const bool half_ok = tu.half_counts >= 0 && counts_mode && dense_path;
    auto halves_of = [&](bool pk) { return half_ok ? (G == 1 && !pk ? 1 : 2) : 0; };
    // LDS words of a histogram bin
    auto bin_words_of = [&](bool pk) -> int64_t { return halves_of(pk) == 2 ? NV / 2 : NV; };
    // packed 16-bit votes: a histogram row and column span at most 2^16 Q8 px
    // and a row's words fit a 16-bit weight
    auto packs = [&](int64_t tx, int64_t ty) {
        return !weighted && tu.packed >= 0 && ((tx + guard_x) << kc) <= 65536 &&
               ((ty + guard_y) << kc) <= 65536 && (tx + guard_x) * bin_words_of(true) * 4 <= 65535;
    };
    // tile shape: the largest interior under the histogram budget with the
    // best ratio of interior to window area (exact windows: the window adds
    // the average spread of a block to each side length); one lane group
    // looks at packed tiles at three workgroups per CU first
    const bool three_ok = G == 1 && !weighted && tu.packed >= 0;
    int32_t TX = tu.tile_x, TY = tu.tile_y;
    auto search = [&](size_t target, bool packed_only) {
        double best = -1.0;
        for (int ty = 1; ty <= 128; ++ty)
            for (int tx = 1; tx <= 128; ++tx) {
                if (tu.tile_x && tx != tu.tile_x) continue;
                if (tu.tile_y && ty != tu.tile_y) continue;
                const bool pk = packs(tx, ty);
                if (packed_only && !pk) continue;
                // the stage of a packed tile takes half the bytes
                const size_t hist_budget = target * (pk ? 17 : 15) / 20;
                const size_t hb = (size_t)(tx + guard_x) * (ty + guard_y) * bin_words_of(pk) * 4;
                if (hb > hist_budget) continue;
                const double wx = tx + 0.5 * spread_x_avg / cellw + 0.5;
                const double wy = ty + 0.5 * spread_y_avg / cellw + 0.5;
                const double score = (double)tx * ty / (wx * wy);
                if (score > best + 1e-9) {
                    best = score;
                    TX = tx;
                    TY = ty;
                }
            }
        return best >= 0;
    };
    bool three = false;  // three workgroups per CU
    if (!TX || !TY) {
        three = three_ok && search(lds_target3, true);
        if (!three && !search(lds_target2, false)) {
            TX = tu.tile_x ? tu.tile_x : 1;
            TY = tu.tile_y ? tu.tile_y : 1;
        }
    } else {
        three = three_ok && packs(TX, TY);
    }
    const size_t lds_target = three ? lds_target3 : lds_target2;
    if (TX < 1 || TY < 1 || TX > 4096 || TY > 4096)
        return fail(SAS_E_INVALID, "sas_plan_create: tile_x and tile_y must be in [1, 4096]");
    const int64_t HX = TX + guard_x, HY = TY + guard_y;
    const int packed = packs(TX, TY) ? 1 : 0;
    const int halves = halves_of(packed != 0);
    const int64_t bin_words = bin_words_of(packed != 0);
    const size_t entry_bytes = packed ? sizeof(uint32_t) : sizeof(int2);
    if (!cl) cl = kc + 1;  // window-index cells of 2 x 2 histogram cells
    while (ncells_of(cl, ex[0], ex[1]) > 32767 || ncells_of(cl, ex[2], ex[3]) > 32767 ||
           ((((int64_t)d->n_epochs + 7) / 8) << log2_ceil(rows_bound(cl, TY))) > kMaxWavePairs)
        ++cl;
    if (cl > 30) return fail(SAS_E_UNSUPPORTED, "sas_plan_create: footprint too large");
    const int64_t ncx = ncells_of(cl, ex[0], ex[1]), ncy = ncells_of(cl, ex[2], ex[3]);
    const int64_t n_cells = (int64_t)d->n_epochs * ncx * ncy;
    // the column-major copy of the offsets holds E (ncx + 1) ncy words
    if (n_cells >= ((int64_t)1 << 30) || (int64_t)d->n_epochs * (ncx + 1) * ncy >= ((int64_t)1 << 30))
        return fail(SAS_E_INVALID, "sas_plan_create: window index too large; raise cell_log2");
    const int rows_log2 = log2_ceil(rows_bound(cl, TY));
    const size_t hist_bytes = (size_t)HX * HY * bin_words * 4;
    int64_t stage_cap = tu.stage_cap;
    if (!stage_cap) {
        const size_t fixed = dense_lds_bytes(G, (int)HX, (int)HY, 0, packed, halves);
        const size_t room = lds_target > fixed ? (lds_target - fixed) / entry_bytes : 0;
        int64_t want = (int64_t)room;
        if (tu.n_det_hint > 0) {
            const double win = ((double)TX * cellw + 0.5 * spread_x_avg) *
                               ((double)TY * cellw + 0.5 * spread_y_avg);
            want = std::min<int64_t>(want, (int64_t)(1.5 * tu.n_det_hint * win / area) + 256);
        }
        stage_cap = std::max<int64_t>(want, 256);
    }
    // one part per wave of the workgroup, at least two detections each
    stage_cap = std::max<int64_t>((stage_cap + kVoteWaves - 1) / kVoteWaves * kVoteWaves,
                                  2 * kVoteWaves);
    const size_t lds = dense_lds_bytes(G, (int)HX, (int)HY, (int)stage_cap, packed, halves);
    if (HX > 65535 || HY > 65535 || hist_bytes > lds_cap || lds > lds_cap)
        return fail(SAS_E_INVALID, "sas_plan_create: tile + guard cells + stage exceed the LDS of "
                                   "a workgroup; lower tile_x, tile_y, stage_cap or vblock");
    if (weighted && (HX << kc) >= ((int64_t)1 << 24))  // x - S < 2^24 with the weight below it
        return fail(SAS_E_UNSUPPORTED, "sas_plan_create: a weighted tile row spans 2^24 Q8 px or "
                                       "more; lower tile_x or vblock_x");
    {   // window and projected positions are held in 32 bits by the kernels
        int64_t vmax_abs = 0;
        for (int64_t j = 0; j < 2 * n_v; ++j)
            vmax_abs = std::max<int64_t>(vmax_abs, d->v_host[j] < 0 ? -(int64_t)d->v_host[j]
                                                                    : d->v_host[j]);
        const __int128 shift_q8 = ((__int128)vmax_abs * span >> 16) + 1;
        const __int128 tile_q8 = (__int128)(std::max(HX, HY) + 1) << kc;
        const __int128 reach = (__int128)std::max<int64_t>(std::max<int64_t>(
                                   std::abs((int64_t)ex[0]), std::abs((int64_t)ex[1])),
                                   std::max<int64_t>(std::abs((int64_t)ex[2]),
                                                     std::abs((int64_t)ex[3]))) +
                               2 * shift_q8 + 2 * tile_q8;
        if (reach >= ((__int128)1 << 30))
            return fail(SAS_E_UNSUPPORTED, "sas_plan_create: footprint + largest shift + tile "
                                           "must stay below 2^30 Q8 px");
        if (weighted && reach >= ((__int128)1 << 23))  // the index holds 256 x + w in 32 bits
            return fail(SAS_E_UNSUPPORTED, "sas_plan_create: weighted plans need footprint + "
                                           "largest shift + tile below 2^23 Q8 px (32768 px)");
    }

    std::unique_ptr<sas_plan> p(new sas_plan());
    hipError_t he = hipGetDevice(&p->device);
    if (he != hipSuccess) return hip_fail(he, "sas_plan_create: no device");
    p->n_epochs = d->n_epochs;
    p->t.assign(d->t_q16, d->t_q16 + d->n_epochs);
    p->span = span;
    p->binw = d->binw_q8;
    p->log2b = log2b;
    p->n_min = d->n_min;
    p->mode = d->mode;
    p->count_sat = d->count_sat;
    p->path = d->path == SAS_PATH_AUTO ? SAS_PATH_DENSE : d->path;
    std::memcpy(p->ext, ex, sizeof(p->ext));
    p->n_v = n_v;
    p->coarse_log2 = m;
    if (weighted)
        p->dense_mode = d->mode == SAS_MODE_WEIGHTED_DETECTIONS && m == 0 ? kWeightDet : kWeightRef;
    else if (m > 0 || (d->mode == SAS_MODE_EPOCHS && d->n_epochs > 32))
        p->dense_mode = kCountRef;
    else
        p->dense_mode = d->mode == SAS_MODE_DETECTIONS ? kCountDet : kMask32;
    p->refine_cap = tu.refine_cap ? tu.refine_cap
                                  : std::min<int64_t>((int64_t)1 << 26,
                                                      std::max<int64_t>((int64_t)1 << 22,
                                                                        (int64_t)(16 * expected_flags)));
    p->halves = halves;
    p->tile_x = TX;
    p->tile_y = TY;
    p->vbx = vbx;
    p->vby = vby;
    p->groups = G;
    p->hx = (int32_t)HX;
    p->hy = (int32_t)HY;
    p->stage_cap = (int32_t)stage_cap;
    p->rows = (int32_t)rows_bound(cl, TY);
    p->rows_log2 = rows_log2;
    p->packed = packed;
    p->lds_bytes = lds + lds_static;
    p->cell_log2 = cl;
    p->ncx = (int32_t)ncx;
    p->ncy = (int32_t)ncy;
    p->n_cells = n_cells;

    // Tiles of each segment: the projections x - v dt of the footprint for v
    // in the segment's box and dt in [0, span] lie inside the convex hull of
    // the footprint's corners and their shifts by the box corners times span.
    // Every tile row gets the x range of that hull.
    //
    // Coverage.  In EPOCHS mode a bin's count is at most the number of epochs
    // whose detections can reach it.  For a tile of a segment, epoch e can
    // contribute only if its exact window (the tile shifted by S(v, d_e) over
    // the segment's box, as the kernel stages it) meets the footprint; a tile
    // with fewer than N_min such epochs holds no candidate and is not voted.
    // d_e is taken from the earliest scheduled epoch e_first; when that epoch
    // holds no detection the reference epoch is later, and the kernel votes
    // the skipped tiles too (they follow the kept items in the list).
    const __int128 B = (__int128)1 << (16 + kc);  // one histogram cell in Q24
    const __int128 lim_bins = (__int128)1 << 29;
    const bool prune = tu.prune == 0 && d->mode == SAS_MODE_EPOCHS && p->path == SAS_PATH_DENSE;
    int32_t e_first = 0;
    for (int e = 1; e < d->n_epochs; ++e)
        if (d->t_q16[e] < d->t_q16[e_first]) e_first = e;
    std::vector<int64_t> dq(d->n_epochs);
    for (int e = 0; e < d->n_epochs; ++e) dq[e] = d->t_q16[e] - d->t_q16[e_first];
    const int64_t TWq = (int64_t)TX << kc, THq = (int64_t)TY << kc;  // tile size, Q8
    auto shift_of = [](int64_t v, int64_t dd) { return (v * dd + 65535) >> 16; };  // floor
    std::vector<int32_t> items, tail;  // kept items, then the skipped tiles' items
    int64_t n_tiles = 0, n_tiles_kept = 0;
    std::vector<std::array<int64_t, 3>> rows_of_seg;  // (tile row r, first, last tile column)
    std::vector<int32_t> cov;
    for (int64_t sg = 0; sg < n_seg && p->path == SAS_PATH_DENSE; ++sg) {
        rows_of_seg.clear();
        const int32_t vx_lo = seg[4 * sg], vx_hi = seg[4 * sg + 1];
        const int32_t vy_lo = seg[4 * sg + 2], vy_hi = seg[4 * sg + 3];
        std::vector<std::pair<__int128, __int128>> pts;
        for (int cx = 0; cx < 2; ++cx)
            for (int cy = 0; cy < 2; ++cy) {
                const __int128 X = (__int128)ex[cx] * 65536, Y = (__int128)ex[2 + cy] * 65536;
                pts.push_back({X, Y});
                for (int32_t ux : {vx_lo, vx_hi})
                    for (int32_t uy : {vy_lo, vy_hi})
                        pts.push_back({X - (__int128)ux * span, Y - (__int128)uy * span});
            }
        const std::vector<std::pair<__int128, __int128>> hull = convex_hull(pts);
        __int128 ymin = hull[0].second, ymax = hull[0].second;
        for (const auto &q : hull) { ymin = std::min(ymin, q.second); ymax = std::max(ymax, q.second); }
        const __int128 RB = (__int128)TY * B;  // one tile row in Q24
        const int64_t r0 = floor_div(ymin, RB), r1 = floor_div(ymax, RB);
        for (int64_t r = r0; r <= r1; ++r) {
            long double xlo, xhi;
            if (!hull_x_range(hull, (long double)(r * RB), (long double)((r + 1) * RB), &xlo, &xhi))
                continue;
            const int64_t bxl = (int64_t)std::floor(xlo / (long double)B) - 1;
            const int64_t bxh = (int64_t)std::floor(xhi / (long double)B) + 1;
            const int64_t byl = r * TY, byh = r * TY + TY - 1;
            for (int64_t v : {bxl, bxh, byl, byh})
                if (v <= -lim_bins || v >= lim_bins)
                    return fail(SAS_E_UNSUPPORTED, "sas_plan_create: projected bins exceed +-2^29");
            const int64_t t0x = floor_div(bxl, TX), t1x = floor_div(bxh, TX);
            rows_of_seg.push_back({r, t0x, t1x});
            n_tiles += t1x - t0x + 1;
        }
        if (rows_of_seg.empty()) continue;
        // coverage of every (tile row, tile column) of the segment: per epoch
        // the rows and columns whose window meets the footprint form a
        // rectangle; a 2-D difference array sums them
        const int64_t ra0 = rows_of_seg.front()[0], ra1 = rows_of_seg.back()[0];
        int64_t ka0 = rows_of_seg[0][1], ka1 = rows_of_seg[0][2];
        for (const auto &q : rows_of_seg) { ka0 = std::min(ka0, q[1]); ka1 = std::max(ka1, q[2]); }
        const int64_t nr = ra1 - ra0 + 1, nk = ka1 - ka0 + 1;
        const bool seg_prune = prune && nr * nk <= ((int64_t)1 << 22);
        if (seg_prune) {
            cov.assign((size_t)((nr + 1) * (nk + 1)), 0);
            for (int e = 0; e < d->n_epochs; ++e) {
                const int64_t s0 = shift_of(vx_lo, dq[e]), s1 = shift_of(vx_hi, dq[e]);
                const int64_t s2 = shift_of(vy_lo, dq[e]), s3 = shift_of(vy_hi, dq[e]);
                // window rows [oy + s2, oy + s3 + TH) meet [y0, y1): oy = r TH
                const int64_t rb = std::max(ra0, floor_div((__int128)ex[2] - s3 - THq, THq) + 1);
                const int64_t re = std::min(ra1, floor_div((__int128)ex[3] - s2 - 1, THq));
                // window columns [ox + s0, ox + s1 + TW) meet [x0, x1): ox = k TW
                const int64_t kb = std::max(ka0, floor_div((__int128)ex[0] - s1 - TWq, TWq) + 1);
                const int64_t ke = std::min(ka1, floor_div((__int128)ex[1] - s0 - 1, TWq));
                if (rb > re || kb > ke) continue;
                const int64_t r0i = rb - ra0, r1i = re - ra0 + 1, k0i = kb - ka0, k1i = ke - ka0 + 1;
                cov[r0i * (nk + 1) + k0i] += 1;
                cov[r0i * (nk + 1) + k1i] -= 1;
                cov[r1i * (nk + 1) + k0i] -= 1;
                cov[r1i * (nk + 1) + k1i] += 1;
            }
            for (int64_t i = 0; i < nr; ++i)
                for (int64_t k = 0; k < nk; ++k) {
                    int32_t &c = cov[i * (nk + 1) + k];
                    if (i > 0) c += cov[(i - 1) * (nk + 1) + k];
                    if (k > 0) c += cov[i * (nk + 1) + k - 1];
                    if (i > 0 && k > 0) c -= cov[(i - 1) * (nk + 1) + k - 1];
                }
        }
        for (const auto &q : rows_of_seg) {
            const int64_t r = q[0], t0x = q[1], t1x = q[2];
            int64_t k0 = t0x, k1 = t1x;  // kept tile columns [k0, k1]
            if (seg_prune) {
                const int32_t *row = &cov[(r - ra0) * (nk + 1)];  // column k at row[k - ka0]
                while (k0 <= t1x && row[k0 - ka0] < d->n_min) ++k0;
                while (k1 >= k0 && row[k1 - ka0] < d->n_min) --k1;
            }
            auto push = [&](std::vector<int32_t> &dst, int64_t a, int64_t b) {
                if (a > b) return;
                dst.insert(dst.end(), {(int32_t)sg, (int32_t)(r * TY), (int32_t)(a * TX),
                                       (int32_t)(b - a + 1)});
            };
            push(items, k0, k1);
            n_tiles_kept += std::max<int64_t>(0, k1 - k0 + 1);
            if (k0 > k1) {
                push(tail, t0x, t1x);
            } else {
                push(tail, t0x, k0 - 1);
                push(tail, k1 + 1, t1x);
            }
        }
    }
    // Work order: segments of one velocity-block row share their y shifts,
    // so (block row, band of tile rows, segment, tile row) keeps the windows
    // of neighbouring items in one band of the catalog; the kernel gives each
    // XCD a contiguous range of this order, so the workgroups resident on one
    // XCD read from one L2-sized band.  The kept items and the tail are
    // ordered separately.
    for (std::vector<int32_t> *list : {&items, &tail}) {
        std::vector<int32_t> &items = *list;
        const int64_t n_it = (int64_t)items.size() / 4;
        const int64_t band = 4 * (int64_t)TY;
        std::vector<int64_t> idx(n_it);
        for (int64_t q = 0; q < n_it; ++q) idx[q] = q;
        auto key = [&](int64_t q) {
            const int64_t sgq = items[4 * q], tyq = items[4 * q + 1];
            return std::make_tuple(seg_ky[sgq], floor_div(tyq, band), sgq, (int64_t)tyq);
        };
        std::stable_sort(idx.begin(), idx.end(), [&](int64_t u, int64_t w) { return key(u) < key(w); });
        std::vector<int32_t> sorted(items.size());
        for (int64_t q = 0; q < n_it; ++q)
            for (int k = 0; k < 4; ++k) sorted[4 * q + k] = items[4 * idx[q] + k];
        items.swap(sorted);
    }
    p->n_segments = n_seg;
    p->n_items_kept = (int64_t)items.size() / 4;
    items.insert(items.end(), tail.begin(), tail.end());
    p->n_items = (int64_t)items.size() / 4;
    p->n_tiles = n_tiles;
    p->n_tiles_kept = n_tiles_kept;
    p->e_first = e_first;
    if (p->n_items >= ((int64_t)1 << 31))
        return fail(SAS_E_UNSUPPORTED, "sas_plan_create: too many work items");

    // Sort path: blocks of consecutive segments, up to sort_vblock velocities,
    // each with the bin extent every (velocity, detection) of it can reach.
    std::vector<int32_t> sort_vel, sort_vidx;
    if (p->path == SAS_PATH_SORT) {
        int64_t vb = tu.sort_vblock;
        if (vb <= 0)
            vb = tu.n_det_hint > 0 ? std::max<int64_t>(1, std::min<int64_t>(1024,
                                         ((int64_t)1 << 25) / tu.n_det_hint))
                                   : 64;
        const int lb = log2b;
        auto bin_range = [&](int32_t v, int32_t lo, int32_t hi, int64_t *b0, int64_t *b1) {
            // x - S(v, d) for x in [lo, hi), d in [0, D]: S is monotone in d
            const int64_t sD = (int64_t)(((__int128)v * D + 65535) >> 16);
            const int64_t smin = std::min<int64_t>(0, sD), smax = std::max<int64_t>(0, sD);
            *b0 = floor_div((__int128)lo - smax, (__int128)1 << lb);
            *b1 = floor_div((__int128)hi - 1 - smin, (__int128)1 << lb);
        };
        SortBlock cur{};
        int64_t bx0 = 0, bx1 = 0, by0 = 0, by1 = 0;
        auto flush = [&]() -> bool {
            if (cur.nv == 0) return true;
            const int64_t nbx = bx1 - bx0 + 1, nby = by1 - by0 + 1;
            const __int128 span_keys = (__int128)cur.nv * nbx * nby;
            int bits = 0;
            while (((__int128)1 << bits) < span_keys) ++bits;
            if (bits > 56 || nbx >= ((int64_t)1 << 31) || nby >= ((int64_t)1 << 31)) return false;
            cur.bx0 = (int32_t)bx0;
            cur.by0 = (int32_t)by0;
            cur.nbx = (int32_t)nbx;
            cur.nby = (int32_t)nby;
            cur.key_bits = std::max(bits, 1);
            p->sort_blocks.push_back(cur);
            p->sort_max_nv = std::max<int64_t>(p->sort_max_nv, cur.nv);
            cur = SortBlock{};
            cur.v_off = (int32_t)(sort_vidx.size());
            return true;
        };
        for (int64_t sg = 0; sg < n_seg; ++sg)
            for (int l = 0; l < NV; ++l) {
                const int32_t vi = seg_v[sg * NV + l];
                if (vi < 0) continue;
                const int32_t u = seg_vel[2 * (sg * NV + l)], w = seg_vel[2 * (sg * NV + l) + 1];
                int64_t a0, a1, c0, c1;
                bin_range(u, ex[0], ex[1], &a0, &a1);
                bin_range(w, ex[2], ex[3], &c0, &c1);
                if (cur.nv == 0) {
                    bx0 = a0; bx1 = a1; by0 = c0; by1 = c1;
                } else {
                    bx0 = std::min(bx0, a0); bx1 = std::max(bx1, a1);
                    by0 = std::min(by0, c0); by1 = std::max(by1, c1);
                }
                if (bx0 <= -((int64_t)1 << 31) || bx1 >= ((int64_t)1 << 31) ||
                    by0 <= -((int64_t)1 << 31) || by1 >= ((int64_t)1 << 31))
                    return fail(SAS_E_UNSUPPORTED, "sas_plan_create: sort-path bins exceed 32 bits");
                sort_vel.push_back(u);
                sort_vel.push_back(w);
                sort_vidx.push_back(vi);
                ++cur.nv;
                if (cur.nv == vb && !flush())
                    return fail(SAS_E_UNSUPPORTED, "sas_plan_create: sort keys exceed 64 bits; "
                                                   "lower sort_vblock");
            }
        if (!flush())
            return fail(SAS_E_UNSUPPORTED, "sas_plan_create: sort keys exceed 64 bits; lower "
                                           "sort_vblock");
        p->sort_vblock = (int32_t)vb;
    }

    std::vector<int32_t> vel(V, V + 2 * n_v);
    sas_status st;
    if ((st = upload(p.get(), &p->d_vel, vel)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_seg, seg)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_seg_v, seg_v)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_seg_vel, seg_vel)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_seg_guard, seg_guard)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_items, items)) != SAS_OK) goto fail_free;
    p->h_items = items;
    for (int64_t j = 0; j < n_v; ++j)
        p->vmax = std::max(p->vmax, std::sqrt((double)V[2 * j] * V[2 * j] +
                                              (double)V[2 * j + 1] * V[2 * j + 1]));
    p->footprint_cells = std::max(1.0, area / ((double)cellw * (double)cellw));
    if ((st = upload(p.get(), &p->d_t, p->t)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_sort_vel, sort_vel)) != SAS_OK) goto fail_free;
    if ((st = upload(p.get(), &p->d_sort_vidx, sort_vidx)) != SAS_OK) goto fail_free;
    *plan_out = p.release();
    return SAS_OK;
fail_free:
    for (void *a : p->allocs) hipFree(a);
    p->allocs.clear();
    return st;
}

sas_status sas_plan_destroy(sas_plan *p) {
    if (!p) return SAS_OK;
    for (void *a : p->allocs) hipFree(a);
    delete p;
    return SAS_OK;
}

sas_status sas_plan_get_info(const sas_plan *p, sas_plan_info *info) {
    if (!p || !info) return fail(SAS_E_INVALID, "sas_plan_get_info: null argument");
    info->n_items = p->n_items;
    info->n_tiles = p->n_tiles;
    info->n_items_kept = p->n_items_kept;
    info->n_tiles_kept = p->n_tiles_kept;
    info->n_blocks = p->path == SAS_PATH_SORT ? (int64_t)p->sort_blocks.size() : p->n_segments;
    info->path = p->path;
    info->tile_x = p->tile_x;
    info->tile_y = p->tile_y;
    info->vblock_x = p->vbx;
    info->vblock_y = p->vby;
    info->coarse_log2 = p->coarse_log2;
    info->mode_variant = p->dense_mode;
    info->cell_log2 = p->cell_log2;
    info->n_v = p->n_v;
    info->groups = p->groups;
    info->hist_x = p->hx;
    info->hist_y = p->hy;
    info->stage_cap = p->stage_cap;
    info->lds_bytes = (int32_t)p->lds_bytes;
    info->packed = p->packed;
    info->half_counts = p->halves;
    return SAS_OK;
}

sas_status sas_plan_set_probe(sas_plan *p, void *ev_before, void *ev_after) {
    if (!p) return fail(SAS_E_INVALID, "sas_plan_set_probe: null plan");
    if ((ev_before == nullptr) != (ev_after == nullptr))
        return fail(SAS_E_INVALID, "sas_plan_set_probe: give both events or neither");
    p->probe[0] = (hipEvent_t)ev_before;
    p->probe[1] = (hipEvent_t)ev_after;
    return SAS_OK;
}

sas_status sas_plan_set_counter(sas_plan *p, uint64_t *counter_dev) {
    if (!p) return fail(SAS_E_INVALID, "sas_plan_set_counter: null plan");
    p->counter = (unsigned long long *)counter_dev;
    return SAS_OK;
}

sas_status sas_vote_workspace_size(const sas_plan *p, int64_t n, size_t *bytes) {
    if (!p || !bytes || n < 0) return fail(SAS_E_INVALID, "sas_vote_workspace_size: bad argument");
    *bytes = ws_layout(p, n).total;
    return SAS_OK;
}

}  // extern "C"

namespace {

sas_status vote_impl(const sas_plan *p, const int32_t *x_q8, const int32_t *y_q8,
                     const uint8_t *epoch, const uint8_t *weight, int64_t n,
                     sas_candidate *cand_dev, int64_t cand_cap, sas_vote_result *res_dev,
                     void *workspace, size_t ws_bytes, void *stream) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SAS_E_INVALID, "sas_vote: n must be in [0, 2^31)");
    if (n > 0 && (!x_q8 || !y_q8 || !epoch)) return fail(SAS_E_INVALID, "sas_vote: null catalog array");
    if (!res_dev) return fail(SAS_E_INVALID, "sas_vote: null result pointer");
    if (cand_cap < 0 || (cand_cap > 0 && !cand_dev))
        return fail(SAS_E_INVALID, "sas_vote: bad candidate buffer");
    const WsLayout L = ws_layout(p, n);
    if (!workspace || ws_bytes < L.total)
        return fail(SAS_E_WORKSPACE, "sas_vote: workspace smaller than sas_vote_workspace_size()");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(SAS_E_INVALID, "sas_vote: workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)workspace;
    const PrepBuffers pb = prep_buffers(L, w);
    hipError_t e = launch_prep(x_q8, y_q8, epoch, weight, n, p->d_t, p->n_epochs, p->ncx, p->ncy,
                               p->cell_log2, p->ext, p->n_cells, pb, res_dev, s);
    if (e != hipSuccess) return hip_fail(e, "sas_vote: preparation launch");
    if (n == 0 || p->n_v == 0) return SAS_OK;

    if (p->path == SAS_PATH_SORT) {
        if (p->sort_max_nv * n >= ((int64_t)1 << 31))
            return fail(SAS_E_INVALID, "sas_vote: sort block of n x sort_vblock keys exceeds 2^31; "
                                       "lower tuning.sort_vblock");
        SortArgs sa{};
        sa.x = x_q8;
        sa.y = y_q8;
        sa.epoch = epoch;
        sa.n = n;
        sa.dt = pb.dt;
        sa.n_epochs = p->n_epochs;
        sa.log2b = p->log2b;
        sa.n_min = p->n_min;
        sa.count_sat = p->count_sat;
        sa.mode_epochs = p->mode == SAS_MODE_EPOCHS ? 1 : 0;
        sa.vel = p->d_sort_vel;
        sa.v_idx = p->d_sort_vidx;
        sa.keys = (uint64_t *)(w + L.keys);
        sa.keys_alt = (uint64_t *)(w + L.keys_alt);
        sa.hist = (int32_t *)(w + L.hist);
        sa.hist_blocksum = (int32_t *)(w + L.hist_blocksum);
        sa.cand = cand_dev;
        sa.cand_cap = cand_cap;
        sa.res = res_dev;
        if (p->probe[0]) {
            e = hipEventRecord(p->probe[0], s);
            if (e != hipSuccess) return hip_fail(e, "sas_vote: probe");
        }
        for (const SortBlock &b : p->sort_blocks) {
            e = launch_vote_sort_block(sa, b, s);
            if (e != hipSuccess) return hip_fail(e, "sas_vote: sort-path launch");
        }
        if (p->probe[1]) {
            e = hipEventRecord(p->probe[1], s);
            if (e != hipSuccess) return hip_fail(e, "sas_vote: probe");
        }
        return SAS_OK;
    }

    const DenseArgs a = dense_args(p, L, w, pb, cand_dev, cand_cap, res_dev);
    e = launch_vote_dense(p->dense_mode, p->groups, a, s, p->probe[0], p->probe[1]);
    if (e != hipSuccess) return hip_fail(e, "sas_vote: vote launch");
    return SAS_OK;
}

}  // namespace

extern "C" {

sas_status sas_vote(const sas_plan *p, const int32_t *x_q8, const int32_t *y_q8,
                    const uint8_t *epoch, int64_t n, sas_candidate *cand_dev, int64_t cand_cap,
                    sas_vote_result *res_dev, void *workspace, size_t ws_bytes, void *stream) {
    if (!p) return fail(SAS_E_INVALID, "sas_vote: null plan");
    if (is_weighted(p->mode))
        return fail(SAS_E_INVALID, "sas_vote: the plan counts weights; use sas_vote_weighted");
    return vote_impl(p, x_q8, y_q8, epoch, nullptr, n, cand_dev, cand_cap, res_dev, workspace,
                     ws_bytes, stream);
}

sas_status sas_vote_weighted(const sas_plan *p, const int32_t *x_q8, const int32_t *y_q8,
                             const uint8_t *epoch, const uint8_t *weight, int64_t n,
                             sas_candidate *cand_dev, int64_t cand_cap, sas_vote_result *res_dev,
                             void *workspace, size_t ws_bytes, void *stream) {
    if (!p) return fail(SAS_E_INVALID, "sas_vote_weighted: null plan");
    if (!is_weighted(p->mode))
        return fail(SAS_E_INVALID, "sas_vote_weighted: the plan does not count weights; use "
                                   "sas_vote");
    if (n > 0 && !weight) return fail(SAS_E_INVALID, "sas_vote_weighted: null weight array");
    return vote_impl(p, x_q8, y_q8, epoch, weight, n, cand_dev, cand_cap, res_dev, workspace,
                     ws_bytes, stream);
}

sas_status sas_peaks(const sas_candidate *cand_dev, const sas_vote_result *res_dev,
                     int64_t cand_cap, int32_t order, int64_t top_k, sas_candidate *out_host,
                     int64_t out_cap, int64_t *n_out, void *stream) {
    if (!res_dev || !n_out || cand_cap < 0 || out_cap < 0 || top_k < 0)
        return fail(SAS_E_INVALID, "sas_peaks: bad argument");
    if (order != SAS_ORDER_CANONICAL && order != SAS_ORDER_BY_COUNT)
        return fail(SAS_E_INVALID, "sas_peaks: unknown order");
    hipStream_t s = (hipStream_t)stream;
    sas_vote_result r{};
    hipError_t e = hipMemcpyAsync(&r, res_dev, sizeof(r), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "sas_peaks: reading the vote result");
    *n_out = 0;
    if (r.status & SAS_DATA_BAD_EPOCH)
        return fail(SAS_E_INVALID, "sas_peaks: the catalog holds an epoch index >= n_epochs");
    if (r.status & SAS_DATA_OUTSIDE)
        return fail(SAS_E_INVALID, "sas_peaks: a detection lies outside the plan's footprint");
    if (r.status & SAS_DATA_INTERNAL)
        return fail(SAS_E_DEVICE, "sas_peaks: internal error: a tile window exceeded the plan's "
                                  "run table or guard cells");
    if (r.status & SAS_DATA_REFINE_FULL)
        return fail(SAS_E_OVERFLOW, "sas_peaks: more flagged histogram cells than the plan's "
                                    "refinement list holds; raise tuning.refine_cap or use "
                                    "tuning.coarse_log2 = -1");
    if (r.n_cand > cand_cap) {
        *n_out = r.n_cand;
        return fail(SAS_E_OVERFLOW, "sas_peaks: more candidates than the vote buffer held");
    }
    std::vector<sas_candidate> c((size_t)r.n_cand);
    if (r.n_cand > 0) {
        if (!cand_dev) return fail(SAS_E_INVALID, "sas_peaks: null candidate buffer");
        e = hipMemcpyAsync(c.data(), cand_dev, sizeof(sas_candidate) * c.size(),
                           hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "sas_peaks: copying candidates");
    }
    sort_candidates(c, order == SAS_ORDER_BY_COUNT);
    const int64_t k = top_k > 0 ? std::min<int64_t>(top_k, (int64_t)c.size()) : (int64_t)c.size();
    if (k > out_cap || (k > 0 && !out_host)) {
        *n_out = k;
        return fail(SAS_E_OVERFLOW, "sas_peaks: output capacity too small; *n_out holds the size");
    }
    if (k > 0) std::memcpy(out_host, c.data(), sizeof(sas_candidate) * (size_t)k);
    *n_out = k;
    return SAS_OK;
}

}  // extern "C"

struct sas_batch {
    struct Chip {
        sas_batch_chip b;
        size_t ws_off = 0;
        WsLayout L{};
        DenseArgs args{};
    };
    struct Class {
        int mode = 0, groups = 1, packed = 0;
        int32_t *d_items5 = nullptr;
        int64_t n_items = 0, n_kept = 0;
        int32_t hist_words_max = 0;
        size_t lds = 0;
    };
    std::vector<Chip> chips;
    std::vector<Class> classes;
    DenseArgs *d_args = nullptr;
    char *ws = nullptr;
    std::vector<void *> allocs;
    hipEvent_t probe[2] = {nullptr, nullptr};
    unsigned long long *counter = nullptr;
    unsigned long long *queues = nullptr;  // [classes][kXcds] item queues
};

namespace {

constexpr int kMaxBatchClasses = 18;  // 3 cell variants x 3 lane-group counts x 2 vote forms

int batch_class(const sas_plan *p) {
    return (p->dense_mode * 3 + (p->groups == 1 ? 0 : p->groups == 2 ? 1 : 2)) * 2 + p->packed;
}

sas_status batch_layout(const sas_batch_chip *chips, int32_t n_chips, std::vector<size_t> *offs,
                        size_t *total) {
    if (n_chips < 1 || !chips) return fail(SAS_E_INVALID, "batch: no chips");
    size_t o = 0;
    offs->clear();
    for (int32_t c = 0; c < n_chips; ++c) {
        const sas_plan *p = chips[c].plan;
        if (!p) return fail(SAS_E_INVALID, "batch: null plan");
        if (p->path != SAS_PATH_DENSE)
            return fail(SAS_E_INVALID, "batch: every chip needs a dense-path plan");
        if (is_weighted(p->mode))
            return fail(SAS_E_UNSUPPORTED, "batch: weighted plans are voted with sas_vote_weighted");
        if (chips[c].n < 0 || chips[c].n >= ((int64_t)1 << 31))
            return fail(SAS_E_INVALID, "batch: chip n must be in [0, 2^31)");
        offs->push_back(o);
        o = align_up(o + ws_layout(p, chips[c].n).total);
    }
    *total = o;
    return SAS_OK;
}

}  // namespace

extern "C" {

sas_status sas_batch_workspace_size(const sas_batch_chip *chips, int32_t n_chips, size_t *bytes) {
    if (!bytes) return fail(SAS_E_INVALID, "sas_batch_workspace_size: null argument");
    std::vector<size_t> offs;
    return batch_layout(chips, n_chips, &offs, bytes);
}

sas_status sas_batch_create(const sas_batch_chip *chips, int32_t n_chips, void *workspace,
                            size_t ws_bytes, sas_batch **out) {
    if (!out) return fail(SAS_E_INVALID, "sas_batch_create: null argument");
    *out = nullptr;
    std::vector<size_t> offs;
    size_t total = 0;
    sas_status st = batch_layout(chips, n_chips, &offs, &total);
    if (st != SAS_OK) return st;
    if (!workspace || ws_bytes < total)
        return fail(SAS_E_WORKSPACE, "sas_batch_create: workspace smaller than "
                                     "sas_batch_workspace_size()");
    if (((uintptr_t)workspace & 255) != 0)
        return fail(SAS_E_INVALID, "sas_batch_create: workspace must be 256-byte aligned");
    for (int32_t c = 0; c < n_chips; ++c) {
        const sas_batch_chip &b = chips[c];
        if (b.n > 0 && (!b.x_q8 || !b.y_q8 || !b.epoch))
            return fail(SAS_E_INVALID, "sas_batch_create: null catalog array");
        if (!b.res_dev || b.cand_cap < 0 || (b.cand_cap > 0 && !b.cand_dev))
            return fail(SAS_E_INVALID, "sas_batch_create: bad output buffers");
    }
    std::unique_ptr<sas_batch> bt(new sas_batch());
    bt->ws = (char *)workspace;
    std::vector<DenseArgs> args(n_chips);
    for (int32_t c = 0; c < n_chips; ++c) {
        sas_batch::Chip ch;
        ch.b = chips[c];
        ch.ws_off = offs[c];
        ch.L = ws_layout(ch.b.plan, ch.b.n);
        char *w = bt->ws + ch.ws_off;
        ch.args = dense_args(ch.b.plan, ch.L, w, prep_buffers(ch.L, w), ch.b.cand_dev,
                             ch.b.cand_cap, ch.b.res_dev);
        args[c] = ch.args;
        bt->chips.push_back(ch);
    }
    // Merge the chips' items per kernel class: chip-major (largest chips
    // first), each chip's items in the chip's own L2-friendly order.  Cost of
    // a chip: its tiles times (expected votes of a tile + a fixed per-tile
    // cost in vote units).
    struct It {
        int32_t v[5];
    };
    std::vector<double> chip_cost(n_chips, 0.0);
    for (int32_t c = 0; c < n_chips; ++c) {
        const sas_plan *p = chips[c].plan;
        const double dens = (double)chips[c].n / p->footprint_cells;  // detections per cell
        chip_cost[c] = (double)p->n_tiles_kept *
                       ((double)p->tile_x * p->tile_y * dens * (64 / p->groups) + 4096.0);
    }
    std::vector<int32_t> chip_order(n_chips);
    for (int32_t c = 0; c < n_chips; ++c) chip_order[c] = c;
    std::stable_sort(chip_order.begin(), chip_order.end(),
                     [&](int32_t u, int32_t w) { return chip_cost[u] > chip_cost[w]; });
    // Per class: every chip's kept items (chip-major), then every chip's
    // skipped tiles (voted only for a chip whose earliest epoch is empty).
    std::vector<std::vector<It>> per_class(kMaxBatchClasses), tails(kMaxBatchClasses);
    for (int32_t c : chip_order) {
        const sas_plan *p = chips[c].plan;
        if (chips[c].n == 0 || p->n_items == 0) continue;
        const int k = batch_class(p);
        for (int64_t q = 0; q < p->n_items; ++q) {
            It it;
            const int32_t *src = &p->h_items[4 * q];
            const bool kept = q < p->n_items_kept;
            it.v[0] = kept ? c : ~c;  // skipped tiles carry ~chip
            it.v[1] = src[0];
            it.v[2] = src[1];
            it.v[3] = src[2];
            it.v[4] = src[3];
            (kept ? per_class[k] : tails[k]).push_back(it);
        }
    }
    for (int k = 0; k < kMaxBatchClasses; ++k) {
        if (per_class[k].empty() && tails[k].empty()) continue;
        const int64_t n_kept = (int64_t)per_class[k].size();
        per_class[k].insert(per_class[k].end(), tails[k].begin(), tails[k].end());
        const std::vector<It> &v = per_class[k];
        sas_batch::Class cl;
        cl.n_kept = n_kept;
        cl.mode = k / 6;
        cl.groups = (k / 2 % 3 == 0) ? 1 : (k / 2 % 3 == 1) ? 2 : 4;
        cl.packed = k % 2;
        std::vector<int32_t> flat;
        flat.reserve(v.size() * 5);
        for (const It &it : v) flat.insert(flat.end(), it.v, it.v + 5);
        for (int32_t c = 0; c < n_chips; ++c) {
            const sas_plan *p = chips[c].plan;
            if (batch_class(p) != k) continue;
            cl.hist_words_max = std::max(cl.hist_words_max, p->hx * p->hy * (64 / p->groups) /
                                                                (p->halves == 2 ? 2 : 1));
            cl.lds = std::max(cl.lds, dense_lds_bytes(p->groups, p->hx, p->hy, p->stage_cap,
                                                      p->packed, p->halves));
        }
        cl.n_items = (int64_t)v.size();
        void *d = nullptr;
        hipError_t e = hipMalloc(&d, flat.size() * sizeof(int32_t));
        if (e != hipSuccess) {
            for (void *a : bt->allocs) hipFree(a);
            return fail(SAS_E_NOMEM, "sas_batch_create: item table");
        }
        bt->allocs.push_back(d);
        e = hipMemcpy(d, flat.data(), flat.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            for (void *a : bt->allocs) hipFree(a);
            return hip_fail(e, "sas_batch_create: item upload");
        }
        cl.d_items5 = (int32_t *)d;
        bt->classes.push_back(cl);
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(unsigned long long) * kXcds *
                                     std::max<size_t>(1, bt->classes.size()));
    if (e != hipSuccess) {
        for (void *a : bt->allocs) hipFree(a);
        return fail(SAS_E_NOMEM, "sas_batch_create: item queues");
    }
    bt->allocs.push_back(q);
    bt->queues = (unsigned long long *)q;
    void *d = nullptr;
    e = hipMalloc(&d, sizeof(DenseArgs) * n_chips);
    if (e != hipSuccess) {
        for (void *a : bt->allocs) hipFree(a);
        return fail(SAS_E_NOMEM, "sas_batch_create: chip table");
    }
    bt->allocs.push_back(d);
    e = hipMemcpy(d, args.data(), sizeof(DenseArgs) * n_chips, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        for (void *a : bt->allocs) hipFree(a);
        return hip_fail(e, "sas_batch_create: chip table upload");
    }
    bt->d_args = (DenseArgs *)d;
    *out = bt.release();
    return SAS_OK;
}

sas_status sas_batch_destroy(sas_batch *b) {
    if (!b) return SAS_OK;
    for (void *a : b->allocs) hipFree(a);
    delete b;
    return SAS_OK;
}

sas_status sas_batch_set_probe(sas_batch *b, void *ev_before, void *ev_after) {
    if (!b) return fail(SAS_E_INVALID, "sas_batch_set_probe: null batch");
    if ((ev_before == nullptr) != (ev_after == nullptr))
        return fail(SAS_E_INVALID, "sas_batch_set_probe: give both events or neither");
    b->probe[0] = (hipEvent_t)ev_before;
    b->probe[1] = (hipEvent_t)ev_after;
    return SAS_OK;
}

sas_status sas_batch_set_counter(sas_batch *b, uint64_t *counter_dev) {
    if (!b) return fail(SAS_E_INVALID, "sas_batch_set_counter: null batch");
    b->counter = (unsigned long long *)counter_dev;
    return SAS_OK;
}

sas_status sas_vote_batch(const sas_batch *b, void *stream) {
    if (!b) return fail(SAS_E_INVALID, "sas_vote_batch: null batch");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    for (const sas_batch::Chip &ch : b->chips) {
        const sas_plan *p = ch.b.plan;
        char *w = b->ws + ch.ws_off;
        e = launch_prep(ch.b.x_q8, ch.b.y_q8, ch.b.epoch, nullptr, ch.b.n, p->d_t, p->n_epochs, p->ncx,
                        p->ncy, p->cell_log2, p->ext, p->n_cells, prep_buffers(ch.L, w),
                        ch.b.res_dev, s);
        if (e != hipSuccess) return hip_fail(e, "sas_vote_batch: preparation launch");
    }
    if (b->probe[0] && (e = hipEventRecord(b->probe[0], s)) != hipSuccess)
        return hip_fail(e, "sas_vote_batch: probe");
    for (size_t k = 0; k < b->classes.size(); ++k) {
        const sas_batch::Class &cl = b->classes[k];
        e = launch_vote_dense_batch(cl.mode, cl.groups, cl.packed, b->d_args,
                                    (int32_t)b->chips.size(), cl.d_items5, cl.n_items, cl.n_kept,
                                    cl.hist_words_max, cl.lds, b->queues + kXcds * k,
                                    b->counter, s);
        if (e != hipSuccess) return hip_fail(e, "sas_vote_batch: vote launch");
    }
    if (b->probe[1] && (e = hipEventRecord(b->probe[1], s)) != hipSuccess)
        return hip_fail(e, "sas_vote_batch: probe");
    for (const sas_batch::Chip &ch : b->chips) {
        if (!refines(ch.b.plan->dense_mode) || ch.b.n == 0) continue;
        e = launch_refine(ch.args, s);
        if (e != hipSuccess) return hip_fail(e, "sas_vote_batch: refinement launch");
    }
    return SAS_OK;
}

}  // extern "C"

namespace {

struct FeatScratch {
    size_t keys, keys_alt, hist, hist_blocksum, total;
};

FeatScratch feat_scratch_layout(int64_t n_cand) {
    FeatScratch L{};
    const int64_t tiles = (n_cand + kSortKeysPerTile - 1) / kSortKeysPerTile;
    const int64_t hist = 256 * tiles;
    size_t o = 0;
    L.keys = o; o = align_up(o + sizeof(uint64_t) * n_cand);
    L.keys_alt = o; o = align_up(o + sizeof(uint64_t) * n_cand);
    L.hist = o; o = align_up(o + sizeof(int32_t) * hist);
    L.hist_blocksum = o; o = align_up(o + sizeof(int32_t) * ((hist + kScanTile - 1) / kScanTile));
    L.total = o;
    return L;
}

constexpr int64_t kMaxFeatureCands = (int64_t)1 << 31;

}  // namespace

extern "C" sas_status sas_features_scratch_size(int64_t n_cand, size_t *bytes) {
    if (!bytes || n_cand < 0 || n_cand >= kMaxFeatureCands)
        return fail(SAS_E_INVALID, "sas_features_scratch_size: bad argument");
    *bytes = feat_scratch_layout(n_cand).total;
    return SAS_OK;
}

extern "C" sas_status sas_features(const sas_plan *p, const void *workspace, size_t ws_bytes,
                                   int64_t n, const float *snr_dev, const sas_candidate *cand_dev,
                                   int64_t n_cand, int32_t spacing_q8, void *scratch,
                                   size_t scratch_bytes, float *feat_dev, void *stream) {
    if (!p || n < 0 || n_cand < 0 || n_cand >= kMaxFeatureCands || spacing_q8 < 0 ||
        (n_cand > 0 && (!cand_dev || !feat_dev)))
        return fail(SAS_E_INVALID, "sas_features: bad argument");
    if (p->path != SAS_PATH_DENSE)
        return fail(SAS_E_INVALID, "sas_features: needs the window index of a dense-path plan");
    if (is_weighted(p->mode))
        return fail(SAS_E_UNSUPPORTED, "sas_features: indicator plans only (EPOCHS or DETECTIONS)");
    const WsLayout L = ws_layout(p, n);
    if (!workspace || ws_bytes < L.total)
        return fail(SAS_E_WORKSPACE, "sas_features: workspace smaller than sas_vote_workspace_size()");
    const FeatScratch S = feat_scratch_layout(n_cand);
    if (spacing_q8 > 0 && n_cand > 0 && (!scratch || scratch_bytes < S.total))
        return fail(SAS_E_WORKSPACE, "sas_features: scratch smaller than sas_features_scratch_size()");
    if (n_cand == 0 || n == 0) return SAS_OK;
    char *w = (char *)workspace;
    const PrepBuffers pb = prep_buffers(L, w);
    FeatureArgs a{};
    a.cat = dense_args(p, L, w, pb, nullptr, 0, nullptr).cat;
    a.log2b = p->log2b;
    a.span = std::max<int64_t>(p->span, 1);
    a.vmax = p->vmax;
    a.vel = p->d_vel;
    a.snr = snr_dev;
    a.cand = cand_dev;
    a.n_cand = n_cand;
    a.feat = feat_dev;
    a.spacing = spacing_q8;
    if (spacing_q8 > 0) {
        char *s = (char *)scratch;
        a.keys = (uint64_t *)(s + S.keys);
        a.keys_alt = (uint64_t *)(s + S.keys_alt);
        a.hist = (int32_t *)(s + S.hist);
        a.hist_blocksum = (int32_t *)(s + S.hist_blocksum);
    }
    hipError_t e = launch_features(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sas_features: launch");
    return SAS_OK;
}

namespace {

struct ExtractScratch {
    size_t first, blocksum, member, member_epoch, member_cell, inv_first, inv_blocksum,
        inv_cursor, inv, count, dirty, live, open, best, slot, taken, perm, counters, total;
};

ExtractScratch extract_layout(int64_t n, int64_t n_cand, int64_t member_cap) {
    ExtractScratch L{};
    size_t o = 0;
    L.first = o; o = align_up(o + sizeof(int32_t) * (n_cand + 1));
    L.blocksum = o; o = align_up(o + sizeof(int32_t) * ((n_cand + 1 + kScanTile - 1) / kScanTile));
    L.member = o; o = align_up(o + sizeof(int32_t) * member_cap);
    L.member_epoch = o; o = align_up(o + member_cap);
    L.member_cell = o; o = align_up(o + sizeof(int32_t) * member_cap);
    L.inv_first = o; o = align_up(o + sizeof(int32_t) * (n + 1));
    L.inv_blocksum = o; o = align_up(o + sizeof(int32_t) * ((n + 1 + kScanTile - 1) / kScanTile));
    L.inv_cursor = o; o = align_up(o + sizeof(int32_t) * n);
    L.inv = o; o = align_up(o + sizeof(int32_t) * member_cap);
    L.count = o; o = align_up(o + sizeof(int32_t) * n_cand);
    L.dirty = o; o = align_up(o + sizeof(uint32_t) * n_cand);
    L.live = o; o = align_up(o + n);
    L.open = o; o = align_up(o + n_cand);
    L.best = o; o = align_up(o + sizeof(int32_t) * n);
    L.slot = o; o = align_up(o + sizeof(int32_t) * n_cand);
    L.taken = o; o = align_up(o + sizeof(int32_t) * n_cand);
    L.perm = o; o = align_up(o + sizeof(int32_t) * n_cand);
    L.counters = o; o = align_up(o + sizeof(int32_t) * kExtractCounters);
    L.total = o;
    return L;
}

constexpr int64_t kMaxMembers = ((int64_t)1 << 31) - 1;

}  // namespace

extern "C" sas_status sas_extract_scratch_size(int64_t n, int64_t n_cand, int64_t member_cap,
                                               size_t *bytes) {
    if (!bytes || n < 0 || n_cand < 0 || n_cand >= kMaxFeatureCands || member_cap < 0 ||
        member_cap > kMaxMembers)
        return fail(SAS_E_INVALID, "sas_extract_scratch_size: bad argument");
    *bytes = extract_layout(n, n_cand, member_cap).total;
    return SAS_OK;
}

extern "C" sas_status sas_extract_clusters(const sas_plan *p, const void *workspace,
                                           size_t ws_bytes, int64_t n,
                                           const sas_candidate *cand_dev, int64_t n_cand,
                                           int64_t member_cap, void *scratch,
                                           size_t scratch_bytes, sas_candidate *clusters_dev,
                                           int64_t cluster_cap, int32_t *cluster_of_dev,
                                           sas_extract_result *res_dev, int32_t rounds,
                                           void *stream) {
    if (!p || n < 0 || n_cand < 0 || n_cand >= kMaxFeatureCands || member_cap < 0 ||
        member_cap > kMaxMembers || cluster_cap < 0 || !res_dev ||
        (n_cand > 0 && !cand_dev) || (cluster_cap > 0 && !clusters_dev) ||
        (n > 0 && !cluster_of_dev) || rounds < -1 || rounds > kExtractRounds)
        return fail(SAS_E_INVALID, "sas_extract_clusters: bad argument");
    if (p->path != SAS_PATH_DENSE)
        return fail(SAS_E_INVALID, "sas_extract_clusters: needs the window index of a dense-path plan");
    if (is_weighted(p->mode))
        return fail(SAS_E_UNSUPPORTED, "sas_extract_clusters: indicator counts only (EPOCHS or "
                                       "DETECTIONS plans)");
    const WsLayout L = ws_layout(p, n);
    if (!workspace || ws_bytes < L.total)
        return fail(SAS_E_WORKSPACE, "sas_extract_clusters: workspace smaller than sas_vote_workspace_size()");
    const ExtractScratch S = extract_layout(n, n_cand, member_cap);
    if (!scratch || scratch_bytes < S.total)
        return fail(SAS_E_WORKSPACE, "sas_extract_clusters: scratch smaller than sas_extract_scratch_size()");
    char *w = (char *)workspace, *s = (char *)scratch;
    const PrepBuffers pb = prep_buffers(L, w);
    ExtractArgs a{};
    a.cat = dense_args(p, L, w, pb, nullptr, 0, nullptr).cat;
    a.log2b = p->log2b;
    a.n_min = p->n_min;
    a.mode_epochs = p->mode == SAS_MODE_EPOCHS ? 1 : 0;
    a.count_sat = p->count_sat;
    a.vel = p->d_vel;
    a.cand = cand_dev;
    a.n_cand = n_cand;
    a.n = n;
    a.first = (int32_t *)(s + S.first);
    a.scan_blocksum = (int32_t *)(s + S.blocksum);
    a.member = (int32_t *)(s + S.member);
    a.member_epoch = (uint8_t *)(s + S.member_epoch);
    a.member_cell = (int32_t *)(s + S.member_cell);
    a.member_cap = member_cap;
    a.inv_first = (int32_t *)(s + S.inv_first);
    a.inv_blocksum = (int32_t *)(s + S.inv_blocksum);
    a.inv_cursor = (int32_t *)(s + S.inv_cursor);
    a.inv = (int32_t *)(s + S.inv);
    a.count = (int32_t *)(s + S.count);
    a.dirty = (uint32_t *)(s + S.dirty);
    a.live = (uint8_t *)(s + S.live);
    a.open = (uint8_t *)(s + S.open);
    a.best = (int32_t *)(s + S.best);
    a.slot = (int32_t *)(s + S.slot);
    a.taken = (int32_t *)(s + S.taken);
    a.perm = (int32_t *)(s + S.perm);
    a.counters = (int32_t *)(s + S.counters);
    a.clusters = clusters_dev;
    a.cluster_cap = cluster_cap;
    a.cluster_of = cluster_of_dev;
    a.res = res_dev;
    a.rounds = rounds == 0 ? kExtractDefaultRounds : rounds < 0 ? 0 : rounds;
    hipError_t e = launch_extract(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sas_extract_clusters: launch");
    return SAS_OK;
}

extern "C" sas_status sas_refine_clusters(const sas_plan *p, const void *workspace,
                                          size_t ws_bytes, const int32_t *x_q8,
                                          const int32_t *y_q8, const uint8_t *epoch, int64_t n,
                                          const int32_t *first_dev, const int32_t *members_dev,
                                          int64_t n_members, int64_t n_clusters,
                                          const uint32_t *starts_dev, int32_t n_starts,
                                          int32_t radius_q8, sas_refined *out_dev,
                                          int32_t *gathered_dev, int32_t gather_cap,
                                          int32_t *subset_dev, void *stream) {
    if (!p || n < 0 || n >= ((int64_t)1 << 31) || n_members < 0 || n_clusters < 0 ||
        n_clusters >= ((int64_t)1 << 31) || n_starts < 1 || n_starts > SAS_REFINE_MAX_STARTS ||
        radius_q8 < 0 || gather_cap < 0 || (n > 0 && (!x_q8 || !y_q8 || !epoch)) ||
        (n_clusters > 0 && (!first_dev || !out_dev || !starts_dev)) ||
        (n_members > 0 && !members_dev) || (gathered_dev && gather_cap == 0))
        return fail(SAS_E_INVALID, "sas_refine_clusters: bad argument");
    if (p->path != SAS_PATH_DENSE)
        return fail(SAS_E_INVALID, "sas_refine_clusters: needs the window index of a dense-path plan");
    const WsLayout L = ws_layout(p, n);
    if (!workspace || ws_bytes < L.total)
        return fail(SAS_E_WORKSPACE, "sas_refine_clusters: workspace smaller than sas_vote_workspace_size()");
    char *w = (char *)workspace;
    const PrepBuffers pb = prep_buffers(L, w);
    RefineArgs a{};
    a.cat = dense_args(p, L, w, pb, nullptr, 0, nullptr).cat;
    a.weighted = is_weighted(p->mode) ? 1 : 0;
    a.x = x_q8;
    a.y = y_q8;
    a.epoch = epoch;
    a.n = n;
    a.first = first_dev;
    a.members = members_dev;
    a.n_members = n_members;
    a.n_clusters = n_clusters;
    a.starts = starts_dev;
    a.n_starts = n_starts;
    a.radius_px = (double)(radius_q8 ? radius_q8 : p->binw) / 256.0;
    a.out = out_dev;
    a.gathered = gathered_dev;
    a.gather_cap = gather_cap;
    a.subset = subset_dev;
    a.subset_clusters = subset_dev ? n_clusters : 0;
    hipError_t e = launch_refine_clusters(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sas_refine_clusters: launch");
    return SAS_OK;
}

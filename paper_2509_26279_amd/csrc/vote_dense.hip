// Dense LDS voting path for gfx950.
//
// Steps 1-2 of Sec. 2.1 (Project, Cluster) with the Step-3 threshold.  The
// velocity grid is cut into segments of up to NV = 64 / G velocities (a block
// of the velocity lattice).  A workgroup takes a (segment, row of tiles); a
// tile is TX x TY histogram cells (a cell is one bin, or 2^m x 2^m bins for
// the coarse filter below).  For each tile:
//   1. each wave takes the epochs e = wave (mod 8).  Per epoch, the exact
//      window of the original frame whose detections can land in the tile
//      for some velocity of the segment is computed; the window index
//      (detections grouped by epoch, cell row, cell column) gives one run of
//      detections per (epoch, cell row), and a wave scan lays the runs end to
//      end.  The wave then reads that sequence 64 consecutive entries at a
//      time (coalesced) and packs the detections inside the exact window into
//      its part of a stage in LDS, grouped by epoch (large windows are staged
//      in chunks); the next tile is staged right after this one's votes;
//   2. lane = (group g < G, velocity j < NV), and the G
//      groups vote G staged detections per instruction.  With d = t_e - t0
//      and S(v) = ceil(v d / 65536), the bin of Step 2,
//      floor((65536 x - v d) / (65536 b)), equals (x - S(v)) >> log2(b).  The
//      histogram of every lane has guard cells on each side, sized from a
//      bound on S(v) - S(v_lo) over the segment, so that a staged detection
//      always lands inside it: a vote is two subtracts, two shifts, a
//      multiply-add and an or for the address, and one LDS atomic with no
//      return value and no bounds check.  The NV words of a bin are
//      consecutive, so a group's lanes touch NV consecutive banks;
//   3. after a barrier, one pass over the histogram reads and clears it;
//      interior cells at or above N_min are emitted (wavefront ballot + one
//      global atomic per wave) or queued for refinement, and a second
//      barrier ends the tile.  With 16-bit counts (counting variants) lanes
//      j and j + NV / 2 share a word: one lane group with 32-bit votes keeps
//      two histograms that alternate by tile, so the second barrier goes;
//      the other plans keep one histogram in half the LDS (larger tiles, or
//      a third workgroup per CU for one lane group with packed votes).  A
//      tile whose window entries could reach 2^16 takes 32-bit counts.
// Cell variants:
//   kMask32  - EPOCHS with E <= 32: epoch bitmask per cell;
//   kCountDet - DETECTIONS: counter per cell;
//   kCountRef - counter of detections per cell as a filter: a bin can hold
//               N_min distinct epochs (or detections) only if its cell holds
//               N_min detections.  Used for EPOCHS with E > 32 and for coarse
//               cells; k_refine resolves queued cells into exact bins.
//   kWeightDet - weighted detections, single bins: the sum of the weights.
//   kWeightRef - sum of the weights per cell as a filter (it bounds both
//               weighted counts of every bin of the cell); k_refine resolves
//               queued cells.
// Weighted plans keep x as 256 x + w in the window index itself (w < 256 in
// the low byte), so the weight rides along with the position through the
// staging unchanged: the window's x bounds are scaled by 256 too, and the
// bin of (256 x + w) - 256 S shifted by log2(b) + 8 is the bin of x - S.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace sas {
namespace {

constexpr int T = kVoteThreads;
constexpr int NW = T / 64;

struct Shared {
    int32_t dt[kMaxEpochs];
    int4 es[kMaxEpochs];        // per epoch: S(vx_lo), S(vx_hi), S(vy_lo), S(vy_hi) of the segment
    int32_t voted[4];           // window entries staged for tile t % 4 (all waves; summed
                                // before the tile is voted)
    int32_t sv[64];             // segment: v_idx of each velocity lane (-1: unused)
    int32_t svx[64], svy[64];   // segment: velocity of each lane
    int32_t sg[64];             // segment: left guard cells of each lane, gx | gy << 16
    int32_t heads[NW][64];      // per wave: marks of the runs that start in the block being staged
    int32_t bad;
    int32_t spill[2];           // tile t % 2 was staged in chunks (set by its waves)
    int32_t n_spill;            // tiles staged in chunks, not yet added to the result
    int32_t count_on;           // measurement: count the LDS atomic vote instructions
    unsigned long long n_instr; // their number in this workgroup
    unsigned long long ticket;  // the item queue's answer to this workgroup
};

// Epochs per wave whose lane shifts stay in registers over a work item (two
// registers each, or one packed).
constexpr int kEpochRegs = 8;
constexpr int kEpochRegsPacked = 8;  // packed: one register per epoch

// Waves per SIMD the vote kernels are compiled for: 4 (128 registers, two
// workgroups of 8 waves per CU); 6 (80 registers, three workgroups) for one
// lane group with packed votes, whose LDS the planner sizes for three.
template <int G, bool PK>
constexpr int kWavesPerSimd = G == 1 && PK ? 6 : 4;
// Epoch shifts kept in registers by those kernels.
constexpr int kEpochRegsPacked6 = 4;

// ceil(v * d / 65536) for d >= 0: the shift v (t_e - t0) in Q8 pixels,
// rounded so that the floor of the shifted position is exact.
__device__ inline int32_t shift_q8(int32_t v, int32_t d) {
    return (int32_t)(((int64_t)v * (int64_t)d + 65535) >> 16);
}

// Device memory reached through the pointers of the argument struct.  The
// batched kernel reads that struct from a table in device memory, where the
// compiler cannot tell the pointers' address space; flat accesses count
// against the LDS wait counter as well, so every LDS wait of the kernel would
// also wait for the catalog loads in flight.  Accesses through gmem() are
// global accesses.
template <class T>
__device__ __attribute__((always_inline)) inline __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
// The HIP vector types are classes whose operators take generic objects:
// 8- and 16-byte records go through plain vector types.
typedef int32_t gv2i __attribute__((ext_vector_type(2)));
typedef uint32_t gv4u __attribute__((ext_vector_type(4)));
__device__ __attribute__((always_inline)) inline int2 load_g(const int2 *p) {
    const gv2i v = *gmem((const gv2i *)p);
    return make_int2(v.x, v.y);
}
__device__ __attribute__((always_inline)) inline void store_g(void *p, uint32_t x, uint32_t y,
                                                              uint32_t z, uint32_t w) {
    *gmem((gv4u *)p) = gv4u{x, y, z, w};
}

__device__ inline void write_cand(sas_candidate *cand, int64_t idx, uint32_t v_idx, int32_t bx,
                                  int32_t by, uint32_t cnt, uint32_t sat) {
    store_g(cand + idx, v_idx, (uint32_t)bx, (uint32_t)by,
            (cnt > sat ? sat : cnt) | ((cnt > sat ? 1u : 0u) << 16));
}

// Wave-aggregated append: one global atomic per wave; returns the slot of
// this lane (valid when ok).  All lanes of the wave must call.
__device__ inline int64_t wave_append(bool ok, unsigned long long *counter) {
    const uint64_t mask = __ballot(ok);
    if (mask == 0) return 0;
    unsigned long long base = 0;
    if (__lane_id() == 0)
        base = __hip_atomic_fetch_add(gmem(counter), (unsigned long long)__popcll(mask),
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, 0, 64);
    const uint32_t pre = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    return (int64_t)base + pre;
}

// Cell rows/columns of the window index that an axis interval [lo, hi) of
// Q8 positions touches, clamped to the footprint; false when none.
__device__ inline bool cell_span(int64_t lo, int64_t hi, int32_t f0, int32_t f1, int cl, int *c0,
                                 int *c1) {
    if (hi <= f0 || lo >= f1) return false;
    *c0 = (int)((max(lo, (int64_t)f0) - f0) >> cl);
    *c1 = (int)((min(hi, (int64_t)f1) - 1 - f0) >> cl);
    return true;
}

__device__ inline bool cell_span(int32_t lo, int32_t hi, int32_t f0, int32_t f1, int cl, int *c0,
                                 int *c1) {
    if (hi <= f0 || lo >= f1) return false;
    *c0 = (max(lo, f0) - f0) >> cl;
    *c1 = (min(hi, f1) - 1 - f0) >> cl;
    return true;
}

template <int MODE>
constexpr bool weighted_mode() { return MODE == kWeightDet || MODE == kWeightRef; }
template <int MODE>
constexpr bool refined_mode() { return MODE == kCountRef || MODE == kWeightRef; }

template <int MODE>
__device__ inline uint32_t cell_count(uint32_t w) {
    return MODE == kMask32 ? (uint32_t)__popc(w) : w;
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// LDS address of histogram word (iy, ix, lane): iy * row_bytes + (ix << lb) +
// lane_addr (the lane's word in bin 0), as one shift-add and one 24-bit
// multiply-add.
__device__ inline uint32_t hist_addr(uint32_t ix, uint32_t iy, uint32_t row_bytes, uint32_t lb,
                                     uint32_t lane_addr) {
    uint32_t t;
    asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(t) : "v"(ix), "s"(lb), "v"(lane_addr));
    return __umul24(iy, row_bytes) + t;
}

template <int MODE>
__device__ inline void lds_vote(uint32_t addr, uint32_t val) {
    lds_u32 *p = (lds_u32 *)(uintptr_t)addr;
    if (MODE == kMask32)
        __hip_atomic_fetch_or(p, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        __hip_atomic_fetch_add(p, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pack16(int32_t x, int32_t y) {
    return ((uint32_t)x & 0xffffu) | ((uint32_t)y << 16);
}

// Word address of a vote: lane shift (sx, sy) = S(v_j, d) plus the Q8 origin
// of the lane's histogram; bin (ix, iy) = ((x - sx) >> kc, (y - sy) >> kc).
// 32-bit form: two subtracts, two shifts, a shift-add and a 24-bit
// multiply-add.
struct VoteAddr32 {
    typedef int2 Entry;
    uint32_t sx, sy, row_bytes, lane_addr;
    int kc, lb;
    __device__ uint32_t operator()(int2 q) const {
        const uint32_t ix = ((uint32_t)q.x - sx) >> kc;
        const uint32_t iy = ((uint32_t)q.y - sy) >> kc;
        return hist_addr(ix, iy, row_bytes, lb, lane_addr);
    }
    __device__ uint32_t value(int2, uint32_t val) const { return val; }
};

// Weighted form: entries hold (256 x + w, y) and sx is the lane shift
// times 256 (modulo 2^32).  Every staged detection has 0 <= x - S < 2^24
// (planner), so the modular difference is exact; the vote adds w.
struct VoteAddr32W {
    typedef int2 Entry;
    uint32_t sx, sy, row_bytes, lane_addr;
    int kc, lb;
    __device__ uint32_t operator()(int2 q) const {
        const uint32_t ix = ((uint32_t)q.x - sx) >> (kc + 8);
        const uint32_t iy = ((uint32_t)q.y - sy) >> kc;
        return hist_addr(ix, iy, row_bytes, lb, lane_addr);
    }
    __device__ uint32_t value(int2 q, uint32_t) const { return (uint32_t)q.x & 0xffu; }
};

// Packed form, for tiles whose histogram spans at most 2^16 Q8 px in x and
// y: entries and shifts keep the low 16 bits of x (low half) and y (high
// half).  Every staged detection satisfies 0 <= x - sx < 2^16 (guard cells),
// so the halves' differences modulo 2^16 are exact: one packed subtract, one
// packed shift and one dot product (ix * NV * 4 + iy * row_bytes + lane).
struct VoteAddr16 {
    typedef uint32_t Entry;
    us2 s, kcv, wts;
    uint32_t lane_addr;
    __device__ uint32_t operator()(uint32_t q) const {
        const us2 d = __builtin_bit_cast(us2, q) - s;
        return __builtin_amdgcn_udot2(d >> kcv, wts, lane_addr, false);
    }
    __device__ uint32_t value(uint32_t, uint32_t val) const { return val; }
};

// U consecutive votes of lane group g: detections st[g], st[g + G], ...,
// st[g + (U - 1) G].
template <int MODE, int G, int U, class V>
__device__ __attribute__((always_inline)) inline void vote_block(const typename V::Entry *st,
                                                                int g, const V &va,
                                                                uint32_t val) {
    typename V::Entry q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = st[u * G + g];
    uint32_t addr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) addr[u] = va(q[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) lds_vote<MODE>(addr[u], va.value(q[u], val));
}

// Votes of n staged detections st[0, n) of one epoch: lane (g, j) takes
// detections g, g + G, ...  Blocks of 4 G, then 2 G and G detections while
// they last (block-uniform branches, no wasted votes); with G > 1 the last
// partial round is voted by the groups g < n mod G only.
template <int MODE, int G, class V>
__device__ inline void vote_run(const typename V::Entry *st, int32_t n, const V &va,
                                uint32_t val, int g) {
    int32_t i = 0;
    for (; i + 4 * G <= n; i += 4 * G) vote_block<MODE, G, 4>(st + i, g, va, val);
    if (i + 2 * G <= n) {
        vote_block<MODE, G, 2>(st + i, g, va, val);
        i += 2 * G;
    }
    if (i + G <= n) {
        vote_block<MODE, G, 1>(st + i, g, va, val);
        i += G;
    }
    if (G > 1 && i + g < n) vote_block<MODE, G, 1>(st + i, g, va, val);
}

// Window-index row r of epoch e for the item's tile row at oy: the index of
// its cell column 0 in the offsets by column (offT), or -1 when the epoch's
// window misses the footprint in y or touches fewer rows (tile independent).
// The lanes of one epoch hold consecutive rows, so their offsets are
// adjacent words.
__device__ __attribute__((always_inline)) inline int32_t window_row(
    const DenseArgs &a, const Shared &sh, int e, int r, int32_t oy, int32_t H) {
    const PreparedCatalog &c = a.cat;
    if (sh.dt[e] < 0) return -1;
    const int32_t ylo = oy + sh.es[e].z, yhi = oy + sh.es[e].w + H;
    int cy0, cy1;
    if (!cell_span(ylo, yhi, c.y0, c.y1, c.cell_log2, &cy0, &cy1)) return -1;
    if (r == 0 && cy1 - cy0 + 1 > a.rows)  // excluded by the planner
        __hip_atomic_fetch_or(gmem(&a.res->status), (int32_t)SAS_DATA_INTERNAL, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    if (cy0 + r > cy1) return -1;
    return e * (c.ncx + 1) * c.ncy + cy0 + r;  // < 2^30 words (planner)
}

// Run of that row for the tile whose Q8 x origin is oxw: source offset and
// end offset in the window index (0, 0 when the window misses in x).
__device__ __attribute__((always_inline)) inline void window_run(
    const PreparedCatalog &c, const Shared &sh, int e, int32_t row, int32_t oxw, int32_t W,
    int32_t &src, int32_t &end) {
    src = 0;
    end = 0;
    if (row < 0) return;
    int cx0, cx1;
    if (!cell_span(oxw + sh.es[e].x, oxw + sh.es[e].y + W, c.x0, c.x1, c.cell_log2, &cx0,
                   &cx1))
        return;
    src = gmem(c.offT)[row + cx0 * c.ncy];
    end = gmem(c.offT)[row + (cx1 + 1) * c.ncy];
}

// Exclusive scan over the 64 lanes of a wave (all lanes active); *total gets
// the sum.  Data-parallel primitive moves only, no LDS round trips: a
// Hillis-Steele scan inside each row of 16 lanes (row shifts by 1, 2, 4, 8;
// lanes shifted in from outside the row add 0), then lane 15 of rows 0 and 2
// is broadcast into rows 1 and 3, and lane 31 into rows 2 and 3.
__device__ __attribute__((always_inline)) inline int32_t wave_scan(int32_t v, int32_t *total) {
    int32_t x = v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    *total = __builtin_amdgcn_readlane(x, 63);
    return x - v;
}

// Inclusive maximum scan of non-negative values over the 64 lanes of a wave
// (all lanes active), by the same moves as wave_scan.
__device__ __attribute__((always_inline)) inline int32_t wave_max_scan(int32_t v) {
    int32_t x = v;
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return x;
}

// Exact window of epoch e for the tile whose Q8 origin is (oxw, oy).
struct Window {
    int32_t x0, x1, y0, y1;
    __device__ bool holds(int2 q) const {
        return (uint32_t)(q.x - x0) < (uint32_t)(x1 - x0) &&
               (uint32_t)(q.y - y0) < (uint32_t)(y1 - y0);
    }
};

__device__ __attribute__((always_inline)) inline Window window_of(const Shared &sh, int e,
                                                                 int32_t oxw, int32_t oy,
                                                                 int32_t W, int32_t H) {
    const int4 s = sh.es[e];
    return Window{oxw + s.x, oxw + s.y + W, oy + s.z, oy + s.w + H};
}

// A staged entry: the detection (x, y), or its packed low halves.
__device__ inline void put_entry(int2 *dst, int2 q) { *dst = q; }
__device__ inline void put_entry(uint32_t *dst, int2 q) { *dst = pack16(q.x, q.y); }

// Blocks of 64 window-index entries whose loads a wave issues before testing
// any of them (one: measured faster than two, three or four in every kernel,
// whose other waves keep the loads' latency covered).
constexpr int kStageBlocks = 1;

// Dynamic LDS: histogram [HY][HX][NV] words, then the stage (int2), one
// part of stage_cap / NW detections per wave.
// One work item: a segment and a row of ntiles tiles starting at tile column
// txf (cells), tile row ty0.  The histogram is all zero on entry and on exit;
// sh.dt holds the catalog's d_e.
template <int MODE, int G, bool PK>
__device__ void vote_item(const DenseArgs &a, Shared &sh, uint4 *smem4, int32_t sg, int32_t ty0,
                          int32_t txf, int32_t ntiles, int32_t &tseq) {
    constexpr int NV = 64 / G;
    constexpr int LNV = G == 1 ? 6 : G == 2 ? 5 : 4;
    constexpr bool WT = weighted_mode<MODE>();
    static_assert(!(WT && PK), "weighted votes use the 32-bit form");
    typedef typename std::conditional<
        PK, VoteAddr16, typename std::conditional<WT, VoteAddr32W, VoteAddr32>::type>::type VA;
    typedef typename VA::Entry Entry;
    constexpr int ER = !PK ? kEpochRegs : kWavesPerSimd<G, PK> == 6 ? kEpochRegsPacked6
                                                                    : kEpochRegsPacked;
    uint32_t *hist = (uint32_t *)smem4;
    const int hist_words = a.hx * a.hy * NV;  // words of a 32-bit histogram
    // halves = 2 plans hold half of that
    Entry *stage = (Entry *)(hist + (a.halves == 2 ? hist_words / 2 : hist_words));

    const PreparedCatalog &c = a.cat;
    // held in registers: the batched kernel's arguments live in device memory,
    // and the staging's wavefront fences would reload it per block of entries
    const int2 *const sxy = c.sxy;
    const int E = c.n_epochs;
    const int tid = threadIdx.x, lane = __lane_id();
    // the wave index in a scalar register: the per-epoch and per-chunk
    // decisions that depend on it are then scalar branches
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = G == 1 ? 0 : lane >> LNV, j = lane & (NV - 1);
    const int kc = a.log2b + a.coarse_log2;
    const int32_t cellw = (int32_t)1 << kc;
    const int32_t W = a.tile_x << kc, H = a.tile_y << kc;  // tile size, Q8
    const uint32_t nmin = (uint32_t)a.n_min;
    // 16-bit counts (counting modes): velocity lanes j and j + NV / 2 add 1
    // and 2^16 to one word of a bin's NV / 2.  halves = 1 (G = 1, 32-bit
    // votes): tiles alternate between two such histograms in the LDS of one
    // 32-bit histogram, and a tile whose window entries could reach 2^16 is
    // voted in the 32-bit form over both.  halves = 2: one such histogram in
    // half the LDS (larger tiles, or three workgroups per CU), and a tile
    // whose entries could reach 2^16 is voted twice with 32-bit counts, by the
    // lanes j < NV / 2 and then by the others, each pass read out on its own
    // (block uniform).
    constexpr bool kHalvesOk = MODE == kCountDet || MODE == kCountRef;
    // the planner's forms: two histograms only for one lane group with
    // 32-bit votes, one histogram for the rest
    const bool hv = G == 1 && !PK && kHalvesOk && a.halves == 1;
    const bool hs = (G > 1 || PK) && kHalvesOk && a.halves == 2;
    const int LR = a.rows_log2;  // run rows per epoch: 2^LR
    const int32_t vx_lo = gmem(a.seg)[4 * sg], vx_hi = gmem(a.seg)[4 * sg + 1];
    const int32_t vy_lo = gmem(a.seg)[4 * sg + 2], vy_hi = gmem(a.seg)[4 * sg + 3];
    __syncthreads();  // the previous item no longer reads the segment tables
    if (tid < NV) {
        const int64_t o = (int64_t)sg * NV + tid;
        sh.sv[tid] = gmem(a.seg_v)[o];
        sh.svx[tid] = gmem(a.seg_vel)[2 * o];
        sh.svy[tid] = gmem(a.seg_vel)[2 * o + 1];
        sh.sg[tid] = gmem(a.seg_guard)[o];
    }
    if (tid < E) {  // shifts of the segment's box edges
        const int32_t d = sh.dt[tid];
        sh.es[tid] = d >= 0 ? make_int4(shift_q8(vx_lo, d), shift_q8(vx_hi, d), shift_q8(vy_lo, d),
                                        shift_q8(vy_hi, d))
                            : make_int4(0, 0, 0, 0);
    }
    if (tid == 0) sh.bad = 0;
    __syncthreads();
    const int32_t my_vx = sh.svx[j], my_vy = sh.svy[j];
    const int32_t my_gx = sh.sg[j] & 0xffff, my_gy = sh.sg[j] >> 16;
    const int32_t oy = ty0 * cellw;
    // Q8 origin of this lane's histogram row 0: (ty0 - gy) cells
    const uint32_t oy_lane = (uint32_t)(ty0 - my_gy) * (uint32_t)cellw;
    // The current tile's histogram form (block uniform):
    //   kForm32: 32-bit counts, NV words per bin;
    //   kFormHalves: 16-bit halves, NV / 2 words per bin (halves = 1: the
    //     histogram of tile t % 2; halves = 2: the only one);
    //   kFormHalfLanes: 32-bit counts of the lanes j with j / (NV / 2) equal to
    //     the pass, NV / 2 words per bin (the other lanes add 0);
    // with its row bytes, the lane's increment, the log2 of a bin's bytes and
    // the LDS address of the lane's word in bin 0.
    enum { kForm32 = 0, kFormHalves = 1, kFormHalfLanes = 2 };
    const uint32_t hist_base = (uint32_t)(uintptr_t)(lds_u32 *)hist;
    int form = kForm32, fpass = 0;
    uint32_t row_bytes = 0, cval = 1, lane_addr = 0;
    int lbt = 0;
    us2 wts;  // packed form: (bytes of a bin, row bytes)
    const auto set_form = [&](int f, int32_t t, int pass) __attribute__((always_inline)) {
        const int nc = f == kForm32 ? NV : NV / 2;  // words per bin
        form = f;
        fpass = pass;
        row_bytes = (uint32_t)(a.hx * nc * 4);
        const bool hi = j >= NV / 2;
        cval = f == kFormHalves      ? (hi ? 65536u : 1u)
               : f == kFormHalfLanes ? (hi == (pass != 0) ? 1u : 0u)
                                     : 1u;
        lbt = f == kForm32 ? LNV + 2 : LNV + 1;
        wts = us2{(unsigned short)(nc * 4), (unsigned short)row_bytes};
        lane_addr = hist_base + (uint32_t)((f == kForm32 ? j : (j & (NV / 2 - 1))) * 4) +
                    (f == kFormHalves && hv ? (uint32_t)(t & 1) * (uint32_t)(hist_words * 2) : 0u);
    };
    set_form(hs ? kFormHalves : kForm32, 0, 0);

    // Lane shifts of this wave's epochs e = wave + k NW (k < ER), kept in
    // registers for the whole item with the Q8 origin of the lane's
    // histogram added (row 0 at ty0 - gy cells, column 0 at tx0 - gx cells of
    // the current tile; packed: low 16 bits of x and y in one register).  The
    // window of any tile lands inside every lane's histogram (tile
    // independent; checked here).
    const uint32_t ox_lane0 = (uint32_t)(txf - my_gx) * (uint32_t)cellw;
    int32_t Sx[ER], Sy[PK ? 1 : ER];
    bool bad = false;
    const auto guard_fails = [&](int e, int64_t sxe, int64_t sye) __attribute__((always_inline)) {
        const int64_t gxq = (int64_t)my_gx << kc, gyq = (int64_t)my_gy << kc;
        const int4 s = sh.es[e];
        return (int64_t)s.x - sxe - 1 + gxq < 0 || (int64_t)s.z - sye - 1 + gyq < 0 ||
               (int64_t)s.y - sxe + W - 1 + gxq >= ((int64_t)a.hx << kc) ||
               (int64_t)s.w - sye + H - 1 + gyq >= ((int64_t)a.hy << kc);
    };
#pragma unroll
    for (int k = 0; k < ER; ++k) {
        const int e = wave + k * NW;
        int32_t sxe = 0, sye = 0;
        if (e < E) {
            const int32_t d = sh.dt[e];
            if (d >= 0) {
                sxe = shift_q8(my_vx, d);
                sye = shift_q8(my_vy, d);
                bad |= guard_fails(e, sxe, sye);
            }
        }
        if (PK) {
            Sx[k] = (int32_t)pack16(sxe + (int32_t)ox_lane0, sye + (int32_t)oy_lane);
        } else {
            Sx[k] = (int32_t)((uint32_t)(sxe + (int32_t)ox_lane0) << (WT ? 8 : 0));
            Sy[PK ? 0 : k] = sye + (int32_t)oy_lane;
        }
    }
    for (int e = wave + ER * NW; e < E; e += NW) {  // epochs past the registers
        const int32_t d = sh.dt[e];
        if (d >= 0) bad |= guard_fails(e, shift_q8(my_vx, d), shift_q8(my_vy, d));
    }
    const us2 kcv = {(unsigned short)kc, (unsigned short)kc};
    // vote address of lane shift (sx, sy) (full Q8 values; packed: low bits)
    const auto vote_addr = [&](int32_t sx, int32_t sy) __attribute__((always_inline)) {
        if constexpr (PK) {
            return VoteAddr16{__builtin_bit_cast(us2, (uint32_t)sx), kcv, wts, lane_addr};
        } else {
            return VA{(uint32_t)sx, (uint32_t)sy, row_bytes, lane_addr, kc, lbt};
        }
    };

    // Each wave stages and votes its own epochs e = wave + NW k (k < KW)
    // without waiting for the others: its (epoch, index row) pairs
    // q = (k << LR) + r sit in two slots of its lanes (q = lane, 64 + lane),
    // their runs are laid out by wave scans, and the detections inside the
    // exact windows are packed epoch-major into the wave's part of the stage.
    const int KW = E > wave ? (E - wave + NW - 1) / NW : 0;
    const int nq = KW << LR;  // <= 128 (planner)
    const int32_t wcap = a.stage_cap / NW;
    Entry *wst = stage + wave * wcap;
    int32_t rsb[2], rlen[2], rpre[2];  // per slot: run source - position, length, position
    int32_t Mw = 0;              // this wave's window-index entries of the tile (wave uniform)
    int32_t my_b = 0, my_n = 0;  // lane k < KW: stage start and count of epoch k
    // lane k < KW: d of epoch wave + k NW.  The per-epoch loop takes it with a
    // lane read: an LDS load there would wait for every vote the wave has in
    // flight.
    const int32_t my_d = lane < KW ? sh.dt[wave + lane * NW] : -1;
    int32_t rowb[2];             // window-index row of each slot's pair (-1: none)
    // epoch of slot s2's pair (clamped for empty slots)
    const auto pair_epoch = [&](int s2) __attribute__((always_inline)) {
        return wave + NW * min((s2 * 64 + lane) >> LR, max(KW - 1, 0));
    };
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        const int q = s2 * 64 + lane;
        rowb[s2] = q < nq ? window_row(a, sh, pair_epoch(s2), q & ((1 << LR) - 1), oy, H) : -1;
    }

    // a tile's run bounds (window-index offsets), loaded ahead of the scans
    int32_t src[2], end[2];
    const auto run_bounds = [&](int32_t oxw) __attribute__((always_inline)) {
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
            window_run(c, sh, pair_epoch(s2), rowb[s2], oxw, W, src[s2], end[s2]);
    };
    // Wave priorities: the window runs and the staging gate the next tile
    // and run at priority 2, the read-out at 1; the votes, which other waves
    // of the CU keep issuing, at 0.
    const auto runs = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_s_setprio(2);
        // the bounds are consumed here and no earlier: nothing that waits for
        // their loads is moved above the votes they overlap
        asm volatile("" : "+v"(src[0]), "+v"(end[0]), "+v"(src[1]), "+v"(end[1]));
        int32_t t0, t1;
        rlen[0] = end[0] - src[0];
        rlen[1] = end[1] - src[1];
        rpre[0] = wave_scan(rlen[0], &t0);
        rpre[1] = t0 + wave_scan(rlen[1], &t1);
        rsb[0] = src[0] - rpre[0];
        rsb[1] = src[1] - rpre[1];
        Mw = t0 + t1;
    };
    // The entries [c0, c0 + wcap) of the wave's runs (in pair order) that lie
    // in their epoch's exact window, packed into the wave's stage.  Lane l
    // takes entries c0 + 64 i + l, so that the loads of a block of 64 entries
    // read a few consecutive stretches of the index.  The pair owning an
    // entry is the last non-empty run starting at or before it: each block's
    // run starts are marked in the wave's row of sh.heads (pair + 1), and a
    // lane takes the nearest mark at or below it, else the previous block's
    // owner.  kStageBlocks blocks are loaded before any is tested.
    int32_t *const hd = sh.heads[wave];
    const auto stage_chunk = [&](int32_t oxw, int32_t c0) __attribute__((always_inline)) {
        __builtin_amdgcn_s_setprio(2);
        const int32_t c1 = min(c0 + wcap, Mw);
        const bool two = nq > 64;  // slot 1 holds pairs (wave uniform)
        // owner of entry c0: its run may have started in an earlier chunk
        int32_t own;
        {
            const uint64_t m0 = __ballot(rpre[0] <= c0 && c0 < rpre[0] + rlen[0]);
            const uint64_t m1 = __ballot(rpre[1] <= c0 && c0 < rpre[1] + rlen[1]);
            own = m0 ? __builtin_ctzll(m0) : m1 ? 64 + __builtin_ctzll(m1) : 0;
        }
        // lane k < KW: position of epoch k's first entry, clamped to the chunk
        const int qk = min(lane, 31) << LR;
        const int32_t pk0 = __shfl(rpre[0], qk & 63, 64), pk1 = __shfl(rpre[1], qk & 63, 64);
        const int32_t pk = min(max(lane < KW ? (qk < 64 ? pk0 : pk1) : Mw, c0), c1);
        int32_t mb = 0, kept = 0;
        constexpr int SB = kStageBlocks;
        for (int32_t b0 = c0; b0 < c1; b0 += SB * 64) {
            int2 ent[SB];
            int32_t ek[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int32_t P0 = b0 + 64 * u, p = P0 + lane;
                ent[u] = make_int2(0, 0);
                ek[u] = 0;
                if (P0 >= c1) break;  // wave uniform
                if (rlen[0] > 0 && (uint32_t)(rpre[0] - P0) < 64u) hd[rpre[0] - P0] = lane + 1;
                if (two && rlen[1] > 0 && (uint32_t)(rpre[1] - P0) < 64u)
                    hd[rpre[1] - P0] = lane + 65;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int32_t h = hd[lane];
                hd[lane] = 0;
                // marks grow with the position: the scan's maximum is the last one
                const int32_t hm = wave_max_scan(h);
                const int32_t q = hm ? hm - 1 : own;
                own = __builtin_amdgcn_readlane(q, 63);
                int32_t sb = __shfl(rsb[0], q & 63, 64);
                if (two) {
                    const int32_t sbh = __shfl(rsb[1], q & 63, 64);
                    sb = q < 64 ? sb : sbh;
                }
                if (p < c1) {
                    ent[u] = load_g(sxy + p + sb);
                    ek[u] = q >> LR;
                }
            }
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int32_t P0 = b0 + 64 * u;
                if (P0 >= c1) break;  // wave uniform
                Window w = window_of(sh, wave + NW * ek[u], oxw, oy, W, H);
                if (WT) {  // the index holds 256 x + w
                    w.x0 = (int32_t)((uint32_t)w.x0 << 8);
                    w.x1 = (int32_t)((uint32_t)w.x1 << 8);
                }
                const bool keep = P0 + lane < c1 && w.holds(ent[u]);
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const uint32_t at = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
                    put_entry(wst + kept + (int32_t)at, ent[u]);
                }
                if (pk < c1 && (uint32_t)(pk - P0) < 64u)
                    mb = kept + __popcll(km & ((1ull << (pk - P0)) - 1));
                kept += __popcll(km);
            }
        }
        if (pk >= c1) mb = kept;
        // lane k < KW: stage start and count of epoch k's entries
        my_b = mb;
        const int32_t nb = __shfl(my_b, min(lane + 1, 63), 64);
        my_n = lane < KW ? nb - my_b : 0;
        if (sh.count_on) {  // measurement: the chunk's votes take ceil(n / G) instructions per epoch
            int32_t tot;
            wave_scan((my_n + G - 1) / G, &tot);
            if (lane == 0 && tot) atomicAdd(&sh.n_instr, (unsigned long long)tot);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_s_setprio(0);
    };

    run_bounds(txf * cellw);
    runs();
    if (Mw > 0) {
        stage_chunk(txf * cellw, 0);
        if (lane == 0) atomicAdd(&sh.voted[tseq & 3], Mw);
    }
    // This barrier publishes the guard check and completes the first tile's
    // staged total (with 16-bit counts every tile's form follows from it).
    if (bad) sh.bad = 1;
    __syncthreads();
    if (sh.bad) {  // excluded by the planner's guard cells; block uniform
        if (tid == 0) {
            __hip_atomic_fetch_or(gmem(&a.res->status), (int32_t)SAS_DATA_INTERNAL, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            sh.voted[tseq & 3] = 0;  // the first tile is not voted
        }
        return;
    }
    int32_t staged = sh.voted[tseq & 3];  // this tile's total (block uniform)
    for (int32_t ti = 0; ti < ntiles; ++ti, ++tseq) {
        const int32_t tx0 = txf + ti * a.tile_x;
        const int32_t ox = tx0 * cellw;
        const uint32_t ox_lane = (uint32_t)(tx0 - my_gx) * (uint32_t)cellw;
        const bool next = ti + 1 < ntiles;  // block uniform
        const int32_t oxn = ox + a.tile_x * cellw;
        // the next tile's run bounds load while this tile is voted
        if (next) run_bounds(oxn);
        if (hv) {
            // a count is at most the tile's window entries; from 2^16 on the
            // tile takes the 32-bit form, which spans both histograms, after
            // the previous tile's read-out
            const bool h = staged < 65536;
            if (!h) __syncthreads();
            set_form(h ? kFormHalves : kForm32, tseq, 0);
        }
        // halves = 2: from 2^16 entries on, two passes of half the lanes
        const int npass = hs && staged >= 65536 ? 2 : 1;
        const bool any = staged != 0;
        if (Mw > wcap && lane == 0) sh.spill[tseq & 1] = 1;
        for (int pass = 0; pass < npass; ++pass) {
            if (hs) set_form(npass == 2 ? kFormHalfLanes : kFormHalves, tseq, pass);

            // 2. vote this wave's entries, chunk by chunk (the first is staged;
            // a second pass stages it again when later chunks replaced it)
            for (int32_t c0 = 0; c0 < Mw; c0 += wcap) {
                if (c0 > 0 || (pass > 0 && Mw > wcap)) stage_chunk(ox, c0);
#pragma unroll
                for (int k = 0; k < ER; ++k) {
                    const int e = wave + k * NW;
                    if (e >= E) break;
                    const int32_t n = __builtin_amdgcn_readlane(my_n, k);
                    if (n == 0) continue;
                    const int32_t b = __builtin_amdgcn_readlane(my_b, k);
                    vote_run<MODE, G>(wst + b, n, vote_addr(Sx[k], Sy[PK ? 0 : k]),
                                      MODE == kMask32 ? (1u << e) : cval, g);
                }
                for (int k = ER; wave + k * NW < E; ++k) {
                    const int e = wave + k * NW;
                    const int32_t n = __builtin_amdgcn_readlane(my_n, k);
                    if (n == 0) continue;
                    const int32_t b = __builtin_amdgcn_readlane(my_b, k);
                    const int32_t d = __builtin_amdgcn_readlane(my_d, k);
                    const int32_t sx = shift_q8(my_vx, d) + (int32_t)ox_lane;
                    const int32_t sy = shift_q8(my_vy, d) + (int32_t)oy_lane;
                    const int32_t sxv = PK   ? (int32_t)pack16(sx, sy)
                                        : WT ? (int32_t)((uint32_t)sx << 8)
                                             : sx;
                    vote_run<MODE, G>(wst + b, n, vote_addr(sxv, sy),
                                      MODE == kMask32 ? (1u << e) : cval, g);
                }
                __builtin_amdgcn_wave_barrier();  // the stage is read before it is refilled
            }
            const bool last = pass == npass - 1;
            // the next tile's runs and first chunk, while other waves still vote
            if (last && next) {
                runs();
                if (Mw > 0) {
                    stage_chunk(oxn, 0);
                    if (lane == 0) atomicAdd(&sh.voted[(tseq + 1) & 3], Mw);
                }
            }
            __syncthreads();  // every vote of this tile (pass) is in the histogram
            // The total of tile t is summed before the barrier that ends tile t - 1
            // (the first tile of an item: after the item's setup barriers) and read
            // after the one that ends tile t; slot t + 3 (last read after the
            // barrier ending tile t - 1, next summed after the one ending tile
            // t + 1) is cleared here.  With one barrier per tile (16-bit counts in
            // two histograms) this tile's read-out overlaps other waves' votes of
            // tile t + 1 and the summing of tile t + 2, which use the other slots.
            if (last) {
                staged = sh.voted[(tseq + 1) & 3];  // the next tile's, complete at this barrier
                if (tid == 0) {
                    sh.voted[(tseq + 3) & 3] = 0;
                    // a spill flag is set before the barrier ending its tile and
                    // cleared here, before the barrier ending the next one (after
                    // which the flag's next tile sets it)
                    if (sh.spill[tseq & 1]) {
                        ++sh.n_spill;
                        sh.spill[tseq & 1] = 0;
                    }
                }
            }

            // 3. read and clear the histogram; emit or queue interior cells
            if (any) {
                __builtin_amdgcn_s_setprio(1);
                // words of this tile's histogram, and its first word
                const int rw = form == kForm32 ? hist_words : hist_words / 2;
                uint4 *hb = smem4 + (form == kFormHalves && hv ? (tseq & 1) * (hist_words / 8) : 0);
                // count cnt of lane jj's velocity in bin `bin` (all lanes call)
                const auto emit = [&](uint32_t cnt, int jj,
                                      int bin) __attribute__((always_inline)) {
                    bool ok = false;
                    uint32_t v = 0;
                    int32_t bx = 0, by = 0;
                    if (cnt >= nmin) {
                        const int iy = bin / a.hx, ix = bin - iy * a.hx;
                        const int cx = ix - (sh.sg[jj] & 0xffff), cy = iy - (sh.sg[jj] >> 16);
                        ok = sh.sv[jj] >= 0 && cx >= 0 && cx < a.tile_x && cy >= 0 && cy < a.tile_y;
                        v = (uint32_t)sh.sv[jj];
                        bx = tx0 + cx;
                        by = ty0 + cy;
                    }
                    if (refined_mode<MODE>()) {
                        const int64_t idx = wave_append(ok, a.refine_count);
                        if (ok && idx < a.refine_cap)
                            store_g(a.refine + idx, v, (uint32_t)bx, (uint32_t)by, 0u);
                    } else {
                        const int64_t idx = wave_append(ok, (unsigned long long *)&a.res->n_cand);
                        if (ok && idx < a.cand_cap)
                            write_cand(a.cand, idx, v, bx, by, cnt, (uint32_t)a.count_sat);
                    }
                };
                for (int w0 = 0; w0 < rw / 4; w0 += T) {
                    const int w4 = w0 + tid;
                    uint4 h = make_uint4(0, 0, 0, 0);
                    if (w4 < rw / 4) {
                        h = hb[w4];
                        hb[w4] = make_uint4(0, 0, 0, 0);
                    }
                    const uint32_t hw[4] = {h.x, h.y, h.z, h.w};
                    if (form == kFormHalves) {  // word wi: bin wi / (NV / 2), velocity lanes
                                                // wi % (NV / 2) (low half) and that + NV / 2
                        uint32_t m = 0;
#pragma unroll
                        for (int k = 0; k < 4; ++k) m = max(m, max(hw[k] & 0xffffu, hw[k] >> 16));
                        if (!__any(m >= nmin)) continue;  // wave uniform
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int wi = 4 * w4 + k;
                            emit(hw[k] & 0xffffu, wi & (NV / 2 - 1), wi >> (LNV - 1));
                            emit(hw[k] >> 16, (wi & (NV / 2 - 1)) + NV / 2, wi >> (LNV - 1));
                        }
                    } else if (form == kFormHalfLanes) {  // word wi: bin wi / (NV / 2), velocity
                                                          // lane wi % (NV / 2) + the pass's half
                        const uint32_t m = max(max(h.x, h.y), max(h.z, h.w));
                        if (!__any(m >= nmin)) continue;  // wave uniform
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int wi = 4 * w4 + k;
                            emit(hw[k], (wi & (NV / 2 - 1)) + fpass * (NV / 2), wi >> (LNV - 1));
                        }
                    } else {
                        const uint32_t m = max(max(cell_count<MODE>(h.x), cell_count<MODE>(h.y)),
                                               max(cell_count<MODE>(h.z), cell_count<MODE>(h.w)));
                        if (!__any(m >= nmin)) continue;  // wave uniform
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int wi = 4 * w4 + k;
                            emit(cell_count<MODE>(hw[k]), wi & (NV - 1), wi >> LNV);
                        }
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
            // the histogram is clear before the next tile's (pass's) votes; after
            // a 16-bit tile of two histograms the next one votes into the other
            // histogram, cleared before this tile's barrier
            if (!(hv && form == kFormHalves)) __syncthreads();
        }  // passes
#pragma unroll
        for (int k = 0; k < ER; ++k) {
            if constexpr (PK) {  // low half only, modulo 2^16
                const us2 step = {(unsigned short)(a.tile_x << kc), 0};
                Sx[k] = (int32_t)__builtin_bit_cast(uint32_t, __builtin_bit_cast(us2, Sx[k]) + step);
            } else {
                Sx[k] = (int32_t)((uint32_t)Sx[k] + ((uint32_t)(a.tile_x * cellw) << (WT ? 8 : 0)));
            }
        }
    }
}

// Dynamic LDS: histogram [HY][HX][NV] words, then the stage (int2, or one
// packed word per detection), one part of stage_cap / NW detections per wave.
template <int MODE, int G, bool PK>
__global__ void __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<G, PK>))) k_vote_dense(DenseArgs a) {
    extern __shared__ uint4 smem4[];
    __shared__ Shared sh;
    const int tid = threadIdx.x;
    const int hist_words = a.hx * a.hy * (64 / G) / (a.halves == 2 ? 2 : 1);  // as allocated
    for (int i = tid; i < hist_words / 4; i += T) smem4[i] = make_uint4(0, 0, 0, 0);
    if (tid < a.cat.n_epochs) sh.dt[tid] = a.cat.dt[tid];
    int32_t tseq = 0;  // tiles done by this workgroup (flag ring of sh.voted)
    if (tid < 4) sh.voted[tid] = 0;
    sh.heads[tid >> 6][tid & 63] = 0;  // each wave's own row, clear between blocks
    if (tid == 0) {
        sh.count_on = a.atomics != nullptr;
        sh.n_instr = 0;
        sh.spill[0] = sh.spill[1] = 0;
        sh.n_spill = 0;
    }
    // The items past n_items_kept hold tiles that fewer than N_min epochs
    // reach when the reference epoch is the earliest scheduled one; they are
    // voted only when that epoch holds no detection (then t0 is later).
    const int64_t n_walk = a.cat.dt[a.e_first] == 0 ? a.n_items_kept : a.n_items;
    // Persistent workgroups (as many as are resident) take items from queues:
    // XCD x's range is [x n / 8, (x + 1) n / 8) of the L2-friendly item order
    // and workgroups are dispatched round-robin over the XCDs (each with its
    // own L2), so a workgroup first takes its own XCD's items, one atomic
    // ticket each, then helps with the other ranges in turn.  Every ticket
    // below a range's size is one item, taken once; every workgroup ends after
    // one ticket past the end of each range.
    const int x0 = blockIdx.x % kXcds;
    for (int k = 0; k < kXcds; ++k) {
        const int x = (x0 + k) % kXcds;
        const int64_t lo = x * n_walk / kXcds, n_x = (x + 1) * n_walk / kXcds - lo;
        for (;;) {
            __syncthreads();  // every thread has read the previous ticket
            if (tid == 0) sh.ticket = atomicAdd(&a.item_queue[x], 1ull);
            __syncthreads();
            const int64_t t = (int64_t)sh.ticket;  // block uniform
            if (t >= n_x) break;
            const int32_t *it = a.items + 4 * (lo + t);
            vote_item<MODE, G, PK>(a, sh, smem4, it[0], it[1], it[2], it[3], tseq);
        }
    }
    __syncthreads();
    if (tid == 0 && sh.count_on && sh.n_instr) atomicAdd(a.atomics, sh.n_instr);
    // one add per workgroup: the count of every chunked tile to one global
    // word would serialise at that word's L2 channel
    if (tid == 0 && sh.n_spill) atomicAdd(&a.res->n_spilled, sh.n_spill);
}

// Many catalogs in one persistent launch (one workgroup per resident slot):
// the merged items (items5: chip, segment, ty0, txf, ntiles; chip-major, each
// chip in its own L2-friendly order) are taken from per-XCD queues like the
// single-catalog kernel takes its items (so an XCD's range holds few chips),
// and each item reads its chip's parameters from
// chips[].  Every chip of the launch uses this kernel's cell variant and lane
// groups (and vote form); hist_words_max covers the largest histogram among
// them.  Items [0, n_kept) are every chip's kept items; the rest hold tiles
// that fewer than N_min epochs reach (see k_vote_dense), with the chip stored
// as ~chip, voted only for the chips whose earliest scheduled epoch holds no
// detection.
template <int MODE, int G, bool PK>
__global__ void __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<G, PK>))) k_vote_dense_batch(const DenseArgs *__restrict__ chips,
                                                         int32_t n_chips,
                                                         const int32_t *__restrict__ items5,
                                                         int64_t n_items, int64_t n_kept,
                                                         int32_t hist_words_max,
                                                         unsigned long long *queue,
                                                         unsigned long long *atomics) {
    extern __shared__ uint4 smem4[];
    __shared__ Shared sh;
    const int tid = threadIdx.x;
    for (int i = tid; i < hist_words_max / 4; i += T) smem4[i] = make_uint4(0, 0, 0, 0);
    int32_t tseq = 0, chip_now = -1;  // tseq: tiles done by this workgroup
    if (tid < 4) sh.voted[tid] = 0;
    sh.heads[tid >> 6][tid & 63] = 0;  // each wave's own row, clear between blocks
    if (tid == 0) {
        sh.count_on = atomics != nullptr;
        sh.n_instr = 0;
        sh.spill[0] = sh.spill[1] = 0;
        sh.n_spill = 0;
    }
    int later_t0 = 0;  // some chip's reference epoch is later than its earliest epoch
    for (int c = tid; c < n_chips; c += T)
        later_t0 |= gmem(chips[c].cat.dt)[chips[c].e_first] != 0;
    later_t0 = __syncthreads_or(later_t0);
    const int64_t n_walk = later_t0 ? n_items : n_kept;
    const int x0 = blockIdx.x % kXcds;
    for (int k = 0; k < kXcds; ++k) {
      const int x = (x0 + k) % kXcds;
      const int64_t lo = x * n_walk / kXcds, n_x = (x + 1) * n_walk / kXcds - lo;
      for (;;) {
        __syncthreads();  // every thread has read the previous ticket
        if (tid == 0) sh.ticket = atomicAdd(&queue[x], 1ull);
        __syncthreads();
        const int64_t t = (int64_t)sh.ticket;  // block uniform
        if (t >= n_x) break;
        const int32_t *it = items5 + 5 * (lo + t);
        int chip = it[0];
        if (chip < 0) {  // skipped tiles of chip ~chip: block uniform
            chip = ~chip;
            if (gmem(chips[chip].cat.dt)[chips[chip].e_first] == 0) continue;
        }
        const DenseArgs &a = chips[chip];
        if (chip != chip_now) {
            __syncthreads();  // the previous item no longer reads sh.dt or the stage
            if (tid == 0 && sh.n_spill) {  // the previous chip's chunked tiles
                __hip_atomic_fetch_add(gmem(&chips[chip_now].res->n_spilled), sh.n_spill,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh.n_spill = 0;
            }
            if (tid < a.cat.n_epochs) sh.dt[tid] = gmem(a.cat.dt)[tid];
            // this chip's histogram may cover what was the previous chip's stage
            const int hw = a.hx * a.hy * (64 / G) / (a.halves == 2 ? 2 : 1);
            for (int i = tid; i < hw / 4; i += T) smem4[i] = make_uint4(0, 0, 0, 0);
            chip_now = chip;
        }
        vote_item<MODE, G, PK>(a, sh, smem4, it[1], it[2], it[3], it[4], tseq);
      }
    }
    __syncthreads();
    if (tid == 0 && sh.count_on && sh.n_instr) atomicAdd(atomics, sh.n_instr);
    if (tid == 0 && sh.n_spill)
        __hip_atomic_fetch_add(gmem(&chips[chip_now].res->n_spilled), sh.n_spill, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Exact bins of a queued cell: for velocity v and the cell's 2^m x 2^m
// bins, gather the detections that project into it (window index, one
// epoch per lane), count distinct epochs (or detections) per bin, emit the
// bins at or above N_min.  One wave per queued cell.
// WM: kRefineCount (the indicator counts of mode_epochs), kRefineWeightDet
// (sum of the weights) or kRefineWeightEpochs (per epoch the largest
// weight, summed: each lane keeps its epoch's maxima in a private column of
// LDS and adds them to the bins when the epoch is done).
constexpr int kRefineBins = 64;  // up to 8 x 8 bins per cell
enum RefineMode : int { kRefineCount = 0, kRefineWeightDet = 1, kRefineWeightEpochs = 2 };

template <int WM>
__global__ void __launch_bounds__(T) k_refine(DenseArgs a) {
    __shared__ uint32_t masks[NW][kRefineBins * kSlotWords];
    __shared__ uint8_t best[WM == kRefineWeightEpochs ? NW : 1][kRefineBins][64];
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
    for (int64_t qi = (int64_t)blockIdx.x * NW + wave; qi < n_q; qi += (int64_t)gridDim.x * NW) {
        const int4 q = a.refine[qi];
        const int32_t v = q.x;
        const int32_t vx = a.vel[2 * (int64_t)v], vy = a.vel[2 * (int64_t)v + 1];
        const int32_t fbx0 = q.y * cw, fby0 = q.z * cw;  // first bin of the cell
        for (int i = lane; i < kRefineBins * kSlotWords; i += 64) mk[i] = 0;
        if (WM == kRefineWeightEpochs)
            for (int i = 0; i < kRefineBins; ++i) best[wave][i][lane] = 0;
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
            uint64_t touched = 0;  // kRefineWeightEpochs: bins this lane's epoch reached
            for (int cy = cy0; cy <= cy1; ++cy) {
                const int64_t base = ((int64_t)e * c.ncy + cy) * c.ncx;
                const int32_t j1 = c.off[base + cx1 + 1];
                // kCopyAhead detections loaded at a time, then binned
                for (int32_t j0 = c.off[base + cx0]; j0 < j1; j0 += kCopyAhead) {
                    int2 pq[kCopyAhead];
#pragma unroll
                    for (int u = 0; u < kCopyAhead; ++u)
                        if (j0 + u < j1) pq[u] = c.sxy[j0 + u];
#pragma unroll
                    for (int u = 0; u < kCopyAhead; ++u) {
                        if (j0 + u >= j1) break;
                        const int2 p = pq[u];
                        // weighted plans: the index holds 256 x + w
                        const int32_t px = WM == kRefineCount ? p.x : p.x >> 8;
                        const uint32_t wt = (uint32_t)p.x & 0xffu;
                        const int32_t bx = ((px - sx) >> k) - fbx0, by = ((p.y - sy) >> k) - fby0;
                        if ((uint32_t)bx < (uint32_t)cw && (uint32_t)by < (uint32_t)cw) {
                            const int bin = by * cw + bx;
                            if (WM == kRefineWeightDet) {
                                atomicAdd(&mk[bin * kSlotWords], wt);
                            } else if (WM == kRefineWeightEpochs) {
                                if (wt > best[wave][bin][lane]) best[wave][bin][lane] = (uint8_t)wt;
                                touched |= (uint64_t)1 << bin;
                            } else if (a.mode_epochs) {
                                atomicOr(&mk[bin * kSlotWords + (e >> 5)], 1u << (e & 31));
                            } else {
                                atomicAdd(&mk[bin * kSlotWords], 1u);
                            }
                        }
                    }
                }
            }
            // kRefineWeightEpochs: the epoch is done; add its largest weights
            while (WM == kRefineWeightEpochs && touched) {
                const int bin = __builtin_ctzll(touched);
                touched &= touched - 1;
                atomicAdd(&mk[bin * kSlotWords], (uint32_t)best[wave][bin][lane]);
                best[wave][bin][lane] = 0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        uint32_t cnt = 0;
        if (lane < nb) {
            if (WM == kRefineCount && a.mode_epochs) {
                for (int w = 0; w < kSlotWords; ++w) cnt += __popc(mk[lane * kSlotWords + w]);
            } else {
                cnt = mk[lane * kSlotWords];
            }
        }
        const bool ok = lane < nb && cnt >= (uint32_t)a.n_min;
        const int64_t idx = wave_append(ok, (unsigned long long *)&a.res->n_cand);
        if (ok && idx < a.cand_cap)
            write_cand(a.cand, idx, (uint32_t)v, fbx0 + (lane % cw), fby0 + (lane / cw), cnt,
                       (uint32_t)a.count_sat);
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t set_lds_limit(const void *fn, size_t lds, size_t *lds_set) {
    if (lds > 65536 && lds > *lds_set) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        *lds_set = lds;
    }
    return hipSuccess;
}

// Persistent vote launches: the workgroups resident at once (LDS and waves
// per SIMD), at most one per kept item (those walked unless the reference
// epoch is a later one); the item queues balance the work.
template <int G, bool PK>
int64_t resident_grid(size_t lds, int64_t kept) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n_cu <= 0)
        n_cu = 256;  // MI355X
    const int64_t per_cu = std::max<int64_t>(
        1, std::min<int64_t>(kLdsPerCU / (int64_t)(lds + sizeof(Shared)),
                             kWavesPerSimd<G, PK> * 4 / NW));
    return std::min<int64_t>(std::max<int64_t>(kept, 1), (int64_t)n_cu * per_cu);
}

template <int MODE, int G, bool PK>
hipError_t launch_mg(const DenseArgs &a, size_t lds, hipStream_t stream, hipEvent_t ev0,
                     hipEvent_t ev1) {
    static size_t lds_set = 0;  // dynamic LDS limit raised so far for this kernel
    hipError_t e = set_lds_limit((const void *)k_vote_dense<MODE, G, PK>, lds, &lds_set);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)resident_grid<G, PK>(lds, a.n_items_kept)), block(T);
    if (ev0 && (e = hipEventRecord(ev0, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_vote_dense<MODE, G, PK>), grid, block, lds, stream, a);
    if (ev1 && (e = hipEventRecord(ev1, stream)) != hipSuccess) return e;
    if (refined_mode<MODE>()) return launch_refine(a, stream);
    return hipGetLastError();
}

template <int MODE, bool PK>
hipError_t launch_m(int groups, const DenseArgs &a, size_t lds, hipStream_t s, hipEvent_t e0,
                    hipEvent_t e1) {
    switch (groups) {
    case 1: return launch_mg<MODE, 1, PK>(a, lds, s, e0, e1);
    case 2: return launch_mg<MODE, 2, PK>(a, lds, s, e0, e1);
    default: return launch_mg<MODE, 4, PK>(a, lds, s, e0, e1);
    }
}

struct BatchLaunch {
    const DenseArgs *chips;
    int32_t n_chips;
    const int32_t *items5;
    int64_t n_items, n_kept;
    int32_t hist_words_max;
    size_t lds;
    unsigned long long *queue;
    unsigned long long *atomics;
};

__global__ void k_zero_queue(unsigned long long *queue) {
    if (threadIdx.x < kXcds) queue[threadIdx.x] = 0;
}

template <int MODE, int G, bool PK>
hipError_t launch_batch_mg(const BatchLaunch &b, hipStream_t stream) {
    static size_t lds_set = 0;
    hipError_t e = set_lds_limit((const void *)k_vote_dense_batch<MODE, G, PK>, b.lds, &lds_set);
    if (e != hipSuccess) return e;
    // a fill kernel, not a memset: the launch may be captured in a graph
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, stream, b.queue);
    const int64_t grid = resident_grid<G, PK>(b.lds, b.n_kept);
    hipLaunchKernelGGL((k_vote_dense_batch<MODE, G, PK>), dim3((unsigned)grid), dim3(T), b.lds,
                       stream, b.chips, b.n_chips, b.items5, b.n_items, b.n_kept,
                       b.hist_words_max, b.queue, b.atomics);
    return hipGetLastError();
}

template <int MODE, bool PK>
hipError_t launch_batch_m(int groups, const BatchLaunch &b, hipStream_t s) {
    switch (groups) {
    case 1: return launch_batch_mg<MODE, 1, PK>(b, s);
    case 2: return launch_batch_mg<MODE, 2, PK>(b, s);
    default: return launch_batch_mg<MODE, 4, PK>(b, s);
    }
}

template <bool PK>
hipError_t launch_batch_p(int mode, int groups, const BatchLaunch &b, hipStream_t s) {
    switch (mode) {
    case kMask32: return launch_batch_m<kMask32, PK>(groups, b, s);
    case kCountDet: return launch_batch_m<kCountDet, PK>(groups, b, s);
    default: return launch_batch_m<kCountRef, PK>(groups, b, s);
    }
}

template <bool PK>
hipError_t launch_p(int mode, int groups, const DenseArgs &a, size_t lds, hipStream_t s,
                    hipEvent_t e0, hipEvent_t e1) {
    switch (mode) {
    case kMask32: return launch_m<kMask32, PK>(groups, a, lds, s, e0, e1);
    case kCountDet: return launch_m<kCountDet, PK>(groups, a, lds, s, e0, e1);
    default: return launch_m<kCountRef, PK>(groups, a, lds, s, e0, e1);
    }
}

// Weighted variants: 32-bit votes only.
hipError_t launch_w(int mode, int groups, const DenseArgs &a, size_t lds, hipStream_t s,
                    hipEvent_t e0, hipEvent_t e1) {
    if (mode == kWeightDet) return launch_m<kWeightDet, false>(groups, a, lds, s, e0, e1);
    return launch_m<kWeightRef, false>(groups, a, lds, s, e0, e1);
}

}  // namespace

size_t dense_lds_bytes(int groups, int hx, int hy, int stage_cap, int packed, int halves) {
    // histogram: 32-bit words, or 16-bit counts in one histogram (halves = 2)
    size_t b = (size_t)hx * hy * (64 / groups) * (halves == 2 ? 2 : sizeof(uint32_t));
    b += (size_t)stage_cap * (packed ? sizeof(uint32_t) : sizeof(int2));  // stage (NW parts)
    return (b + 15) & ~(size_t)15;
}

size_t dense_static_lds_bytes() { return sizeof(Shared); }

hipError_t launch_vote_dense_batch(int mode, int groups, int packed, const DenseArgs *chips_dev,
                                   int32_t n_chips, const int32_t *items5_dev, int64_t n_items,
                                   int64_t n_kept, int32_t hist_words_max, size_t lds,
                                   unsigned long long *queue, unsigned long long *atomics,
                                   hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
    const BatchLaunch b{chips_dev, n_chips, items5_dev, n_items, n_kept, hist_words_max, lds,
                        queue, atomics};
    return packed ? launch_batch_p<true>(mode, groups, b, stream)
                  : launch_batch_p<false>(mode, groups, b, stream);
}

hipError_t launch_refine(const DenseArgs &a, hipStream_t stream) {
    if (a.weighted == SAS_MODE_WEIGHTED_EPOCHS)
        hipLaunchKernelGGL(k_refine<kRefineWeightEpochs>, dim3(kRefineGrid), dim3(T), 0, stream,
                           a);
    else if (a.weighted == SAS_MODE_WEIGHTED_DETECTIONS)
        hipLaunchKernelGGL(k_refine<kRefineWeightDet>, dim3(kRefineGrid), dim3(T), 0, stream, a);
    else
        hipLaunchKernelGGL(k_refine<kRefineCount>, dim3(kRefineGrid), dim3(T), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_vote_dense(int mode, int groups, const DenseArgs &a, hipStream_t stream,
                             hipEvent_t ev0, hipEvent_t ev1) {
    if (a.n_items <= 0) return hipSuccess;
    const size_t lds = dense_lds_bytes(groups, a.hx, a.hy, a.stage_cap, a.packed, a.halves);
    if (mode == kWeightDet || mode == kWeightRef) {
        if (a.packed) return hipErrorInvalidValue;  // excluded by the planner
        return launch_w(mode, groups, a, lds, stream, ev0, ev1);
    }
    return a.packed ? launch_p<true>(mode, groups, a, lds, stream, ev0, ev1)
                    : launch_p<false>(mode, groups, a, lds, stream, ev0, ev1);
}

}  // namespace sas

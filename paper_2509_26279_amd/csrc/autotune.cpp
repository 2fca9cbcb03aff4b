// Launch-shape autotuner of the dense vote (host side).
//
// For one catalog the tuner builds a plan per candidate tuning, votes the
// catalog once and collects its candidate list in canonical order, then
// times `reps` more votes with events around the vote kernel (the plan's
// probe) and keeps the median.  Every candidate whose plan fits must give
// the candidate list of the first one that fits: a launch shape may change
// the time of a vote, never its result.  Choices are kept per shape class
// in a text cache, one class per line: "<key> name=value ...".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace sas {
void set_error(const std::string &msg);
}

namespace {

sas_status afail(sas_status s, const std::string &m) {
    sas::set_error(m);
    return s;
}

struct Field {
    const char *name;
    int32_t sas_tuning::*member;
};

const Field kFields[] = {
    {"tile_x", &sas_tuning::tile_x},         {"tile_y", &sas_tuning::tile_y},
    {"vblock_x", &sas_tuning::vblock_x},     {"vblock_y", &sas_tuning::vblock_y},
    {"groups", &sas_tuning::groups},         {"stage_cap", &sas_tuning::stage_cap},
    {"cell_log2", &sas_tuning::cell_log2},   {"sort_vblock", &sas_tuning::sort_vblock},
    {"n_det_hint", &sas_tuning::n_det_hint}, {"coarse_log2", &sas_tuning::coarse_log2},
    {"refine_cap", &sas_tuning::refine_cap}, {"packed", &sas_tuning::packed},
    {"weight_hint", &sas_tuning::weight_hint}, {"half_counts", &sas_tuning::half_counts},
    {"prune", &sas_tuning::prune},
};

std::string tuning_text(const sas_tuning &t) {
    std::ostringstream o;
    bool first = true;
    for (const Field &f : kFields) {
        if (t.*(f.member) == 0) continue;
        o << (first ? "" : " ") << f.name << "=" << t.*(f.member);
        first = false;
    }
    return o.str();
}

// Device buffers of one timed vote.
struct Buffers {
    void *ws = nullptr, *cand = nullptr, *res = nullptr;
    size_t ws_bytes = 0;
    int64_t cand_cap = 0;
    ~Buffers() {
        if (ws) (void)hipFree(ws);
        if (cand) (void)hipFree(cand);
        if (res) (void)hipFree(res);
    }
};

// One candidate: plan, first vote and its list, then the timed votes.
sas_status trial(const sas_plan_desc &d, const sas_tuning &tu, const int32_t *x, const int32_t *y,
                 const uint8_t *e, int64_t n, int32_t reps, hipStream_t s,
                 std::vector<sas_candidate> *list, float *ms) {
    sas_plan_desc dd = d;
    dd.tuning = &tu;
    sas_plan *p = nullptr;
    sas_status st = sas_plan_create(&dd, &p);
    if (st != SAS_OK) return st;
    Buffers b;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<float> times;
    hipError_t he = hipSuccess;
    st = sas_vote_workspace_size(p, n, &b.ws_bytes);
    if (st != SAS_OK) goto done;
    b.cand_cap = (int64_t)1 << 22;
    if ((he = hipMalloc(&b.ws, std::max<size_t>(b.ws_bytes, 256))) != hipSuccess ||
        (he = hipMalloc(&b.cand, sizeof(sas_candidate) * b.cand_cap)) != hipSuccess ||
        (he = hipMalloc(&b.res, sizeof(sas_vote_result))) != hipSuccess) {
        st = afail(SAS_E_NOMEM, std::string("sas_autotune: ") + hipGetErrorString(he));
        goto done;
    }
    st = sas_vote(p, x, y, e, n, (sas_candidate *)b.cand, b.cand_cap, (sas_vote_result *)b.res,
                  b.ws, b.ws_bytes, s);
    if (st != SAS_OK) goto done;
    {
        int64_t got = 0;
        list->assign((size_t)b.cand_cap, sas_candidate{});
        st = sas_peaks((sas_candidate *)b.cand, (sas_vote_result *)b.res, b.cand_cap,
                       SAS_ORDER_CANONICAL, 0, list->data(), b.cand_cap, &got, s);
        if (st != SAS_OK) goto done;
        list->resize((size_t)got);
    }
    if ((he = hipEventCreate(&ev[0])) != hipSuccess || (he = hipEventCreate(&ev[1])) != hipSuccess) {
        st = afail(SAS_E_DEVICE, std::string("sas_autotune: events: ") + hipGetErrorString(he));
        goto done;
    }
    sas_plan_set_probe(p, ev[0], ev[1]);
    for (int r = 0; r < reps; ++r) {
        st = sas_vote(p, x, y, e, n, (sas_candidate *)b.cand, b.cand_cap,
                      (sas_vote_result *)b.res, b.ws, b.ws_bytes, s);
        if (st != SAS_OK) goto done;
        float t = 0.f;
        if ((he = hipEventSynchronize(ev[1])) != hipSuccess ||
            (he = hipEventElapsedTime(&t, ev[0], ev[1])) != hipSuccess) {
            st = afail(SAS_E_DEVICE, std::string("sas_autotune: timing: ") + hipGetErrorString(he));
            goto done;
        }
        times.push_back(t);
    }
    std::sort(times.begin(), times.end());
    *ms = times.empty() ? 0.f : times[times.size() / 2];
done:
    if (p) {
        sas_plan_set_probe(p, nullptr, nullptr);
        sas_plan_destroy(p);
    }
    for (hipEvent_t v : ev)
        if (v) (void)hipEventDestroy(v);
    return st;
}

// Launch shapes around the planner's own choice for each lane-group count.
std::vector<sas_tuning> default_candidates(const sas_tuning &base, int32_t planner_cell_log2) {
    std::vector<sas_tuning> out;
    out.push_back(base);
    for (int g : {1, 2, 4}) {
        sas_tuning t = base;
        t.groups = g;
        out.push_back(t);
        for (int step : {-1, 1}) {  // window-index cells one step finer or coarser
            sas_tuning c = t;
            c.cell_log2 = planner_cell_log2 + step;
            if (c.cell_log2 > 0) out.push_back(c);
        }
        const int shapes[5][2] = {{8, 8}, {12, 10}, {16, 12}, {24, 16}, {16, 24}};
        for (const auto &sh : shapes) {
            sas_tuning c = t;
            c.tile_x = sh[0];
            c.tile_y = sh[1];
            out.push_back(c);
        }
    }
    return out;
}

}  // namespace

extern "C" {

sas_status sas_autotune_default_candidates(const sas_plan_desc *desc, sas_tuning *out,
                                           int32_t cap, int32_t *n_out) {
    if (!desc || !n_out || cap < 0 || (cap > 0 && !out))
        return afail(SAS_E_INVALID, "sas_autotune_default_candidates: bad argument");
    sas_tuning base{};
    if (desc->tuning) base = *desc->tuning;
    sas_plan *p = nullptr;
    sas_status st = sas_plan_create(desc, &p);
    if (st != SAS_OK) return st;
    sas_plan_info info{};
    sas_plan_get_info(p, &info);
    sas_plan_destroy(p);
    const std::vector<sas_tuning> c = default_candidates(base, info.cell_log2);
    *n_out = (int32_t)c.size();
    if ((int32_t)c.size() > cap)
        return afail(SAS_E_OVERFLOW, "sas_autotune_default_candidates: cap too small");
    std::copy(c.begin(), c.end(), out);
    return SAS_OK;
}

sas_status sas_autotune(const sas_plan_desc *desc, const int32_t *x_q8, const int32_t *y_q8,
                        const uint8_t *epoch, int64_t n, const sas_tuning *cands, int32_t n_cands,
                        int32_t reps, sas_autotune_trial *trials_out, sas_tuning *best_out,
                        void *stream) {
    if (!desc || !cands || n_cands < 1 || reps < 1 || !best_out || !trials_out)
        return afail(SAS_E_INVALID, "sas_autotune: bad argument");
    if (desc->path == SAS_PATH_SORT)
        return afail(SAS_E_UNSUPPORTED, "sas_autotune: tunes the dense path");
    if (desc->mode == SAS_MODE_WEIGHTED_EPOCHS || desc->mode == SAS_MODE_WEIGHTED_DETECTIONS)
        return afail(SAS_E_UNSUPPORTED, "sas_autotune: weighted plans are not tuned");
    hipStream_t s = (hipStream_t)stream;
    std::vector<sas_candidate> ref, list;
    bool have_ref = false;
    int best = -1;
    for (int32_t k = 0; k < n_cands; ++k) {
        sas_autotune_trial &tr = trials_out[k];
        tr.tuning = cands[k];
        tr.ms = -1.f;
        float ms = 0.f;
        const sas_status st = trial(*desc, cands[k], x_q8, y_q8, epoch, n, reps, s, &list, &ms);
        tr.status = st;
        if (st == SAS_E_INVALID || st == SAS_E_UNSUPPORTED) continue;  // shape does not fit
        if (st != SAS_OK) return st;
        if (!have_ref) {
            ref.swap(list);
            have_ref = true;
        } else if (list.size() != ref.size() ||
                   (!list.empty() &&
                    std::memcmp(list.data(), ref.data(), sizeof(sas_candidate) * list.size()))) {
            return afail(SAS_E_DEVICE, "sas_autotune: launch shape {" + tuning_text(cands[k]) +
                                           "} changed the candidate list (a library bug)");
        }
        tr.ms = ms;
        if (best < 0 || ms < trials_out[best].ms) best = k;
    }
    if (best < 0) return afail(SAS_E_INVALID, "sas_autotune: no candidate launch shape fits");
    *best_out = cands[best];
    return SAS_OK;
}

sas_status sas_autotune_key(const sas_plan_desc *desc, int64_t n, char *key_out, int64_t cap) {
    if (!desc || !key_out || cap < 1 || n < 0 || desc->n_epochs < 1 || !desc->t_q16)
        return afail(SAS_E_INVALID, "sas_autotune_key: bad argument");
    int64_t tmin = desc->t_q16[0], tmax = desc->t_q16[0];
    for (int e = 1; e < desc->n_epochs; ++e) {
        tmin = std::min(tmin, desc->t_q16[e]);
        tmax = std::max(tmax, desc->t_q16[e]);
    }
    const int64_t span = std::max<int64_t>(tmax - tmin, 1);
    const int64_t spacing = std::max<int64_t>(1, ((int64_t)desc->binw_q8 * 65536) / span);
    auto pow2_floor = [](int64_t v) {
        int64_t p = 1;
        while (p * 2 <= v) p *= 2;
        return p;
    };
    char buf[160];
    std::snprintf(buf, sizeof(buf), "b%d_s%lld_E%lld_n%lld_V%lld_m%d", desc->binw_q8,
                  (long long)spacing, (long long)pow2_floor(desc->n_epochs),
                  (long long)pow2_floor(std::max<int64_t>(n, 1)),
                  (long long)pow2_floor(std::max<int64_t>(desc->n_v, 1)), desc->mode);
    if ((int64_t)std::strlen(buf) + 1 > cap)
        return afail(SAS_E_OVERFLOW, "sas_autotune_key: cap too small");
    std::memcpy(key_out, buf, std::strlen(buf) + 1);
    return SAS_OK;
}

sas_status sas_autotune_cache_get(const char *path, const char *key, sas_tuning *out,
                                  int32_t *found) {
    if (!path || !key || !out || !found) return afail(SAS_E_INVALID, "sas_autotune_cache_get: null");
    *found = 0;
    std::ifstream f(path);
    if (!f) return SAS_OK;  // no cache yet
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        if (!(is >> k) || k != key) continue;
        sas_tuning t{};
        std::string kv;
        while (is >> kv) {
            const size_t eq = kv.find('=');
            if (eq == std::string::npos)
                return afail(SAS_E_INVALID, "sas_autotune_cache_get: bad entry '" + kv + "'");
            const std::string name = kv.substr(0, eq);
            bool ok = false;
            for (const Field &fd : kFields)
                if (name == fd.name) {
                    t.*(fd.member) = (int32_t)std::strtol(kv.c_str() + eq + 1, nullptr, 10);
                    ok = true;
                }
            if (!ok) return afail(SAS_E_INVALID, "sas_autotune_cache_get: unknown field " + name);
        }
        *out = t;
        *found = 1;  // the last line of a key wins
    }
    return SAS_OK;
}

sas_status sas_autotune_cache_put(const char *path, const char *key, const sas_tuning *t) {
    if (!path || !key || !t || !*key || std::strchr(key, ' ') || std::strchr(key, '\n'))
        return afail(SAS_E_INVALID, "sas_autotune_cache_put: bad argument");
    std::vector<std::string> lines;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            std::istringstream is(line);
            std::string k;
            if ((is >> k) && k == key) continue;  // replaced below
            if (!line.empty()) lines.push_back(line);
        }
    }
    lines.push_back(std::string(key) + (tuning_text(*t).empty() ? "" : " ") + tuning_text(*t));
    std::sort(lines.begin(), lines.end());
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        if (!o) return afail(SAS_E_INVALID, "sas_autotune_cache_put: cannot write " + tmp);
        for (const std::string &l : lines) o << l << "\n";
        if (!o) return afail(SAS_E_INVALID, "sas_autotune_cache_put: write failed");
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return afail(SAS_E_INVALID, "sas_autotune_cache_put: cannot replace " + std::string(path));
    return SAS_OK;
}

}  // extern "C"

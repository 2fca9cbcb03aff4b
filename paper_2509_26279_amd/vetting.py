"""Learned vetting of vote candidates.

The vote reports every (velocity, bin) at or above a threshold.  Vetting
scores those candidates with a small network trained on candidates the vote
itself produces from seeded injections, so that a lower threshold can be
used with fewer false candidates:

  * pool: the candidates of a vote at a lowered threshold N_pool, with
    their 32 features (sas_features);
  * labels: a candidate is positive when its track (bin centre moved with
    its trial velocity) stays within one bin width of an injected mover in
    at least half of the epochs;
  * training: an ensemble of MLPs (sas_mlp_*, different seeds) on
    standardised features, binary cross-entropy with positives weighted by
    min(n_neg / n_pos, 100), AdamW; at most `cap` candidates per mover are
    kept for training, so that slow movers with hundreds of ghost stacks do
    not drown the hard ones;
  * score: the mean logit of the members;
  * operating point, on validation catalogs: the lower of (a) the largest
    threshold that keeps every findable mover the plain threshold finds
    there (so the validation recall is at least the plain threshold's,
    mover by mover) and (b) the lowest threshold whose false positives stay
    within a budget, by default a tenth of the plain threshold's.  (b) spends
    part of the gain on a margin: (a) alone is set by the single hardest
    validation mover and misses test movers just below it.

Recall counts findable movers (at least N_min epochs on the chip) with at
least one selected candidate matched to them; false positives are selected
candidates matched to no mover.

Two protocols: fast-style chips (pool at N_pool = 19, mostly mover ghosts)
and wide-style chips (pool threshold from the threshold rule of Sec. 2.2,
noise candidates dominating, about 1e6 candidates over 12 chips).
"""
from __future__ import annotations

import numpy as np

from . import sas


def match_movers(cand, v_q8, binw_q8, t_q16, t0_q16, truth, bin_px, frac=0.5):
    """Mover index matched by each candidate, or -1.

    A candidate matches mover k when |track(t_e) - mover_k(t_e)| < bin_px in
    at least frac * E epochs; the smallest such k is returned.  Both tracks
    are straight, so their distance is a convex function of time and the
    epochs within range form one run; with frac >= 1/2 that run holds one of
    the two middle epochs, which is where candidate pairs are searched
    (k-d tree) before the exact count."""
    from scipy.spatial import cKDTree
    n = len(cand)
    out = np.full(n, -1, dtype=np.int32)
    nm = len(truth["vx"])
    if n == 0 or nm == 0:
        return out
    t = np.asarray(t_q16, dtype=np.float64)
    E = t.shape[0]
    th = (t - float(t0_q16)) / 65536.0               # hours since the reference epoch
    tc = (t - t.min()) / 65536.0                      # the truth's clock
    mx = truth["x_mid"][:, None] + truth["vx"][:, None] * (tc[None, :] - truth["t_mid_h"])
    my = truth["y_mid"][:, None] + truth["vy"][:, None] * (tc[None, :] - truth["t_mid_h"])
    b = binw_q8 / 256.0
    v = np.asarray(v_q8, dtype=np.float64)[np.asarray(cand["v_idx"], dtype=np.int64)] / 256.0
    cx0 = (np.asarray(cand["bx"], dtype=np.float64) + 0.5) * b
    cy0 = (np.asarray(cand["by"], dtype=np.float64) + 0.5) * b
    need = frac * E
    mids = sorted({(E - 1) // 2, E // 2})
    pairs = set()
    for e in mids:
        tree = cKDTree(np.stack([mx[:, e], my[:, e]], axis=1))
        pts = np.stack([cx0 + v[:, 0] * th[e], cy0 + v[:, 1] * th[e]], axis=1)
        for i, ks in enumerate(tree.query_ball_point(pts, r=bin_px)):
            for k in ks:
                pairs.add((i, k))
    for i, k in sorted(pairs):
        cx = cx0[i] + v[i, 0] * th
        cy = cy0[i] + v[i, 1] * th
        close = int((np.hypot(mx[k] - cx, my[k] - cy) < bin_px).sum())
        if close >= need and (out[i] < 0 or k < out[i]):
            out[i] = k
    return out


def findable(truth, n_min):
    """Movers present (on the chip) in at least n_min epochs."""
    return np.asarray(truth["present"]).sum(axis=1) >= n_min


def recall_fp(selected, matched, findable_mask):
    """(recall over findable movers, false positives) of a selection."""
    sel = np.asarray(selected, dtype=bool)
    m = np.asarray(matched)[sel]
    found = np.unique(m[m >= 0])
    fmask = np.asarray(findable_mask, dtype=bool)
    n_find = int(fmask.sum())
    rec = float(fmask[found].sum()) / n_find if n_find else 1.0
    return rec, int((m < 0).sum())


def candidate_pool(wl, v, n_pool, tuning=None, cand_cap=1 << 23):
    """Vote at threshold n_pool; return (records, features, counts, t0)."""
    import torch
    tun = dict(tuning or {})
    tun.setdefault("n_det_hint", wl.n)
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, n_pool, wl.extent_q8, tuning=tun)
    try:
        s = sas.Search(plan, wl.n, cand_cap=cand_cap)
        x, y, e = s.upload(wl.x_q8, wl.y_q8, wl.epoch)
        s.vote(x, y, e)
        s.peaks()  # checks the result (overflow, data errors)
        snr = torch.as_tensor(np.ascontiguousarray(wl.snr, dtype=np.float32)).cuda()
        recs, feat = s.features(wl.n, snr, spacing_q8=sas.grid_spacing(wl.binw_q8, wl.span_q16))
    finally:
        plan.close()
    # canonical order (the device appends candidates in no fixed order)
    order = np.lexsort((recs["bx"], recs["by"], recs["v_idx"]))
    recs, feat = recs[order], feat[order]
    present = np.zeros(wl.n_epochs, dtype=bool)
    present[np.asarray(wl.epoch, dtype=np.int64)] = True
    t0 = int(np.asarray(wl.t_q16)[present].min())
    return recs, feat, recs["count"].astype(np.int32), t0


def balance(matched, cap, seed=0):
    """Mask keeping every negative and at most `cap` (random) candidates of
    each mover; cap 0 keeps everything."""
    m = np.asarray(matched)
    keep = np.ones(len(m), dtype=bool)
    if cap <= 0:
        return keep
    rng = np.random.default_rng(seed)
    for k in np.unique(m[m >= 0]):
        ids = np.nonzero(m == k)[0]
        if len(ids) > cap:
            keep[rng.choice(ids, len(ids) - cap, replace=False)] = False
    return keep


def superset_tau(scores, matched, findable_mask, plain_selected):
    """Largest threshold that keeps every findable mover found by the plain
    selection: the smallest, over those movers, of their best score (inf
    when there are none)."""
    sc = np.asarray(scores)
    m = np.asarray(matched)
    fmask = np.asarray(findable_mask, dtype=bool)
    sel = np.asarray(plain_selected, dtype=bool)
    movers = np.unique(m[sel & (m >= 0)])
    movers = movers[fmask[movers]]
    if len(movers) == 0:
        return float("inf")
    order = np.argsort(m, kind="stable")
    ms = m[order]
    best = np.full(len(fmask), -np.inf)
    pos = ms >= 0
    np.maximum.at(best, ms[pos], sc[order][pos])
    return float(best[movers].min())


def budget_tau(scores, matched, n_fp):
    """Lowest threshold with at most n_fp unmatched candidates at or above
    it (-inf when there are no more than n_fp of them)."""
    neg = np.sort(np.asarray(scores, dtype=np.float32)[np.asarray(matched) < 0])[::-1]
    n_fp = int(n_fp)
    if n_fp >= len(neg):
        return float("-inf")
    return float(np.nextafter(neg[n_fp], np.float32(np.inf)))


class Vetter:
    """Train and apply the vetting ensemble."""

    def __init__(self, members=5, seed=0, max_batch=4096):
        self.nets = [sas.MLP(max_batch=max_batch, seed=seed + k) for k in range(members)]
        self.seed = seed
        self.max_batch = max_batch
        self.mean = None
        self.std = None
        self.tau = None

    def fit(self, feats, labels, epochs=60, lr=1e-3, weight_decay=0.01, log=None):
        import torch
        x = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        self.mean = x.mean(axis=0)
        self.std = x.std(axis=0)
        n_pos = max(float(y.sum()), 1.0)
        pw = min((len(y) - n_pos) / n_pos, 100.0)
        xt = torch.as_tensor(x).cuda()
        yt = torch.as_tensor(y).cuda()
        B = self.max_batch
        for k, net in enumerate(self.nets):
            net.set_norm(self.mean, self.std)
            rng = np.random.default_rng(self.seed + 1000 + k)
            for ep in range(epochs):
                perm = torch.as_tensor(rng.permutation(len(y))).cuda()
                xs, ys = xt[perm].contiguous(), yt[perm].contiguous()
                loss = None
                for b in range(0, len(y) - B + 1 if len(y) >= B else 1, B):
                    loss = net.train_step(xs[b:b + B], ys[b:b + B], pw, lr=lr,
                                          weight_decay=weight_decay)
                if log and loss is not None and (ep == epochs - 1 or ep % 20 == 0):
                    log("member %d epoch %d  loss %.4f  (pos_weight %.1f, %d rows)"
                        % (k, ep, float(loss.cpu()), pw, len(y)))
        return self

    def score(self, feats):
        import torch
        x = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float32)).cuda()
        if x.shape[0] == 0:
            return np.zeros(0, dtype=np.float32)
        out = None
        B = self.max_batch
        for net in self.nets:
            z = torch.cat([net.forward(x[b:b + B]) for b in range(0, x.shape[0], B)])
            out = z if out is None else out + z
        return (out / len(self.nets)).cpu().numpy()

    def choose_tau(self, scores, matched, findable_mask, plain_selected, fp_budget=0.1):
        """Operating point on validation: min(superset_tau, budget_tau with
        fp_budget times the plain selection's false positives)."""
        plain_fp = recall_fp(plain_selected, matched, findable_mask)[1]
        self.tau = min(superset_tau(scores, matched, findable_mask, plain_selected),
                       budget_tau(scores, matched, int(fp_budget * plain_fp)))
        return self.tau

    def close(self):
        for net in self.nets:
            net.close()
        self.nets = []


def pools(seeds, n_pool, n_min, make, log=None):
    """Candidate pools of the catalogs make(seed): features, labels (matched
    mover, or -1, with movers numbered across the catalogs), counts and the
    findable mask of those movers."""
    F, M, C, FIND = [], [], [], []
    off = 0
    for sd in seeds:
        wl = make(sd)
        v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
        recs, feat, cnt, t0 = candidate_pool(wl, v, n_pool)
        m = match_movers(recs, v, wl.binw_q8, wl.t_q16, t0, wl.truth, wl.bin_px)
        fnd = findable(wl.truth, n_min)
        if log:
            log("seed %d: pool %d, matched %d, findable movers %d"
                % (sd, len(recs), int((m >= 0).sum()), int(fnd.sum())))
        F.append(feat)
        M.append(np.where(m >= 0, m + off, -1))
        C.append(cnt)
        FIND.append(fnd)
        off += len(fnd)
    return (np.concatenate(F), np.concatenate(M), np.concatenate(C), np.concatenate(FIND))


def evaluate(train_seeds, val_seeds, test_seeds, n_pool, n_min, make, members=5, cap=8,
             epochs=60, seed=0, fp_budget=0.1, log=None):
    """The vetting protocol: pools at n_pool, training on balanced train
    pools, tau on validation, recall and false positives on test for the
    plain threshold n_min and for the learned selection."""
    tr = pools(train_seeds, n_pool, n_min, make, log)
    va = pools(val_seeds, n_pool, n_min, make, log)
    te = pools(test_seeds, n_pool, n_min, make, log)
    keep = balance(tr[1], cap, seed)
    vet = Vetter(members=members, seed=seed)
    try:
        vet.fit(tr[0][keep], (tr[1][keep] >= 0).astype(np.float32), epochs=epochs, log=log)
        tau = vet.choose_tau(vet.score(va[0]), va[1], va[3], va[2] >= n_min, fp_budget)
        st = vet.score(te[0])
    finally:
        vet.close()
    plain = recall_fp(te[2] >= n_min, te[1], te[3])
    learned = recall_fp(st >= tau, te[1], te[3])
    curve = {int(k): recall_fp(te[2] >= k, te[1], te[3]) for k in range(n_pool, n_min + 5)}
    return {"plain": plain, "learned": learned, "tau": tau, "n_min": n_min, "n_pool": n_pool,
            "pool_test": int(len(te[2])), "findable_test": int(te[3].sum()),
            "train_rows": int(keep.sum()), "members": members, "epochs": epochs,
            "plain_curve": curve}


# Seeds of the fast-style vetting protocol (train / validation / test chips).
TRAIN_SEEDS = tuple(range(100, 136))
VAL_SEEDS = tuple(range(200, 212))
TEST_SEEDS = tuple(range(300, 312))
POOL_N_MIN = 19


def fast_protocol(members=5, epochs=60, log=None, train=TRAIN_SEEDS, val=VAL_SEEDS,
                  test=TEST_SEEDS):
    """The protocol on fast-style chips: pool at N_pool = 19, plain threshold
    from the threshold rule (Sec. 2.2) for the fast style."""
    from . import synth
    return evaluate(train, val, test, POOL_N_MIN, synth.FAST_N_MIN, synth.make_fast,
                    members=members, epochs=epochs, log=log)


# Seeds of the wide-style protocol: noise-dominated pools of the wide chip.
WIDE_TRAIN_SEEDS = tuple(range(400, 408))
WIDE_VAL_SEEDS = (410, 411)
WIDE_TEST_SEEDS = (420, 421)
# Pool threshold: the threshold rule (Sec. 2.2) at this many expected noise
# candidates per chip.  It gives N_pool = 8 on the wide chip, where the pools
# hold about 2.3e5 candidates per chip (2.8e6 over the protocol's 12 chips),
# about 99.8% of them unmatched to any mover.
WIDE_POOL_FALSE = 1e5


def pool_threshold(wl, v, n_false):
    """The threshold rule of Sec. 2.2 (sas_threshold_n_min) for this chip's
    noise density and grid at n_false expected noise candidates."""
    area = float(wl.width_px * wl.height_px)
    mu = wl.n / wl.n_epochs * wl.bin_px ** 2 / area
    return sas.threshold_n_min(wl.n_epochs, mu, len(v) * area / wl.bin_px ** 2, n_false)


def wide_protocol(members=5, epochs=60, log=None, train=WIDE_TRAIN_SEEDS, val=WIDE_VAL_SEEDS,
                  test=WIDE_TEST_SEEDS, n_false=WIDE_POOL_FALSE):
    """The protocol on wide-style chips (slow movers, 100 epochs, 4 px bins):
    pools at N_pool from the threshold rule, dominated by noise candidates;
    the plain threshold is the workload's N_min = 25."""
    from . import synth
    wl = synth.make_wide(train[0])
    n_pool = pool_threshold(wl, sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16), n_false)
    out = evaluate(train, val, test, n_pool, wl.n_min, synth.make_wide, members=members,
                   epochs=epochs, log=log)
    out["pool_false_target"] = n_false
    return out


if __name__ == "__main__":
    import json
    import sys
    import time
    t_start = time.time()

    def _log(msg):
        print("%7.1fs %s" % (time.time() - t_start, msg), file=sys.stderr, flush=True)

    for name, proto in (("fast", fast_protocol), ("wide", wide_protocol)):
        if len(sys.argv) > 1 and sys.argv[1] != name:
            continue
        out = proto(log=_log)
        out["plain_curve"] = {str(k): v for k, v in out["plain_curve"].items()}
        out["protocol"] = name
        print(json.dumps(out), flush=True)

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
  * training: the MLP of sas_mlp_* on standardised features, binary
    cross-entropy with positives weighted by min(n_neg / n_pos, 100), AdamW;
  * operating point: the score threshold tau is the largest one whose
    recall on validation catalogs reaches the plain threshold's recall there.

Recall counts findable movers (at least N_min epochs on the chip) with at
least one selected candidate matched to them; false positives are selected
candidates matched to no mover.
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
        recs, feat = s.features(wl.n, snr)
    finally:
        plan.close()
    # canonical order (the device appends candidates in no fixed order)
    order = np.lexsort((recs["bx"], recs["by"], recs["v_idx"]))
    recs, feat = recs[order], feat[order]
    present = np.zeros(wl.n_epochs, dtype=bool)
    present[np.asarray(wl.epoch, dtype=np.int64)] = True
    t0 = int(np.asarray(wl.t_q16)[present].min())
    return recs, feat, recs["count"].astype(np.int32), t0


class Vetter:
    """Train and apply the vetting network."""

    def __init__(self, seed=0, max_batch=4096):
        self.net = sas.MLP(max_batch=max_batch, seed=seed)
        self.max_batch = max_batch
        self.mean = None
        self.std = None
        self.tau = None

    def fit(self, feats, labels, epochs=6, lr=1e-3, weight_decay=0.01, seed=0, log=None):
        import torch
        x = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        self.mean = x.mean(axis=0)
        self.std = x.std(axis=0)
        self.net.set_norm(self.mean, self.std)
        n_pos = max(float(y.sum()), 1.0)
        pw = min((len(y) - n_pos) / n_pos, 100.0)
        xt = torch.as_tensor(x).cuda()
        yt = torch.as_tensor(y).cuda()
        rng = np.random.default_rng(seed)
        B = self.max_batch
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(len(y))).cuda()
            xs, ys = xt[perm].contiguous(), yt[perm].contiguous()
            tot = 0.0
            nb = 0
            for b in range(0, len(y) - B + 1 if len(y) >= B else 1, B):
                xb, yb = xs[b:b + B], ys[b:b + B]
                loss = self.net.train_step(xb, yb, pw, lr=lr, weight_decay=weight_decay)
                nb += 1
                if nb % 50 == 0 or b + 2 * B > len(y):
                    tot = float(loss.cpu())
            if log:
                log("epoch %d  loss %.4f  (pos_weight %.1f, %d rows)" % (ep, tot, pw, len(y)))
        return self

    def score(self, feats):
        import torch
        x = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float32)).cuda()
        if x.shape[0] == 0:
            return np.zeros(0, dtype=np.float32)
        return self.net.forward(x).cpu().numpy()

    def choose_tau(self, scores, matched, findable_mask, target_recall):
        """Largest threshold whose recall reaches target_recall."""
        order = np.argsort(-scores)
        taus = np.unique(scores)[::-1]
        best = float(taus[-1]) if len(taus) else 0.0
        # scan thresholds from high to low; recall is monotone in tau
        lo, hi = 0, len(taus) - 1
        while lo <= hi:
            mid = (lo + hi) // 2
            r, _ = recall_fp(scores >= taus[mid], matched, findable_mask)
            if r >= target_recall:
                best = float(taus[mid])
                hi = mid - 1
            else:
                lo = mid + 1
        self.tau = best
        return best

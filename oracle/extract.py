"""Greedy cluster extraction, Step 3 of Sec. 2.1 (TEST INFRASTRUCTURE ONLY,
see oracle/__init__.py).

Step 3 repeatedly takes the location of the maximum of the three-dimensional
histogram (trial velocity x 2-D bin); while that maximum is at least N_min,
the catalog points that contributed to it form a cluster and are removed from
the histogram (every cell they counted in loses them), and the loop goes on.

Written out plainly:
  * the contributors of a cell (v, bx, by) are the detections whose exact
    Step-2 bin at velocity v is (bx, by):
        bx_i = floor((65536 x_i - vx d_i) / (65536 b)),  d_i = t_e(i) - t0,
    with t0 the earliest epoch holding a detection (Step 1);
  * a cell's count is the number of distinct epochs among its live
    contributors ("epochs" mode) or their number ("detections");
  * counts only fall as points are removed, so a cell below N_min at the
    start never becomes the maximum: the loop runs over the cells the vote
    reported at N_min;
  * ties of the maximum are broken by (count descending, v_idx, by, bx
    ascending) - the paper does not say which of equal maxima comes first.

Each extracted cluster is reported as (v_idx, bx, by, count at extraction)
with the detections it took (catalog indices), in extraction order.
"""
from __future__ import annotations

import numpy as np

from .features import reference_dt


def contributors(x_q8, y_q8, epoch, t_q16, v_q8, binw_q8, cand):
    """Catalog indices of the contributing detections of each candidate."""
    xa = np.asarray(x_q8, dtype=np.int64)
    ya = np.asarray(y_q8, dtype=np.int64)
    ea = np.asarray(epoch, dtype=np.int64)
    t = np.asarray(t_q16, dtype=np.int64)
    d = reference_dt(t, ea, int(t.shape[0]))[ea]  # d of each detection
    v = np.asarray(v_q8, dtype=np.int64)
    b = 65536 * int(binw_q8)
    out = []
    for c in cand:
        vx, vy = int(v[int(c["v_idx"]), 0]), int(v[int(c["v_idx"]), 1])
        bx = (65536 * xa - vx * d) // b  # floor division
        by = (65536 * ya - vy * d) // b
        out.append(np.nonzero((bx == int(c["bx"])) & (by == int(c["by"])))[0])
    return out


def _count(members, alive, epoch, mode):
    live = members[alive[members]]
    if mode == "epochs":
        return int(np.unique(epoch[live]).shape[0])
    return int(live.shape[0])


def extract(x_q8, y_q8, epoch, t_q16, v_q8, binw_q8, cand, n_min, mode="epochs"):
    """The loop of Step 3 over the candidate cells `cand` (records with
    v_idx, bx, by): list of (v_idx, bx, by, count, detection indices)."""
    ea = np.asarray(epoch, dtype=np.int64)
    members = contributors(x_q8, y_q8, epoch, t_q16, v_q8, binw_q8, cand)
    alive = np.ones(ea.shape[0], dtype=bool)  # detections not yet in a cluster
    open_ = np.ones(len(cand), dtype=bool)    # cells that may still reach N_min
    clusters = []
    while True:
        best, best_key = -1, None
        for k in range(len(cand)):
            if not open_[k]:
                continue
            n = _count(members[k], alive, ea, mode)
            if n < n_min:
                open_[k] = False
                continue
            c = cand[k]
            key = (-n, int(c["v_idx"]), int(c["by"]), int(c["bx"]))
            if best_key is None or key < best_key:
                best, best_key = k, key
        if best < 0:
            return clusters
        took = members[best][alive[members[best]]]
        c = cand[best]
        clusters.append((int(c["v_idx"]), int(c["bx"]), int(c["by"]), -best_key[0], took))
        alive[took] = False
        open_[best] = False

"""Brute-force voting transform in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

This is Steps 1-2 of the algorithm (Sec. 2.1) written with
``fractions.Fraction`` and pure Python loops, for inputs of a few hundred
detections at most:

  * Step 1, Project: the reference time is the earliest observation time in
    the catalog; each detection's position is moved back to it along the
    trial velocity, x0 = x - v (t - t0) (the linear model of eqs. 1-2 solved
    for the position at t0);
  * Step 2, Cluster: a 2-D histogram of the projected positions with square
    bins of side Delta x anchored at the origin (bin k covers
    [k Delta x, (k+1) Delta x));
  * the count of a bin is the number of distinct epochs (or of detections)
    that fall in it, and bins with count >= N_min are reported (the stopping
    rule of Step 3 read as a threshold);
  * weighted counts (a per-detection likelihood accumulated instead of an
    indicator, Conclusions): per epoch the largest weight among the bin's
    detections of that epoch, summed over epochs ("weighted_epochs"), or the
    sum of all their weights ("weighted_detections").

Units: positions in px, velocities in px/h, times in h, all as exact
rationals built from the integer catalog (Q8 px, Q8 px/h, Q16 h).
"""
from __future__ import annotations

import math
from fractions import Fraction


def project(x_q8, t_q16, t0_q16, u_q8):
    """Position (px, exact) at the reference time under velocity u."""
    x = Fraction(int(x_q8), 256)
    dt = Fraction(int(t_q16) - int(t0_q16), 65536)
    return x - Fraction(int(u_q8), 256) * dt


def _score(members, mode):
    """Count of a bin from its (epoch, weight) members."""
    if mode == "epochs":
        return len({e for e, _ in members})
    if mode == "detections":
        return len(members)
    if mode == "weighted_detections":
        return sum(w for _, w in members)
    best = {}
    for e, w in members:
        best[e] = max(best.get(e, 0), w)
    return sum(best.values())


def brute_vote(x_q8, y_q8, epoch, t_q16, v_q8, binw_q8, n_min, mode="epochs",
               count_sat=65535, weight=None):
    """List of (v_idx, bx, by, count, flags) ordered by (v_idx, by, bx)."""
    n = len(x_q8)
    if n == 0:
        return []
    t0 = min(int(t_q16[int(e)]) for e in epoch)
    width = Fraction(int(binw_q8), 256)
    out = []
    for j, (u, w) in enumerate(v_q8):
        bins = {}
        for i in range(n):
            e = int(epoch[i])
            xp = project(x_q8[i], t_q16[e], t0, u)
            yp = project(y_q8[i], t_q16[e], t0, w)
            key = (math.floor(yp / width), math.floor(xp / width))
            bins.setdefault(key, []).append((e, int(weight[i]) if weight is not None else 1))
        for (by, bx) in sorted(bins):
            c = _score(bins[(by, bx)], mode)
            if c >= n_min:
                sat = c > count_sat
                out.append((j, bx, by, min(c, count_sat), 1 if sat else 0))
    return out


def brute_bin(x_q8, y_q8, e, t_q16, t0, u_q8, w_q8, binw_q8):
    """Bin (bx, by) of one detection under one velocity."""
    width = Fraction(int(binw_q8), 256)
    xp = project(x_q8, t_q16[e], t0, u_q8)
    yp = project(y_q8, t_q16[e], t0, w_q8)
    return math.floor(xp / width), math.floor(yp / width)

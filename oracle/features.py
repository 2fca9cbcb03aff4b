"""Candidate features and labels for learned vetting (TEST INFRASTRUCTURE ONLY,
see oracle/__init__.py).

The paper does not define features for vetting candidates; this module is
the plain FP64 definition of the 32 features the GPU path computes, written
as loops over a candidate's contributing detections.

A candidate is a (velocity v, bin (bx, by)) reported by the vote.  Its
contributing detections are those whose exact Step-2 bin at velocity v is
(bx, by) (Sec. 2.1, Steps 1-2): with d = t_e - t0 (Q16 h, t0 the earliest
epoch holding a detection), bx_i = floor((65536 x_i - vx d) / (65536 b)).
A detection's residual inside the bin, in bins, is
    r_x = (65536 x - vx d) / (65536 b) - bx - 1/2  in [-1/2, 1/2),
the offset of its projected position from the bin centre.

With E epochs, span D (Q16 h, last - first epoch of the plan), vmax the
largest |v| of the grid, P the distinct epochs and C the detections
(c = |P|, n = |C|), and time slices s = min(3, floor(4 d / D)):
  f0 c / E                   f1 n / E
  f2 min_P d / D             f3 (max_P d - min_P d) / D
  f4 longest run of consecutive epoch indices in P, / E
  f5 vx / vmax   f6 vy / vmax   f7 |v| / vmax
  f8 sum(snr) / E   f11 mean(snr) - 3
  f9  number of neighbouring candidates / 80
  f10 largest count among neighbouring candidates / own count (0: none)
      Neighbours are the other candidates of the same list whose lattice
      velocity index (v / s rounded half up, s the grid spacing) differs by
      at most 1 in each component and whose bin differs by at most 1 in
      each axis (a real mover's stack spreads over neighbouring velocities
      and bins; a noise stack stands alone).  Counts are capped at 4095;
      candidates that share a lattice index and bin count as one, with
      the largest of their counts.
      Candidates whose lattice index or bin falls outside +-1022 / +-16382
      get no neighbours.
  f12, f13 mean r_x, mean r_y      f14, f15 population std of r_x, r_y
  f16, f17 least-squares slope of r_x, r_y against d / D (bins per span;
           0 when all d are equal)
  f18 + 2s, f19 + 2s  mean r_x, mean r_y over the detections of slice s
           (0 when the slice is empty), s = 0..3
  f26 + s  fraction of C in slice s
  f30 (n - c) / n   (detections sharing an epoch)
  f31 root mean square of r_x and r_y about their least-squares lines
      against d / D (the linear trajectory fit of Sec. 2.1, Step 4, on the
      candidate's own detections): sqrt((SSE_x + SSE_y) / (2 n))
"""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 32


def reference_dt(t_q16, epoch, n_epochs):
    """d_e = t_e - t0 with t0 the earliest epoch holding a detection; -1 for
    epochs without detections (Sec. 2.1, Step 1)."""
    t = np.asarray(t_q16, dtype=np.int64)
    present = np.zeros(n_epochs, dtype=bool)
    present[np.asarray(epoch, dtype=np.int64)] = True
    t0 = int(t[present].min())
    return np.where(present, t - t0, -1).astype(np.int64)


def _lattice(v, s):
    return (2 * int(v) + s) // (2 * s)  # v / s rounded half up


def _packable(ix, iy, bx, by):
    return abs(ix) <= 1022 and abs(iy) <= 1022 and abs(bx) <= 16382 and abs(by) <= 16382


def neighbour_features(cand, v_q8, spacing_q8, rows=None):
    """(f9, f10) of the candidates `rows` (default: all) of the list, their
    neighbours taken among the whole list (definitions above)."""
    n = len(cand)
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), 2), dtype=np.float64)
    if not spacing_q8 or n == 0:
        return out
    v = np.asarray(v_q8, dtype=np.int64)
    keyed = {}
    keys = []
    for i, c in enumerate(cand):
        vx, vy = v[int(c["v_idx"])]
        k = (_lattice(vx, spacing_q8), _lattice(vy, spacing_q8), int(c["bx"]), int(c["by"]))
        keys.append(k)
        if _packable(*k):  # candidates sharing a key: the largest count stands for them
            keyed[k] = max(keyed.get(k, 0), min(int(c["count"]), 4095))
    for r, i in enumerate(rows):
        k = keys[i]
        if not _packable(*k):
            continue
        own = min(int(cand[i]["count"]), 4095)
        cnt, best = 0, 0
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for cx in (-1, 0, 1):
                    for cy in (-1, 0, 1):
                        if a == b == cx == cy == 0:
                            continue
                        q = keyed.get((k[0] + a, k[1] + b, k[2] + cx, k[3] + cy))
                        if q is not None:
                            cnt += 1
                            best = max(best, q)
        out[r, 0] = cnt / 80.0
        out[r, 1] = best / own if cnt and own else 0.0
    return out


def candidate_features(x_q8, y_q8, epoch, snr, t_q16, v_q8, binw_q8, cand, vmax_q8=None,
                       spacing_q8=0):
    """[n_cand, 32] float64 features of the candidates (records with v_idx,
    bx, by, count), following the definitions above; the neighbour features
    look among the candidates of `cand` (zeros when spacing_q8 is 0)."""
    xa = np.asarray(x_q8, dtype=np.int64)
    ya = np.asarray(y_q8, dtype=np.int64)
    ea = np.asarray(epoch, dtype=np.int64)
    sn = np.asarray(snr, dtype=np.float64)
    t = np.asarray(t_q16, dtype=np.int64)
    E = int(t.shape[0])
    d = reference_dt(t, ea, E)
    di_all = d[ea]  # d of each detection
    D = max(int(t.max() - t.min()), 1)
    v = np.asarray(v_q8, dtype=np.int64)
    if vmax_q8 is None:
        vmax_q8 = float(np.sqrt((v.astype(np.float64) ** 2).sum(axis=1)).max()) if len(v) else 1.0
    vmax = max(float(vmax_q8), 1.0)
    b = int(binw_q8)
    out = np.zeros((len(cand), N_FEATURES), dtype=np.float64)
    for k, c in enumerate(cand):
        vx, vy = int(v[int(c["v_idx"]), 0]), int(v[int(c["v_idx"]), 1])
        bx, by = int(c["bx"]), int(c["by"])
        # exact bins of every detection (int64 holds 65536 x - v d exactly;
        # // is floor division), then the contributors one by one
        nx_all = 65536 * xa - vx * di_all
        ny_all = 65536 * ya - vy * di_all
        hit = np.nonzero((nx_all // (65536 * b) == bx) & (ny_all // (65536 * b) == by))[0]
        rows = []  # (epoch, d, r_x, r_y, snr)
        for i in hit:
            nx, ny = int(nx_all[i]), int(ny_all[i])
            rx = nx / (65536.0 * b) - bx - 0.5
            ry = ny / (65536.0 * b) - by - 0.5
            rows.append((int(ea[i]), int(di_all[i]), rx, ry, float(sn[i])))
        f = out[k]
        n = len(rows)
        if n == 0:
            continue
        eps_set = sorted({r[0] for r in rows})
        cnum = len(eps_set)
        f[0] = cnum / E
        f[1] = n / E
        dl = [int(d[e]) for e in eps_set]
        f[2] = min(dl) / D
        f[3] = (max(dl) - min(dl)) / D
        best = run = 1
        for a, bb in zip(eps_set, eps_set[1:]):
            run = run + 1 if bb == a + 1 else 1
            best = max(best, run)
        f[4] = best / E
        f[5] = vx / vmax
        f[6] = vy / vmax
        f[7] = math.hypot(vx, vy) / vmax
        s = [r[4] for r in rows]
        f[8] = sum(s) / E
        f[11] = sum(s) / n - 3.0
        rx = [r[2] for r in rows]
        ry = [r[3] for r in rows]
        mx, my = sum(rx) / n, sum(ry) / n
        f[12], f[13] = mx, my
        f[14] = math.sqrt(sum((a - mx) ** 2 for a in rx) / n)
        f[15] = math.sqrt(sum((a - my) ** 2 for a in ry) / n)
        tau = [r[1] / D for r in rows]
        mt = sum(tau) / n
        stt = sum((a - mt) ** 2 for a in tau)
        if len({r[1] for r in rows}) > 1:  # not all d equal (exact, on the integers)
            f[16] = sum((a - mt) * (bq - mx) for a, bq in zip(tau, rx)) / stt
            f[17] = sum((a - mt) * (bq - my) for a, bq in zip(tau, ry)) / stt
        sse = sum((bq - mx - f[16] * (a - mt)) ** 2 for a, bq in zip(tau, rx)) + \
            sum((bq - my - f[17] * (a - mt)) ** 2 for a, bq in zip(tau, ry))
        f[31] = math.sqrt(sse / (2 * n))
        for sl in range(4):
            idx = [j for j in range(n) if min(3, (4 * rows[j][1]) // D) == sl]
            if idx:
                f[18 + 2 * sl] = sum(rx[j] for j in idx) / len(idx)
                f[19 + 2 * sl] = sum(ry[j] for j in idx) / len(idx)
            f[26 + sl] = len(idx) / n
        f[30] = (n - cnum) / n
    out[:, 9:11] = neighbour_features(cand, v, spacing_q8)
    return out


def label_candidates(cand, v_q8, binw_q8, t_q16, t0_q16, truth, bin_px, frac=0.5):
    """1 for a candidate whose track (bin centre at t0 moved with its trial
    velocity) passes within one bin width of some injected mover in at least
    `frac` of the epochs, else 0.  truth: x_mid, y_mid (px), vx, vy (px/h)
    of each mover and t_mid_h, on a clock that starts at the first epoch."""
    t = np.asarray(t_q16, dtype=np.float64)
    v = np.asarray(v_q8, dtype=np.float64)
    E = t.shape[0]
    th = (t - float(t0_q16)) / 65536.0          # hours since t0
    t_abs_h = (t - t.min()) / 65536.0           # the truth's clock: hours since the first epoch
    out = np.zeros(len(cand), dtype=np.uint8)
    if len(truth["vx"]) == 0:
        return out
    mx = truth["x_mid"][:, None] + truth["vx"][:, None] * (t_abs_h[None, :] - truth["t_mid_h"])
    my = truth["y_mid"][:, None] + truth["vy"][:, None] * (t_abs_h[None, :] - truth["t_mid_h"])
    b = binw_q8 / 256.0
    for k, c in enumerate(cand):
        vx, vy = v[int(c["v_idx"])] / 256.0
        cx = (int(c["bx"]) + 0.5) * b + vx * th
        cy = (int(c["by"]) + 0.5) * b + vy * th
        dist = np.hypot(mx - cx[None, :], my - cy[None, :])
        close = (dist < bin_px).sum(axis=1)
        out[k] = 1 if (close >= frac * E).any() else 0
    return out

"""Weighted votes against the indicator vote on faint movers.

The Conclusions suggest accumulating a detection likelihood instead of the
detected / not-detected indicator, so that a stack of real detections
outweighs a stack of noise peaks, and leave the trade-off open.  This module
measures it on the ``faint`` catalogs (movers whose detections follow from
their flux, noise peaks from the Gaussian tail above SNR 3):

  * indicator: EPOCHS counts at the plain threshold N_min of Sec. 2.2
    (expected pure-noise candidates <= 100 over the grid);
  * weighted: WEIGHTED_EPOCHS scores with the weights of
    ``synth.likelihood_weights`` (per epoch the best detection's
    log-likelihood ratio s^2 / 2, quantised), at the lowest score threshold
    W* whose noise candidates on the validation chips do not exceed the
    indicator's there.  Noise candidates are counted on each chip's
    noise-only catalog (its movers removed), the false alarms that the
    threshold rule of Sec. 2.2 bounds;
  * on the test chips: recall (movers matched by at least one selected
    candidate, by true SNR), noise candidates, unmatched candidates of the
    whole catalog (noise plus the ghosts of real movers at other velocities
    and bins), and the SNR at which half the movers are found (the analogue
    of the depth m50 of Sec. 3).

Both votes run on the GPU through the C ABI; matching and counting are host
bookkeeping.
"""
from __future__ import annotations

import numpy as np

from . import sas, synth
from .vetting import match_movers

VAL_SEEDS = tuple(range(600, 604))
TEST_SEEDS = tuple(range(700, 706))
SNR_BINS = np.arange(1.5, 4.01, 0.25)


def plain_n_min(wl, n_v: int, n_false: float = 100.0) -> int:
    """The threshold rule of Sec. 2.2 for a chip: binomial epochs at the
    chip's mean noise occupancy per bin, n_v velocities x bins stacks."""
    noise = int((np.asarray(wl.is_mover) < 0).sum())
    area = float(wl.width_px * wl.height_px)
    mu = noise / wl.n_epochs * wl.bin_px ** 2 / area
    return sas.threshold_n_min(wl.n_epochs, mu, n_v * area / wl.bin_px ** 2, n_false)


def _reference_time(wl) -> int:
    present = np.zeros(wl.n_epochs, dtype=bool)
    present[np.asarray(wl.epoch, dtype=np.int64)] = True
    return int(np.asarray(wl.t_q16)[present].min())


def chip_lists(wl, v, n_lo: int, w_lo: int, scale: float = 4.0, cand_cap: int = 1 << 22):
    """Both votes of one chip at low thresholds: for the indicator and the
    weighted vote, (counts, matched mover or -1) of the whole catalog and the
    counts of its noise-only catalog."""
    noise = np.asarray(wl.is_mover) < 0
    w_all = synth.likelihood_weights(wl.snr, scale)
    out = []
    for mode, thr in (("epochs", n_lo), ("weighted_epochs", w_lo)):
        tun = {"n_det_hint": wl.n}
        if mode != "epochs":
            tun["weight_hint"] = int(round(float(w_all.mean())))
        plan = sas.Plan(v, wl.t_q16, wl.binw_q8, thr, wl.extent_q8, mode=mode, tuning=tun)
        try:
            s = sas.Search(plan, wl.n, cand_cap=cand_cap)
            wt = plan.weighted
            c = s.run(wl.x_q8, wl.y_q8, wl.epoch, weight=w_all if wt else None)
            cn = s.run(wl.x_q8[noise], wl.y_q8[noise], wl.epoch[noise],
                       weight=w_all[noise] if wt else None)
        finally:
            plan.close()
        m = match_movers(c, v, wl.binw_q8, wl.t_q16, _reference_time(wl), wl.truth, wl.bin_px)
        out.append((c["count"].astype(np.int64), m, cn["count"].astype(np.int64)))
    return out


def _selection(counts, matched, thr, n_movers):
    sel = counts >= thr
    found = np.zeros(n_movers, dtype=bool)
    m = matched[sel]
    found[m[m >= 0]] = True
    return found, int((m < 0).sum())


def snr50(snr, found, bins=SNR_BINS):
    """True SNR at which the found fraction crosses 1/2 (linear between bin
    centres; nan when it never does)."""
    c = 0.5 * (bins[1:] + bins[:-1])
    idx = np.digitize(snr, bins) - 1
    frac = np.array([found[idx == k].mean() if np.any(idx == k) else np.nan
                     for k in range(len(c))])
    for k in range(1, len(c)):
        a, b = frac[k - 1], frac[k]
        if a < 0.5 <= b:
            return float(c[k - 1] + (0.5 - a) / (b - a) * (c[k] - c[k - 1])), frac
    return float("nan"), frac


def compare(val_seeds=VAL_SEEDS, test_seeds=TEST_SEEDS, scale: float = 4.0, n_movers: int = 400,
            log=None) -> dict:
    """The protocol of the module header; returns its numbers."""
    say = log or (lambda m: None)
    chips = {}
    for seed in tuple(val_seeds) + tuple(test_seeds):
        wl = synth.make_faint(seed, n_movers=n_movers)
        v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
        n_min = plain_n_min(wl, len(v))
        w_noise = float(synth.likelihood_weights(
            wl.snr[np.asarray(wl.is_mover) < 0], scale).mean())
        n_lo, w_lo = max(1, n_min - 4), int(w_noise * max(1, n_min - 4))
        (ci, mi, ni), (cw, mw, nw) = chip_lists(wl, v, n_lo, w_lo, scale)
        chips[seed] = dict(wl=wl, n_min=n_min, ci=ci, mi=mi, ni=ni, cw=cw, mw=mw, nw=nw)
        say("faint chip %d: %d detections, |V| = %d, N_min = %d, %d / %d candidates, "
            "%d / %d noise-only" % (seed, wl.n, len(v), n_min, len(ci), len(cw), len(ni),
                                    len(nw)))
    # W*: the lowest score threshold within the indicator's validation noise candidates
    noise_plain = sum(int((chips[s]["ni"] >= chips[s]["n_min"]).sum()) for s in val_seeds)
    cand_w = np.unique(np.concatenate([chips[s]["nw"] for s in val_seeds] + [[w_lo]]))
    w_star = None
    for thr in cand_w:
        if sum(int((chips[s]["nw"] >= thr).sum()) for s in val_seeds) <= noise_plain:
            w_star = int(thr)
            break
    if w_star is None:
        w_star = int(cand_w.max()) + 1
    # the other reading: every unmatched candidate of the full catalogs a false positive
    unm_plain = sum(_selection(chips[s]["ci"], chips[s]["mi"], chips[s]["n_min"], n_movers)[1]
                    for s in val_seeds)
    cand_u = np.unique(np.concatenate([chips[s]["cw"] for s in val_seeds]))
    w_unm = int(cand_u.max()) + 1 if len(cand_u) else w_lo
    for thr in cand_u:
        if sum(_selection(chips[s]["cw"], chips[s]["mw"], thr, n_movers)[1]
               for s in val_seeds) <= unm_plain:
            w_unm = int(thr)
            break
    res = {"val_noise_plain": noise_plain, "w_star": w_star, "scale": scale,
           "val_unmatched_plain": unm_plain, "w_unmatched": w_unm,
           "w_lo": int(min(chips[s]["cw"].min() if len(chips[s]["cw"]) else 0 for s in chips))}
    snr_all, f_i, f_w, f_u = [], [], [], []
    fp_i = fp_w = fp_u = nz_i = nz_w = 0
    for s in test_seeds:
        c = chips[s]
        fi, pi = _selection(c["ci"], c["mi"], c["n_min"], n_movers)
        fw, pw = _selection(c["cw"], c["mw"], w_star, n_movers)
        fu, pu = _selection(c["cw"], c["mw"], w_unm, n_movers)
        snr_all.append(c["wl"].truth["snr"])
        f_i.append(fi)
        f_w.append(fw)
        f_u.append(fu)
        fp_i += pi
        fp_w += pw
        fp_u += pu
        nz_i += int((c["ni"] >= c["n_min"]).sum())
        nz_w += int((c["nw"] >= w_star).sum())
    snr_all, f_i, f_w, f_u = map(np.concatenate, (snr_all, f_i, f_w, f_u))
    s50_i, frac_i = snr50(snr_all, f_i)
    s50_w, frac_w = snr50(snr_all, f_w)
    s50_u, _ = snr50(snr_all, f_u)
    res.update({"test_movers": int(len(snr_all)),
                "indicator": {"recall": float(f_i.mean()), "noise_candidates": nz_i,
                              "unmatched": fp_i, "snr50": s50_i,
                              "recall_by_snr": frac_i.tolist()},
                "weighted": {"recall": float(f_w.mean()), "noise_candidates": nz_w,
                             "unmatched": fp_w, "snr50": s50_w,
                             "recall_by_snr": frac_w.tolist()},
                "weighted_matched_unmatched": {"recall": float(f_u.mean()), "unmatched": fp_u,
                                               "snr50": s50_u},
                "snr_bins": SNR_BINS.tolist(),
                "n_min": {int(s): int(chips[s]["n_min"]) for s in chips}})
    return res


if __name__ == "__main__":
    import json
    import sys
    r = compare(log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(r))

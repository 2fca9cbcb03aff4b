"""The batched survey night: 64 chips of one night, each with its own
catalog, velocity grid, threshold and plan.

Chip c of the night is drawn with seed 4000 + c (synth.night_chip_params):
wide or fast style with probability 1/2, detections log-uniform in
[5e4, 5e5], epochs uniform in {40..120}.  Wide-style chips take N_min =
round(E / 4); fast-style chips take the threshold rule of Sec. 2.2 for their
own epochs, noise density and grid.  Launch shapes come from the tuning
cache, keyed by shape class (or are tuned and stored with retune).
"""
from __future__ import annotations

import concurrent.futures as cf


def setup(n_chips=64, cache=None, retune=False, tune_set="small", log=None):
    """Chips of the night with their thresholds and plans; launch shapes
    from the tuning cache (retune: tune each shape class on its first chip
    and store the choice)."""
    import torch

    from . import autotune, sas, synth
    cache = cache or autotune.CACHE
    specs = []
    for p in synth.night_chip_params(4, n_chips):
        wl = synth.make_night_chip(p, 0)
        v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
        n_min = wl.n_min
        if p["style"] == "fast":  # the threshold rule of Sec. 2.2 for this chip
            area = float(wl.width_px * wl.height_px)
            mu = wl.n / wl.n_epochs * wl.bin_px ** 2 / area
            n_min = sas.threshold_n_min(wl.n_epochs, mu, len(v) * area / wl.bin_px ** 2)
        key = autotune.shape_class(v, wl.t_q16, wl.binw_q8, n_min, wl.extent_q8, wl.n)
        specs.append({"p": p, "wl": wl, "v": v, "n_min": n_min, "key": key,
                      "style": p["style"]})
    tuned, missing = {}, []
    for c in specs:
        if c["key"] in tuned:
            continue
        t = None if retune else autotune.cached(c["key"], cache)
        if t is None and not retune:
            missing.append(c["key"])  # planner defaults
        if t is None and retune:
            wl = c["wl"]
            if log:
                log("tuning class %s on chip %d" % (c["key"], c["p"]["chip"]))
            x = torch.as_tensor(wl.x_q8).cuda()
            y = torch.as_tensor(wl.y_q8).cuda()
            e = torch.as_tensor(wl.epoch).cuda()
            # small: the planner's choice and each lane-group count; full: the
            # library's whole candidate list around the planner's choice
            cands = [{}, {"groups": 1}, {"groups": 2}, {"groups": 4}] if tune_set == "small" \
                else None
            r = autotune.tune(c["v"], wl.t_q16, wl.binw_q8, c["n_min"], wl.extent_q8, x, y, e,
                              base={"n_det_hint": wl.n}, cands=cands, reps=2, log=log)
            t = {k: v_ for k, v_ in r["tuning"].items() if k != "n_det_hint"}
            autotune.store(c["key"], t, cache)
        tuned[c["key"]] = t or {}

    def make_plan(c):
        wl = c["wl"]
        tun = dict(tuned[c["key"]], n_det_hint=wl.n)
        return sas.Plan(c["v"], wl.t_q16, wl.binw_q8, c["n_min"], wl.extent_q8, tuning=tun)

    # plans are host analyses (the library releases the interpreter lock)
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        plans = list(ex.map(make_plan, specs))
    for c, plan in zip(specs, plans):
        wl = c["wl"]
        c["plan"] = plan
        c["x"] = torch.as_tensor(wl.x_q8).cuda()
        c["y"] = torch.as_tensor(wl.y_q8).cuda()
        c["e"] = torch.as_tensor(wl.epoch).cuda()
    return specs, tuned, missing

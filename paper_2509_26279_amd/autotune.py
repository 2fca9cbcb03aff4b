"""Launch-shape autotuner for the dense vote.

For one shape class of catalogs (bin width, lattice spacing, grid shape,
epoch count and detection count, bucketed), the tuner times candidate launch
shapes (lane groups, velocity block, tile, stage capacity) on the device
with the plan's timing probe around the vote kernel, checks that every
candidate produces the identical candidate list (a launch shape must never
change the output), and keeps the fastest.  Choices are cached in a JSON
file keyed by the shape class.

    from paper_2509_26279_amd import autotune
    best = autotune.tune(v, t_q16, binw_q8, n_min, extent_q8, x, y, e)
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import sas


def shape_class(binw_q8: int, spacing_q8: int, n_epochs: int, n_det: int, grid_shape: str,
                mode: str = "epochs") -> str:
    """Key of a class of catalogs that share their best launch shape."""
    e_lo = 1 << int(math.floor(math.log2(max(n_epochs, 1))))
    n_lo = 1 << int(math.floor(math.log2(max(n_det, 1))))
    return "b%d_s%d_E%d_n%d_%s_%s" % (binw_q8, spacing_q8, e_lo, n_lo, grid_shape, mode)


def candidates(base: dict) -> list:
    """Launch shapes around the planner's own choice for each lane-group count."""
    out = [dict()]
    for g in (1, 2, 4):
        out.append({"groups": g})
        for cl in (-1, 1):  # window-index cells one step finer or coarser than the planner's
            out.append({"groups": g, "cell_log2_step": cl})
        for tx, ty in ((8, 8), (12, 10), (16, 12), (24, 16), (16, 24)):
            out.append({"groups": g, "tile_x": tx, "tile_y": ty})
    return [dict(base, **c) for c in out]


def _time_vote(plan, n, x, y, e, reps):
    import torch
    s = sas.Search(plan, n, cand_cap=1 << 22)
    s.vote(x, y, e)
    out = s.peaks()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        b.record()
    torch.cuda.synchronize()
    for a, b in evs:
        plan.set_probe(a, b)
        s.vote(x, y, e)
        s.peaks()
    torch.cuda.synchronize()
    plan.set_probe(None, None)
    return float(np.median([a.elapsed_time(b) for a, b in evs])), out


def tune(v, t_q16, binw_q8, n_min, extent_q8, x, y, e, mode="epochs", count_sat=65535,
         base=None, reps=3, cands=None, log=None):
    """Time the candidate launch shapes on one catalog (device tensors x, y,
    e) and return {"tuning": best, "ms": ..., "table": [...]}.  Raises if two
    shapes disagree on the candidate list."""
    base = dict(base or {})
    base.setdefault("n_det_hint", int(x.numel()))
    ref = None
    table = []
    # explicit candidates are read relative to the base tuning (the shapes
    # are timed with the same hints the plans that use them will have)
    for tun in ([dict(base, **c) for c in cands] if cands else candidates(base)):
        try:
            if "cell_log2_step" in tun:  # relative to the planner's window-index cells
                tun = dict(tun)
                step = tun.pop("cell_log2_step")
                probe = sas.Plan(v, t_q16, binw_q8, n_min, extent_q8, mode=mode,
                                 count_sat=count_sat, tuning=tun)
                tun["cell_log2"] = probe.info()["cell_log2"] + step
                probe.close()
            plan = sas.Plan(v, t_q16, binw_q8, n_min, extent_q8, mode=mode,
                            count_sat=count_sat, tuning=tun)
        except sas.SasError as err:  # shape does not fit (LDS, guard cells)
            table.append({"tuning": tun, "ms": None, "error": str(err)})
            continue
        try:
            ms, out = _time_vote(plan, int(x.numel()), x, y, e, reps)
        finally:
            plan.close()
        if ref is None:
            ref = out
        elif not np.array_equal(out, ref):
            raise RuntimeError("launch shape %s changed the candidate list" % tun)
        table.append({"tuning": tun, "ms": ms})
        if log:
            log("  %-60s %8.3f ms" % (json.dumps(tun), ms))
    timed = [r for r in table if r["ms"] is not None]
    if not timed:
        raise RuntimeError("no candidate launch shape fits")
    best = min(timed, key=lambda r: r["ms"])
    return {"tuning": best["tuning"], "ms": best["ms"], "table": table}


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)

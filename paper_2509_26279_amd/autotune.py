"""Launch-shape autotuner of the dense vote (marshalling over sas_autotune*).

The library times candidate launch shapes (lane groups, velocity block,
tile, window-index cells) of one catalog with events around the vote kernel,
checks that every shape gives the identical candidate list, and returns the
fastest; choices are cached per shape class (bin width, lattice spacing,
epoch, detection and velocity counts by powers of two, mode) in a text file.

    from paper_2509_26279_amd import autotune
    best = autotune.tune(v, t_q16, binw_q8, n_min, extent_q8, x, y, e)

``CACHE`` is the committed cache of the benchmarked workloads' shape classes.
"""
from __future__ import annotations

import os

from . import sas

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.txt")


def shape_class(v, t_q16, binw_q8, n_min, extent_q8, n, mode="epochs") -> str:
    """Key of the class of catalogs that share their best launch shape."""
    return sas.autotune_key(v, t_q16, binw_q8, n_min, extent_q8, n, mode)


def candidates(v, t_q16, binw_q8, n_min, extent_q8, base: dict, mode="epochs",
               count_sat=65535) -> list:
    """The library's launch shapes around the planner's own choice."""
    return sas.autotune_default_candidates(v, t_q16, binw_q8, n_min, extent_q8, mode, count_sat,
                                           base)


def tune(v, t_q16, binw_q8, n_min, extent_q8, x, y, e, mode="epochs", count_sat=65535,
         base=None, reps=3, cands=None, log=None):
    """Time the candidate launch shapes on one catalog (device tensors x, y,
    e) and return {"tuning": best, "ms": ..., "table": [...]}.  Explicit
    candidates are read relative to the base tuning (the shapes are timed
    with the hints the plans that use them will have).  The library raises
    if two shapes disagree on the candidate list."""
    base = dict(base or {})
    base.setdefault("n_det_hint", int(x.numel()))
    cl = ([dict(base, **c) for c in cands] if cands else
          candidates(v, t_q16, binw_q8, n_min, extent_q8, base, mode, count_sat))
    best, table = sas.autotune(v, t_q16, binw_q8, n_min, extent_q8, x, y, e, cl, reps, mode,
                               count_sat)
    rows = [{"tuning": t, "ms": ms, "status": st} for t, ms, st in table]
    if log:
        for r in rows:
            log("  %-70s %s" % (r["tuning"], "%8.3f ms" % r["ms"] if r["ms"] is not None
                                else "does not fit"))
    ms = min(r["ms"] for r in rows if r["ms"] is not None)
    return {"tuning": best, "ms": ms, "table": rows}


def cached(key: str, path: str = CACHE):
    """The cached tuning of a shape class, or None."""
    return sas.autotune_cache_get(path, key)


def store(key: str, tuning: dict, path: str = CACHE) -> None:
    sas.autotune_cache_put(path, key, tuning)

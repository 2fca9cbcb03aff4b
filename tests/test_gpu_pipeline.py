"""The whole method on the GPU, Steps 1-6, on the wide workload: vote,
greedy extraction, FAST-MCD refine/gather.  The refined trajectories are
checked against the injected movers (physics, not parity: each step has its
own parity tests)."""
import sys

import numpy as np
import pytest

from paper_2509_26279_amd import sas, synth

pytestmark = pytest.mark.gpu


def test_wide_pipeline_recovers_movers(gpu):
    wl = synth.make_wide()
    v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8, tuning={"n_det_hint": wl.n})
    try:
        s = sas.Search(plan, wl.n, cand_cap=1 << 22)
        x, y, e = s.upload(wl.x_q8, wl.y_q8, wl.epoch)
        s.vote(x, y, e)
        cells = s.peaks()
        clusters, owner = s.extract(wl.n)
        groups = [np.nonzero(owner == k)[0] for k in range(len(clusters))]
        fits, gathered, _ = s.refine(x, y, e, groups, synth.mcd_starts())
    finally:
        plan.close()
    print("cells", len(cells), "clusters", len(clusters), flush=True)
    sys.stdout.flush()
    assert len(clusters) > 0 and len(fits) == len(clusters)
    # every detection belongs to at most one cluster, and each cluster holds
    # at least N_min distinct epochs of its detections
    for g in groups:
        assert len(np.unique(np.asarray(wl.epoch)[g])) >= wl.n_min
    tr = wl.truth
    ok = fits["status"] == 0
    assert ok.mean() > 0.9
    # a converged fit is a mover's trajectory: its velocity within 1 px/h of
    # the mover its detections mostly belong to
    mid = np.asarray(wl.is_mover)
    good = 0
    for k in np.nonzero(ok)[0]:
        m = mid[gathered[k]]
        m = m[m >= 0]
        if len(m) == 0:
            continue
        mv = np.bincount(m).argmax()
        dv = np.hypot(fits["vx"][k] - tr["vx"][mv], fits["vy"][k] - tr["vy"][mv])
        good += dv < 1.0
    findable = int((tr["present"].sum(axis=1) >= wl.n_min).sum())
    print("recovered", good, "of", findable, "findable movers", flush=True)
    assert good >= 0.8 * findable

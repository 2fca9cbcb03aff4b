"""sas_vote_static (no allocation, static per-GPU scratch) against sas_vote
(caller workspace) through the C ABI: identical candidate lists, record by
record, on consecutive calls whose inputs shrink, so that each call runs on
the scratch contents the previous one left."""
import sys

import numpy as np
import pytest
import torch

from paper_2509_26279_amd import sas, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(plan, x, y, e, cap):
    """(sas_vote list, sas_vote_static list) of one device catalog."""
    s = sas.Search(plan, max(int(x.numel()), 1), cand_cap=cap)
    s.vote(x, y, e)
    ref = s.peaks()
    cand = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    res = torch.zeros(4, dtype=torch.int32, device="cuda")
    sas.vote_static(plan, x, y, e, cand, res)
    got = sas.peaks(cand, res)
    return ref, got


def _same(a, b):
    assert len(a) == len(b), (len(a), len(b))
    for k in ("v_idx", "bx", "by", "count", "flags"):
        assert np.array_equal(a[k], b[k]), k


def test_static_matches_workspace_vote_on_shrinking_inputs(gpu):
    wide = synth.make_wide()
    v = sas.grid_from_spec(wide.grid, wide.binw_q8, wide.span_q16)
    tun = {"n_det_hint": wide.n, "refine_cap": 1 << 20}
    plan = sas.Plan(v, wide.t_q16, wide.binw_q8, wide.n_min, wide.extent_q8, count_sat=255,
                    tuning=tun)
    try:
        need = plan.workspace_size(wide.n)
        assert need <= sas.STATIC_SCRATCH_BYTES, need
        x = torch.as_tensor(wide.x_q8).cuda()
        y = torch.as_tensor(wide.y_q8).cuda()
        e = torch.as_tensor(wide.epoch).cuda()
        # 1: the whole wide catalog over the whole grid
        _say("static vote 1: wide n=%d |V|=%d workspace %d B" % (wide.n, len(v), need))
        ref, got = _both(plan, x, y, e, 1 << 16)
        assert len(ref) > 1000
        _same(ref, got)
        # 2: the same plan on a smaller catalog (the first third of the detections)
        k = wide.n // 3
        _say("static vote 2: wide, first %d detections" % k)
        ref, got = _both(plan, x[:k].contiguous(), y[:k].contiguous(), e[:k].contiguous(),
                         1 << 16)
        _same(ref, got)
    finally:
        plan.close()
    # 3: a smaller catalog with another plan (the tiny workload), on what the
    # wide votes left in the array
    tiny = synth.make_tiny()
    vt = sas.grid_from_spec(tiny.grid, tiny.binw_q8, tiny.span_q16)
    plan = sas.Plan(vt, tiny.t_q16, tiny.binw_q8, tiny.n_min, tiny.extent_q8, count_sat=255)
    try:
        _say("static vote 3: tiny n=%d |V|=%d" % (tiny.n, len(vt)))
        xt = torch.as_tensor(tiny.x_q8).cuda()
        yt = torch.as_tensor(tiny.y_q8).cuda()
        et = torch.as_tensor(tiny.epoch).cuda()
        ref, got = _both(plan, xt, yt, et, 1 << 12)
        assert len(ref) > 0
        _same(ref, got)
    finally:
        plan.close()


def test_static_refuses_plans_beyond_the_maximum(gpu):
    wide = synth.make_wide()
    v = sas.grid_from_spec(wide.grid, wide.binw_q8, wide.span_q16)
    # the default refinement list of this plan alone takes 64 MiB
    plan = sas.Plan(v, wide.t_q16, wide.binw_q8, wide.n_min, wide.extent_q8, count_sat=255,
                    tuning={"n_det_hint": wide.n})
    try:
        assert plan.workspace_size(wide.n) > sas.STATIC_SCRATCH_BYTES
        x = torch.as_tensor(wide.x_q8).cuda()
        y = torch.as_tensor(wide.y_q8).cuda()
        e = torch.as_tensor(wide.epoch).cuda()
        cand = torch.empty((16, 4), dtype=torch.int32, device="cuda")
        res = torch.zeros(4, dtype=torch.int32, device="cuda")
        with pytest.raises(sas.SasError) as ei:
            sas.vote_static(plan, x, y, e, cand, res)
        assert ei.value.status == sas.SAS_E_WORKSPACE
        assert "static maximum" in str(ei.value)
    finally:
        plan.close()

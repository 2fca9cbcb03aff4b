"""GPU parity at the benchmarked sizes.

* The whole candidate lists of the wide and fast workloads (every velocity
  of their grids, every record) against the oracle's lists stored by
  ``tests/golden/make_full_lists.py`` (Sec. 2.1, Steps 1-2 with the Step-3
  threshold).
* Full-size chips of the batched night in one batch, each against its own
  single-chip vote and against the oracle on a velocity sample.
* Coverage pruning (tiles that fewer than N_min epochs can reach are not
  voted): identical lists with and without it, also when the earliest epoch
  of a catalog is empty, so that the reference epoch is a later one.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2509_26279_amd import sas, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location(
    "make_full_lists", os.path.join(HERE, "golden", "make_full_lists.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same(g, o):
    g = np.asarray(g).view(sas.CAND_DTYPE)
    o = np.asarray(o).astype(sas.CAND_DTYPE)
    assert len(g) == len(o), (len(g), len(o))
    for k in ("v_idx", "bx", "by", "count", "flags"):
        bad = np.nonzero(g[k] != o[k])[0]
        assert bad.size == 0, (k, bad[:5], g[bad[:5]], o[bad[:5]])


def _vote(wl, v, n_min, count_sat, tuning=None, x=None, y=None, e=None, cap=1 << 22):
    """Candidate list of one catalog, planned as the benchmark plans it."""
    tun = dict(n_det_hint=wl.n)
    tun.update(tuning or {})
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, n_min, wl.extent_q8, count_sat=count_sat,
                    tuning=tun)
    try:
        s = sas.Search(plan, wl.n, cand_cap=cap)
        if x is None:
            x, y, e = s.upload(wl.x_q8, wl.y_q8, wl.epoch)
        s.vote(x, y, e)
        return s.peaks(), plan.info()
    finally:
        plan.close()


@pytest.mark.parametrize("name", ["wide", "fast"])
def test_whole_grid_list_equals_oracle(gpu, name):
    """Every record of the whole-grid search equals the oracle's stored list."""
    if not os.path.exists(golden.path_of(name)):
        pytest.skip("the oracle's list %s is not written yet (tests/golden/make_full_lists.py)"
                    % os.path.basename(golden.path_of(name)))
    head, ref = golden.read(name)
    wl, v = golden.workload(name)
    assert golden.input_hash(wl, v) == head["input_sha256"], "generator gave other inputs"
    assert int(head["records"]) == len(ref) and golden.records_hash(ref) == head["records_sha256"]
    _say(f"{name} whole grid n={wl.n} |V|={len(v)} stored records {len(ref)}")
    g, info = _vote(wl, v, wl.n_min, golden.SAT[name])
    _say(f"  plan tiles {info['n_tiles']} kept {info['n_tiles_kept']}")
    assert len(ref) > 1000
    assert_same(g, ref)


@pytest.mark.parametrize("name", ["wide", "fast"])
def test_pruning_leaves_whole_lists_unchanged(gpu, name):
    """The same whole-grid search with every tile voted."""
    wl, v = golden.workload(name)
    pruned, info = _vote(wl, v, wl.n_min, golden.SAT[name])
    full, info_full = _vote(wl, v, wl.n_min, golden.SAT[name], tuning=dict(prune=-1))
    _say(f"{name}: tiles {info['n_tiles']}, kept {info['n_tiles_kept']}; "
         f"unpruned plan keeps {info_full['n_tiles_kept']}")
    assert info_full["n_tiles_kept"] == info_full["n_tiles"]
    assert info["n_tiles_kept"] < info["n_tiles"]
    assert_same(pruned, full)


def _drop_first_epoch(wl):
    """The catalog without the detections of its earliest epoch: the
    reference epoch becomes the second one."""
    keep = wl.epoch != np.argmin(wl.t_q16)
    for k in ("x_q8", "y_q8", "epoch", "snr", "is_mover"):
        setattr(wl, k, getattr(wl, k)[keep])
    return wl


def test_pruning_with_a_later_reference_epoch(gpu):
    """Earliest epoch empty: the kept tiles were planned from it, so the
    kernel votes the skipped tiles as well; the list equals the unpruned
    plan's and the oracle's on a velocity sample."""
    wl, v = golden.workload("fast")
    wl = _drop_first_epoch(wl)
    for n_min in (wl.n_min, wl.n_min - 4):
        pruned, info = _vote(wl, v, n_min, 65535)
        full, _ = _vote(wl, v, n_min, 65535, tuning=dict(prune=-1))
        _say(f"fast without epoch 0, n_min {n_min}: {len(pruned)} records")
        assert len(pruned) > 0
        assert_same(pruned, full)
        idx = np.union1d(np.random.default_rng(9).choice(len(v), 48, replace=False),
                         np.unique(pruned["v_idx"])[:: max(1, len(np.unique(pruned["v_idx"])) // 24)])
        o = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[idx], wl.binw_q8, n_min,
                        "epochs", 65535)
        o["v_idx"] = idx[o["v_idx"]]
        assert_same(pruned[np.isin(pruned["v_idx"], idx)], o)


def _night_full_chips(count_per_style):
    """The largest chips of each style of the batched night, at full size,
    with their thresholds set as the night benchmark sets them."""
    params = synth.night_chip_params(4, 64)
    pick = []
    for style in ("fast", "wide"):
        ps = sorted((p for p in params if p["style"] == style), key=lambda p: -p["n_det"])
        pick += ps[:count_per_style]
    chips = []
    for p in pick:
        wl = synth.make_night_chip(p, 0)
        v = golden.ogrid.build_grid(golden.dataclasses.asdict(wl.grid),
                                    golden.ogrid.spacing_q8(wl.binw_q8, wl.span_q16))
        n_min = wl.n_min
        if p["style"] == "fast":  # the threshold rule of Sec. 2.2 for this chip
            area = float(wl.width_px * wl.height_px)
            mu = wl.n / wl.n_epochs * wl.bin_px ** 2 / area
            n_min = sas.threshold_n_min(wl.n_epochs, mu, len(v) * area / wl.bin_px ** 2)
        chips.append((p, wl, v, n_min))
    return chips


def test_night_full_size_batch(gpu):
    """Eight full-size chips (the four largest of each style, fast-style ones
    with their whole 1.23e6-velocity grids) voted in one batch: each chip's
    list equals its single-chip vote, and the oracle's on a velocity sample
    that includes velocities with candidates."""
    import torch
    chips = _night_full_chips(4)
    plans, bound = [], []
    for p, wl, v, n_min in chips:
        plan = sas.Plan(v, wl.t_q16, wl.binw_q8, n_min, wl.extent_q8,
                        tuning=dict(n_det_hint=wl.n))
        x = torch.as_tensor(wl.x_q8).cuda()
        y = torch.as_tensor(wl.y_q8).cuda()
        e = torch.as_tensor(wl.epoch).cuda()
        plans.append(plan)
        bound.append((plan, x, y, e))
    try:
        b = sas.Batch(bound, cand_cap=1 << 21)
        b.vote()
        for k, (p, wl, v, n_min) in enumerate(chips):
            got = b.peaks(k)
            _say(f"night chip {p['chip']} {p['style']} n={wl.n} E={wl.n_epochs} |V|={len(v)} "
                 f"n_min={n_min}: {len(got)} records")
            s = sas.Search(plans[k], wl.n, cand_cap=1 << 21)
            s.vote(*bound[k][1:])
            assert_same(got, s.peaks())
            u = np.unique(got["v_idx"])
            idx = np.union1d(np.random.default_rng(p["chip"]).choice(len(v), 12, replace=False),
                             u[:: max(1, len(u) // 12)])
            o = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[idx], wl.binw_q8, n_min,
                            "epochs", 65535)
            o["v_idx"] = idx[o["v_idx"]]
            assert_same(got[np.isin(got["v_idx"], idx)], o)
        b.close()
    finally:
        for plan in plans:
            plan.close()


def test_batch_with_a_later_reference_epoch(gpu):
    """A batch where one chip's earliest epoch is empty: that chip's skipped
    tiles are voted (the others' are not), and every chip equals its
    unpruned single-chip vote."""
    import torch
    params = [p for p in synth.night_chip_params(4, 64) if p["style"] == "fast"][:2]
    params += [p for p in synth.night_chip_params(4, 64) if p["style"] == "wide"][:1]
    items = []
    for k, p in enumerate(params):
        p = dict(p, n_det=min(p["n_det"], 120000))
        wl = synth.make_night_chip(p, synth.FAST_N_MIN)
        if k == 0:
            wl = _drop_first_epoch(wl)
        v = golden.ogrid.build_grid(golden.dataclasses.asdict(wl.grid),
                                    golden.ogrid.spacing_q8(wl.binw_q8, wl.span_q16))
        items.append((wl, v))
    plans, bound = [], []
    try:
        for wl, v in items:
            plan = sas.Plan(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8,
                            tuning=dict(n_det_hint=wl.n))
            plans.append(plan)
            bound.append((plan, torch.as_tensor(wl.x_q8).cuda(), torch.as_tensor(wl.y_q8).cuda(),
                          torch.as_tensor(wl.epoch).cuda()))
        b = sas.Batch(bound, cand_cap=1 << 21)
        b.vote()
        for k, (wl, v) in enumerate(items):
            got = b.peaks(k)
            full, _ = _vote(wl, v, wl.n_min, 65535, tuning=dict(prune=-1), x=bound[k][1],
                            y=bound[k][2], e=bound[k][3], cap=1 << 21)
            _say(f"batch chip {k} n={wl.n} |V|={len(v)}: {len(got)} records")
            assert len(got) > 0
            assert_same(got, full)
        b.close()
    finally:
        for plan in plans:
            plan.close()


def test_repeated_and_replayed_votes_keep_the_list(gpu):
    """The persistent vote takes its work items by tickets from per-XCD
    queues that the preparation clears on every vote, and most items are
    taken by workgroups of other XCDs once their own range is done.  Votes
    repeated on one workspace, and replays of a captured vote with other
    work between them, each give the oracle's whole wide list."""
    import torch
    if not os.path.exists(golden.path_of("wide")):
        pytest.skip("the oracle's wide list is not written yet (tests/golden/make_full_lists.py)")
    head, ref = golden.read("wide")
    wl, v = golden.workload("wide")
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8,
                    count_sat=golden.SAT["wide"], tuning=dict(n_det_hint=wl.n))
    try:
        info = plan.info()
        _say(f"wide: {info['n_items_kept']} kept items, {info['n_tiles_kept']} kept tiles")
        assert info["n_items_kept"] > 8 * 256  # far more items than resident workgroups
        s = sas.Search(plan, wl.n, cand_cap=1 << 22)
        x, y, e = s.upload(wl.x_q8, wl.y_q8, wl.epoch)
        for rep in range(3):
            _say(f"eager vote {rep}")
            s.vote(x, y, e)
            assert_same(s.peaks(), ref)
        stream = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            s.vote(x, y, e, stream=torch.cuda.current_stream())
        for rep in range(3):
            _say(f"graph replay {rep}")
            s.res.fill_(-1)  # eager work between replays
            s.cand.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert_same(s.peaks(), ref)
    finally:
        plan.close()

"""Weighted votes on the GPU (sas_vote_weighted) against the oracle's
weighted counts, element by element and bit-exact: weighted epochs (the
largest weight per epoch, summed) and weighted detections (the sum of the
weights), single bins and coarse cells with refinement, every lane-group
count, chunked stages, full-size catalogs; and the entry points that refuse
weighted plans."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from oracle import grid as ogrid
from paper_2509_26279_amd import sas, synth

pytestmark = pytest.mark.gpu

MODES = ("weighted_epochs", "weighted_detections")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _extent(x, y):
    return (int(np.min(x)), int(np.max(x)) + 1, int(np.min(y)), int(np.max(y)) + 1)


def _grid(wl):
    return ogrid.build_grid(dataclasses.asdict(wl.grid), ogrid.spacing_q8(wl.binw_q8, wl.span_q16))


def gpu_vote(x, y, e, w, t, v, binw, n_min, mode, count_sat=65535, extent=None, tuning=None,
             cap=1 << 18):
    extent = extent if extent is not None else _extent(x, y)
    plan = sas.Plan(v, t, binw, n_min, extent, mode=mode, count_sat=count_sat, tuning=tuning)
    try:
        s = sas.Search(plan, max(len(x), 1), cand_cap=cap)
        return s.run(x, y, e, weight=w), plan.info()
    finally:
        plan.close()


def assert_same(g, o):
    g = np.asarray(g).view(sas.CAND_DTYPE)
    o = np.asarray(o).astype(sas.CAND_DTYPE)
    assert len(g) == len(o), (len(g), len(o))
    for k in ("v_idx", "bx", "by", "count", "flags"):
        bad = np.nonzero(g[k] != o[k])[0]
        assert bad.size == 0, (k, bad[:5], g[bad[:5]], o[bad[:5]])


def _snr_weights(snr, scale=4.0):
    """A quantised detection likelihood: round(scale * SNR^2 / 2), capped at 255."""
    return np.minimum(np.rint(scale * np.asarray(snr, np.float64) ** 2 / 2.0), 255).astype(np.uint8)


@pytest.mark.parametrize("mode", MODES)
def test_tiny_every_shape(gpu, mode):
    wl = synth.make_tiny()
    v = _grid(wl)
    w = np.random.default_rng(3).integers(0, 256, wl.n).astype(np.uint8)
    n_min = 12 * 128
    o = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8, n_min, mode, weight=w)
    assert len(o) > 0
    for tun in (None, dict(groups=1), dict(groups=2), dict(groups=4),
                dict(coarse_log2=1), dict(coarse_log2=2, groups=4), dict(coarse_log2=3),
                dict(stage_cap=16, groups=2), dict(tile_x=5, tile_y=3, groups=1)):
        _say(f"weighted tiny mode={mode} tuning={tun}")
        g, info = gpu_vote(wl.x_q8, wl.y_q8, wl.epoch, w, wl.t_q16, v, wl.binw_q8, n_min, mode,
                           extent=wl.extent_q8, tuning=tun)
        assert info["packed"] == 0
        assert info["mode_variant"] == (3 if mode == "weighted_detections" and
                                        not (tun or {}).get("coarse_log2") else 4)
        assert_same(g, o)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("mode", MODES)
def test_adversarial(gpu, seed, mode):
    d = synth.make_random_small(seed, n=300, n_epochs=[5, 20, 40, 64, 100, 200, 3, 33][seed],
                                n_v=30, binw_q8=[256, 512, 1024, 2048][seed % 4],
                                extent_q8=50 * 256, dup_frac=0.3)
    w = np.random.default_rng(50 + seed).integers(0, [2, 4, 256][seed % 3],
                                                  len(d["x_q8"])).astype(np.uint8)
    for n_min in (1, 3, 40, 300):
        for tun in (None, dict(groups=2, stage_cap=16), dict(coarse_log2=2, groups=4)):
            sat = 255 if (seed + n_min) % 2 else 65535
            _say(f"weighted adversarial seed={seed} mode={mode} n_min={n_min} tuning={tun}")
            o = oracle.vote(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"],
                            d["binw_q8"], n_min, mode, count_sat=sat, weight=w)
            g, _ = gpu_vote(d["x_q8"], d["y_q8"], d["epoch"], w, d["t_q16"], d["v_q8"],
                            d["binw_q8"], n_min, mode, count_sat=sat, tuning=tun)
            assert_same(g, o)


@pytest.mark.parametrize("maker,k", [(synth.make_wide, 200), (synth.make_fast, 160)])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("hint", [False, True])
def test_full_catalog_velocity_subset(gpu, maker, k, mode, hint):
    """The workload's whole catalog, weights from its detections' SNR, against
    a seeded subset of its grid, at two thresholds; single bins, or the
    coarse cells the weight hint lets the planner choose."""
    wl = maker()
    v = _grid(wl)
    w = _snr_weights(wl.snr)
    idx = np.sort(np.random.default_rng(41).choice(len(v), size=min(k, len(v)), replace=False))
    mean_w = float(w.mean())
    tun = dict(n_det_hint=wl.n)
    if hint:
        tun["weight_hint"] = int(round(mean_w))
    for n_min in (int(wl.n_min * mean_w), int(0.4 * wl.n_min * mean_w)):
        _say(f"weighted {wl.name} |V|={len(idx)} mode={mode} n_min={n_min} tuning={tun}")
        o = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[idx], wl.binw_q8, n_min, mode,
                        weight=w)
        g, info = gpu_vote(wl.x_q8, wl.y_q8, wl.epoch, w, wl.t_q16, v[idx], wl.binw_q8, n_min,
                           mode, extent=wl.extent_q8, tuning=tun, cap=1 << 22)
        _say(f"  coarse_log2={info['coarse_log2']} mode_variant={info['mode_variant']}")
        assert len(o) > 0
        assert_same(g, o)


def test_wide_full_grid_sampled_outputs(gpu):
    """The whole wide grid with SNR weights (the configuration the weighted
    benchmark line times): a seeded velocity sample checked one by one."""
    wl = synth.make_wide()
    v = _grid(wl)
    w = _snr_weights(wl.snr)
    n_min = int(wl.n_min * float(w.mean()))
    _say(f"weighted wide full grid |V|={len(v)} n_min={n_min}")
    g, info = gpu_vote(wl.x_q8, wl.y_q8, wl.epoch, w, wl.t_q16, v, wl.binw_q8, n_min,
                       "weighted_epochs", extent=wl.extent_q8,
                       tuning=dict(n_det_hint=wl.n, weight_hint=int(round(float(w.mean())))),
                       cap=1 << 22)
    assert info["coarse_log2"] > 0  # the sparse wide catalog takes coarse cells
    assert len(g) > 0 and np.all(g["count"] >= n_min)
    idx = np.sort(np.random.default_rng(23).choice(len(v), size=64, replace=False))
    idx = np.union1d(idx, np.unique(g["v_idx"])[:: max(1, len(np.unique(g["v_idx"])) // 32)])
    o = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[idx], wl.binw_q8, n_min,
                    "weighted_epochs", weight=w)
    o["v_idx"] = idx[o["v_idx"]]
    assert_same(g[np.isin(g["v_idx"], idx)], o)


def test_unit_weights_match_indicator_votes(gpu):
    """All weights 1: the weighted votes equal the indicator votes."""
    d = synth.make_random_small(11, n=400, n_epochs=48, n_v=40, binw_q8=1024, dup_frac=0.3)
    ones = np.ones(len(d["x_q8"]), np.uint8)
    for mode, plain in (("weighted_epochs", "epochs"), ("weighted_detections", "detections")):
        plan = sas.Plan(d["v_q8"], d["t_q16"], d["binw_q8"], 2,
                        _extent(d["x_q8"], d["y_q8"]), mode=plain)
        try:
            ref = sas.Search(plan, len(ones)).run(d["x_q8"], d["y_q8"], d["epoch"])
        finally:
            plan.close()
        g, _ = gpu_vote(d["x_q8"], d["y_q8"], d["epoch"], ones, d["t_q16"], d["v_q8"],
                        d["binw_q8"], 2, mode)
        assert_same(g, ref)


def test_empty_and_zero_weights(gpu):
    t = np.arange(4, dtype=np.int64) * 1000
    ext = (0, 1 << 16, 0, 1 << 16)
    z = np.zeros(0, np.int32)
    g, _ = gpu_vote(z, z, np.zeros(0, np.uint8), np.zeros(0, np.uint8), t,
                    np.zeros((3, 2), np.int32), 1024, 1, "weighted_epochs", extent=ext)
    assert len(g) == 0
    x = np.array([5, 6, 7], np.int32)
    g, _ = gpu_vote(x, x, np.array([0, 1, 2], np.uint8), np.zeros(3, np.uint8), t,
                    np.zeros((3, 2), np.int32), 1024, 1, "weighted_detections", extent=ext)
    assert len(g) == 0


def test_entry_points_check_the_mode(gpu):
    import torch
    d = synth.make_random_small(1, n=50, n_epochs=4, n_v=5, binw_q8=1024)
    ext = _extent(d["x_q8"], d["y_q8"])
    wplan = sas.Plan(d["v_q8"], d["t_q16"], 1024, 2, ext, mode="weighted_epochs")
    plan = sas.Plan(d["v_q8"], d["t_q16"], 1024, 2, ext)
    try:
        s = sas.Search(wplan, 64)
        x, y, e, w = s.upload(d["x_q8"], d["y_q8"], d["epoch"], np.ones(50, np.uint8))
        with pytest.raises(sas.SasError) as ei:  # indicator entry point, weighted plan
            sas.vote(wplan, x, y, e, s.cand, s.res, s.ws)
        assert ei.value.status == sas.SAS_E_INVALID
        s2 = sas.Search(plan, 64)
        with pytest.raises(sas.SasError) as ei:  # weighted entry point, indicator plan
            sas.vote(plan, x, y, e, s2.cand, s2.res, s2.ws, weight=w)
        assert ei.value.status == sas.SAS_E_INVALID
        with pytest.raises(sas.SasError) as ei:  # batches take indicator plans only
            sas.Batch([(wplan, x, y, e)])
        assert ei.value.status == sas.SAS_E_UNSUPPORTED
        s.vote(x, y, e, w)
        s.peaks()
        with pytest.raises(sas.SasError) as ei:  # so does the greedy extraction
            s.extract(50)
        assert ei.value.status == sas.SAS_E_UNSUPPORTED
        with pytest.raises(sas.SasError) as ei:  # and the vetting features
            s.features(50)
        assert ei.value.status == sas.SAS_E_UNSUPPORTED
        torch.cuda.synchronize()
    finally:
        wplan.close()
        plan.close()

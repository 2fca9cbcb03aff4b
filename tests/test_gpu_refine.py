"""Steps 4-6 on the GPU (sas_refine_clusters) against the oracle
(oracle/refine.py): per cluster the status, the rounds, the MCD subset and
the gathered set must be identical; the regression (velocity, position at
t0) within 1e-9 and the error covariance within 1e-6, relative (FP64 on both
sides, sums in different orders).  Cluster inputs come from the oracle's
Step-3 extraction or from the generator's truth."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from oracle import extract as ox
from oracle import grid as ogrid
from oracle import refine as R
from paper_2509_26279_amd import sas, synth

pytestmark = pytest.mark.gpu

STARTS = synth.mcd_starts(7, 500)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _extent(x, y):
    return (int(np.min(x)), int(np.max(x)) + 1, int(np.min(y)), int(np.max(y)) + 1)


def gpu_refine(x, y, e, t, v, b, n_min, clusters, starts=STARTS, radius_q8=0, mode="epochs",
               extent=None, weight=None, gather_cap=512):
    extent = extent if extent is not None else _extent(x, y)
    plan = sas.Plan(v, t, b, n_min, extent, mode=mode)
    try:
        s = sas.Search(plan, max(len(x), 1), cand_cap=1 << 20)
        dev = s.upload(x, y, e, weight)
        s.vote(*dev)
        s.peaks()
        return s.refine(dev[0], dev[1], dev[2], clusters, starts, radius_q8,
                        gather_cap=gather_cap)
    finally:
        plan.close()


def check(got, x, y, e, t, clusters, dx_px, starts=STARTS):
    recs, gath, subs = got
    n_conv = 0
    for i, cl in enumerate(clusters):
        o = R.refine_cluster(x, y, e, t, cl, starts, dx_px)
        r = recs[i]
        assert int(r["status"]) == o["status"], (i, r, o["status"])
        assert int(r["rounds"]) == o["rounds"], (i, r, o["rounds"])
        n_conv += o["status"] == R.STATUS_CONVERGED
        if o["rounds"] == 0:
            continue
        assert np.array_equal(subs[i], o["subset"]), i
        assert int(r["n_points"]) == len(o["subset"])
        assert int(r["n_gathered"]) == len(o["gathered"])
        assert np.array_equal(gath[i], o["gathered"]), i
        got_bc = np.array([r["vx"], r["vy"], r["x0"], r["y0"]])
        want_bc = np.concatenate([o["B"], o["c"]])
        assert np.allclose(got_bc, want_bc, rtol=1e-9, atol=1e-9), (i, got_bc, want_bc)
        got_s = np.array([r["sxx"], r["sxy"], r["syy"]])
        want_s = np.array([o["sigma"][0, 0], o["sigma"][0, 1], o["sigma"][1, 1]])
        assert np.allclose(got_s, want_s, rtol=1e-6, atol=1e-9), (i, got_s, want_s)
    return n_conv


def _grid(wl):
    return ogrid.build_grid(dataclasses.asdict(wl.grid), ogrid.spacing_q8(wl.binw_q8, wl.span_q16))


def test_tiny_extracted_clusters(gpu):
    """The clusters of Step 3 (oracle extraction) of the tiny workload."""
    wl = synth.make_tiny()
    v = _grid(wl)
    n_min = 8
    cand = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8, n_min)
    clusters = [c[4] for c in ox.extract(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8,
                                         cand, n_min)]
    _say(f"refine tiny: {len(clusters)} clusters")
    got = gpu_refine(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8, n_min, clusters,
                     extent=wl.extent_q8)
    assert check(got, wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, clusters, wl.binw_q8 / 256.0) > 0


def _movers_in_noise(seed, n_movers=12, E=40, n_noise=6000, outlier_frac=0.3, size=800.0):
    rng = np.random.default_rng(seed)
    t_q16 = (np.arange(E) * (4 * 65536) // (E - 1)).astype(np.int64) + 777
    th = (t_q16 - t_q16[0]) / 65536.0
    xs, ys, es, clusters = [], [], [], []
    k = 0
    for m in range(n_movers):
        vx, vy = rng.uniform(-40, 40, 2)
        x0, y0 = rng.uniform(150, size - 150, 2)
        on = rng.uniform(size=E) < rng.uniform(0.5, 1.0)
        ee = np.nonzero(on)[0]
        xs.append(x0 + vx * th[ee] + rng.normal(0, 0.5, len(ee)))
        ys.append(y0 + vy * th[ee] + rng.normal(0, 0.5, len(ee)))
        es.append(ee)
        clusters.append(list(range(k, k + len(ee))))
        k += len(ee)
    nx, ny = rng.uniform(0, size, n_noise), rng.uniform(0, size, n_noise)
    ne = rng.integers(0, E, n_noise)
    x = np.floor(256 * np.concatenate(xs + [nx])).astype(np.int32)
    y = np.floor(256 * np.concatenate(ys + [ny])).astype(np.int32)
    e = np.concatenate(es + [ne]).astype(np.uint8)
    # each cluster: the mover's detections and noise points around its track
    out = []
    for m, cl in enumerate(clusters):
        cx, cy = x[cl].mean() / 256, y[cl].mean() / 256
        near = np.nonzero((np.abs(nx - cx) < 60) & (np.abs(ny - cy) < 60))[0] + k
        take = near[: int(outlier_frac * len(cl))]
        out.append(np.concatenate([np.asarray(cl), take]))
    return x, y, e, t_q16, out


@pytest.mark.parametrize("seed,frac", [(1, 0.0), (2, 0.3), (3, 0.6), (4, 0.9)])
def test_movers_with_outliers(gpu, seed, frac):
    x, y, e, t, clusters = _movers_in_noise(seed, outlier_frac=frac)
    v = np.array([[0, 0]], np.int32)
    _say(f"refine movers seed={seed} outliers={frac}: {len(clusters)} clusters")
    got = gpu_refine(x, y, e, t, v, 1024, 3, clusters, extent=(0, 800 * 256, 0, 800 * 256))
    assert check(got, x, y, e, t, clusters, 4.0) > 0


def test_wide_movers(gpu):
    """Clusters of the wide workload built from its truth: 40 movers'
    detections with noise around each, refined against the whole catalog."""
    wl = synth.make_wide()
    v = _grid(wl)[:64]
    mid = np.asarray(wl.is_mover)
    rng = np.random.default_rng(5)
    noise = np.nonzero(mid < 0)[0]
    clusters = []
    for m in range(0, 200, 5):
        cl = np.nonzero(mid == m)[0]
        if len(cl) < 5:
            continue
        cx, cy = wl.x_q8[cl].mean(), wl.y_q8[cl].mean()
        near = noise[(np.abs(wl.x_q8[noise] - cx) < 64 * 256) &
                     (np.abs(wl.y_q8[noise] - cy) < 64 * 256)]
        clusters.append(np.concatenate([cl, rng.permutation(near)[: len(cl) // 3]]))
    _say(f"refine wide: {len(clusters)} clusters")
    got = gpu_refine(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8, wl.n_min, clusters,
                     extent=wl.extent_q8)
    assert check(got, wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, clusters, wl.binw_q8 / 256.0) > 0


def test_radius_weighted_plan_and_few_starts(gpu):
    """A given gather radius, a weighted plan's index (256 x + w) and 3 starts."""
    x, y, e, t, clusters = _movers_in_noise(6, n_movers=6, outlier_frac=0.2)
    v = np.array([[0, 0]], np.int32)
    w = np.random.default_rng(1).integers(0, 256, len(x)).astype(np.uint8)
    st = STARTS[:3]
    got = gpu_refine(x, y, e, t, v, 1024, 300, clusters, starts=st, radius_q8=3 * 256,
                     mode="weighted_epochs", weight=w, extent=(0, 800 * 256, 0, 800 * 256))
    check(got, x, y, e, t, clusters, 3.0, starts=st)


def test_edge_cases(gpu):
    x, y, e, t, clusters = _movers_in_noise(7, n_movers=3)
    v = np.array([[0, 0]], np.int32)
    n = len(x)
    cases = [clusters[0][:4],                 # too small from the start
             np.arange(600),                   # more points than a set holds
             np.array([0, 1, 2, n, 3, 4]),     # a member outside the catalog
             clusters[1]]
    recs, gath, subs = gpu_refine(x, y, e, t, v, 1024, 3, cases,
                                  extent=(0, 800 * 256, 0, 800 * 256))
    assert int(recs[0]["status"]) == sas_status("too_small") and int(recs[0]["rounds"]) == 0
    assert int(recs[1]["status"]) == sas_status("too_large")
    assert int(recs[2]["status"]) == sas_status("bad_input")
    check((recs[3:], gath[3:], subs[3:]), x, y, e, t, [clusters[1]], 4.0)
    # every start repeats a point: no fit
    recs, _, _ = gpu_refine(x, y, e, t, v, 1024, 3, [clusters[2]],
                            starts=np.zeros((4, 4), np.uint32),
                            extent=(0, 800 * 256, 0, 800 * 256))
    assert int(recs[0]["status"]) == sas_status("no_start") and int(recs[0]["rounds"]) == 0


def sas_status(name):
    return {v: k for k, v in sas.REFINE_STATUS.items()}[name]


def test_gather_capacity_truncates(gpu):
    """A gather capacity below the gathered set: the true count is reported
    and the first entries (ascending) are written."""
    x, y, e, t, clusters = _movers_in_noise(8, n_movers=4, outlier_frac=0.2)
    v = np.array([[0, 0]], np.int32)
    ext = (0, 800 * 256, 0, 800 * 256)
    full = gpu_refine(x, y, e, t, v, 1024, 3, clusters, extent=ext)
    cut = gpu_refine(x, y, e, t, v, 1024, 3, clusters, extent=ext, gather_cap=4)
    for a, b, ga, gb in zip(full[0], cut[0], full[1], cut[1]):
        assert int(a["n_gathered"]) == int(b["n_gathered"])
        assert np.array_equal(gb, ga[:4])

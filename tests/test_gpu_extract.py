"""Step-3 greedy cluster extraction on the GPU (sas_extract_clusters) against
the oracle's loop: the clusters in extraction order (velocity, bin, count)
and the cluster of every detection must be identical."""
import sys

import numpy as np
import pytest

import oracle
from oracle import extract as ox
from oracle import grid as ogrid
from paper_2509_26279_amd import sas, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _extent(x, y):
    return (int(np.min(x)), int(np.max(x)) + 1, int(np.min(y)), int(np.max(y)) + 1)


def _run(x, y, e, t, v, b, n_min, mode="epochs", extent=None, tuning=None, member_cap=0,
         rounds=0):
    x, y, e = np.asarray(x), np.asarray(y), np.asarray(e)
    extent = extent if extent is not None else _extent(x, y)
    plan = sas.Plan(v, t, b, n_min, extent, mode=mode, count_sat=65535, tuning=tuning)
    try:
        s = sas.Search(plan, max(len(x), 1), cand_cap=1 << 18)
        xd, yd, ed = s.upload(x, y, e)
        s.vote(xd, yd, ed)
        s.peaks()
        return s.extract(len(x), member_cap=member_cap, rounds=rounds)
    finally:
        plan.close()


def _check(got, ref, n):
    clusters, owner = got
    g = [(int(c["v_idx"]), int(c["bx"]), int(c["by"]), int(c["count"])) for c in clusters]
    assert g == [(r[0], r[1], r[2], r[3]) for r in ref], (g[:5], [r[:4] for r in ref[:5]])
    want = np.full(n, -1, dtype=np.int32)
    for i, r in enumerate(ref):
        want[r[4]] = i
    bad = np.nonzero(owner != want)[0]
    assert bad.size == 0, (bad[:5], owner[bad[:5]], want[bad[:5]])


def _case(x, y, e, t, v, b, n_min, mode="epochs", extent=None, tuning=None, member_cap=0,
          rounds=(0, -1, 1, 3)):
    """The oracle's loop against the GPU with parallel rounds (default, a
    few) and without (one take at a time): identical results."""
    cand = oracle.vote(x, y, e, t, v, b, n_min, mode)
    ref = ox.extract(x, y, e, t, v, b, cand, n_min, mode)
    for r in rounds:
        got = _run(x, y, e, t, v, b, n_min, mode, extent, tuning, member_cap, r)
        _check(got, ref, len(x))
    return ref


def _grid(wl):
    import dataclasses
    return ogrid.build_grid(dataclasses.asdict(wl.grid), ogrid.spacing_q8(wl.binw_q8, wl.span_q16))


@pytest.mark.parametrize("n_min", [12, 5])
def test_extract_tiny(gpu, n_min):
    wl = synth.make_tiny()
    v = _grid(wl)
    _say(f"extract tiny n_min={n_min}")
    ref = _case(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8, n_min, extent=wl.extent_q8)
    assert len(ref) > 0


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mode", ["epochs", "detections"])
def test_extract_adversarial(gpu, seed, mode):
    d = synth.make_random_small(seed, n=300, n_epochs=[5, 20, 40, 64, 100, 200][seed], n_v=30,
                                binw_q8=[256, 512, 1024, 2048][seed % 4],
                                extent_q8=50 * 256, dup_frac=0.3)
    for n_min in (1, 2, 3):
        for tun in (None, dict(packed=-1, groups=2)):
            _say(f"extract adversarial seed={seed} mode={mode} n_min={n_min} tuning={tun}")
            _case(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"], n_min,
                  mode, tuning=tun)


@pytest.mark.parametrize("maker,k,n_mins", [(synth.make_wide, 600, (25, 12)),
                                            (synth.make_fast, 1000, (16, 12))])
def test_extract_full_catalog_velocity_subset(gpu, maker, k, n_mins):
    """The workload's whole catalog against a seeded subset of its grid."""
    wl = maker()
    v = _grid(wl)
    idx = np.sort(np.random.default_rng(23).choice(len(v), size=min(k, len(v)), replace=False))
    for n_min in n_mins:
        _say(f"extract {wl.name} |V|={len(idx)} n_min={n_min}")
        ref = _case(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[idx], wl.binw_q8, n_min,
                    extent=wl.extent_q8, tuning=dict(n_det_hint=wl.n))
        assert len(ref) > 0


def test_extract_member_lists_regrown(gpu):
    """A contributor capacity far too small is reported and the binding
    retries with the reported size; the result is unchanged."""
    d = synth.make_random_small(2, n=200, n_epochs=8, n_v=20, binw_q8=1024, dup_frac=0.3)
    _case(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"], 2,
          member_cap=1)


def test_extract_nothing_to_take(gpu):
    """No cell reaches N_min: no cluster, every detection unclaimed."""
    d = synth.make_random_small(4, n=50, n_epochs=6, n_v=5, binw_q8=1024)
    clusters, owner = _run(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"],
                           d["binw_q8"], 7)
    assert len(clusters) == 0 and np.all(owner == -1)


def test_extract_refuses_a_failed_vote(gpu):
    """Extraction and features run only on a complete candidate list: a
    catalog error or an overfull candidate buffer from the vote is raised,
    as sas_peaks would."""
    wl = synth.make_tiny()
    v = _grid(wl)
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, 5, wl.extent_q8)
    try:
        s = sas.Search(plan, wl.n, cand_cap=1 << 16)
        x = wl.x_q8.copy()
        x[3] = wl.extent_q8[1] + 4096  # outside the footprint
        s.vote(*s.upload(x, wl.y_q8, wl.epoch))
        for call in (lambda: s.extract(wl.n), lambda: s.features(wl.n)):
            with pytest.raises(sas.SasError) as ei:
                call()
            assert ei.value.status == sas.SAS_E_INVALID
        small = sas.Search(plan, wl.n, cand_cap=2)
        small.vote(*small.upload(wl.x_q8, wl.y_q8, wl.epoch))
        assert small.result()["n_cand"] > 2
        with pytest.raises(sas.SasError) as ei:
            small.extract(wl.n)
        assert ei.value.status == sas.SAS_E_OVERFLOW
    finally:
        plan.close()


def test_extract_cluster_capacity_reported(gpu):
    """Fewer output slots than clusters: the call reports the true number
    (SAS_EXTRACT_CLUSTERS_FULL) and the binding raises with it."""
    wl = synth.make_tiny()
    v = _grid(wl)
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, 5, wl.extent_q8)
    try:
        s = sas.Search(plan, wl.n, cand_cap=1 << 16)
        s.vote(*s.upload(wl.x_q8, wl.y_q8, wl.epoch))
        s.peaks()
        full, _ = s.extract(wl.n)
        assert len(full) > 1
        with pytest.raises(sas.SasError) as ei:
            s.extract(wl.n, cluster_cap=1)
        assert ei.value.status == sas.SAS_E_OVERFLOW and str(len(full)) in str(ei.value)
    finally:
        plan.close()

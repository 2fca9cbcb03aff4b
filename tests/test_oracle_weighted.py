"""Pins of the oracle's weighted counts (a per-detection weight accumulated
in place of the detection indicator, as the Conclusions suggest): a worked
example by hand, exact rational brute force, the unit-weight special case
(EPOCHS and DETECTIONS), library histograms at v = 0, conservation, scaling
and ordering invariants."""
import dataclasses
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute, grid
from paper_2509_26279_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(c):
    return [tuple(int(v) for v in r) for r in c.tolist()]


def _weights(seed, n, hi=256):
    return np.random.default_rng(1000 + seed).integers(0, hi, n).astype(np.uint8)


def test_hand_example(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "weighted_example.json")))
    args = (g["x_q8"], g["y_q8"], g["epoch"], g["t_q16"], g["v_q8"], g["binw_q8"])
    w = np.array(g["weight"])
    exp = g["expected"]
    for key, n_min, mode, sat in [("weighted_epochs_nmin12", 12, "weighted_epochs", 65535),
                                  ("weighted_epochs_nmin13", 13, "weighted_epochs", 65535),
                                  ("weighted_detections_nmin15", 15, "weighted_detections", 65535),
                                  ("weighted_detections_nmin16", 16, "weighted_detections", 65535),
                                  ("weighted_epochs_nmin12_sat100", 12, "weighted_epochs", 100)]:
        want = [tuple(r) for r in exp[key]]
        assert _rows(oracle.vote(*args, n_min, mode, count_sat=sat, weight=w)) == want, key
        assert brute.brute_vote(*args, n_min, mode, count_sat=sat, weight=w) == want, key


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("mode", ["weighted_epochs", "weighted_detections"])
def test_brute_force_agrees(oracle_lib, seed, mode):
    d = synth.make_random_small(seed, n=50 + 7 * seed, n_epochs=3 + seed % 6,
                                binw_q8=(1 + seed % 5) * 256 + seed * 13, dup_frac=0.3)
    w = _weights(seed, len(d["x_q8"]), hi=[2, 4, 256][seed % 3])
    for n_min in (1, 3, 40, 300):
        sat = 255 if seed % 2 else 65535
        a = oracle.vote(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"],
                        n_min, mode, count_sat=sat, weight=w)
        b = brute.brute_vote(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"],
                             d["binw_q8"], n_min, mode, count_sat=sat, weight=w)
        assert _rows(a) == b


@pytest.mark.parametrize("mode,plain", [("weighted_epochs", "epochs"),
                                        ("weighted_detections", "detections")])
def test_unit_weights_are_the_indicator(oracle_lib, mode, plain):
    d = synth.make_random_small(5, n=400, n_epochs=12, n_v=40, dup_frac=0.3)
    ones = np.ones(len(d["x_q8"]), np.uint8)
    for n_min in (1, 2, 4):
        a = oracle.vote(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"],
                        n_min, mode, weight=ones)
        b = oracle.vote(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"],
                        n_min, plain)
        assert np.array_equal(a, b)


def test_zero_velocity_library_histograms(oracle_lib):
    rng = np.random.default_rng(17)
    n, b = 6000, 1024
    x = rng.integers(0, 40 * b, n).astype(np.int32)
    y = rng.integers(0, 30 * b, n).astype(np.int32)
    e = rng.integers(0, 7, n).astype(np.uint8)
    w = rng.integers(0, 256, n).astype(np.uint8)
    t = np.arange(7, dtype=np.int64) * 30000 - 5
    # weighted detections: numpy's weighted 2-D histogram
    h, out = oracle.histogram(x, y, e, t, 0, 0, b, "weighted_detections", 0, 0, 40, 30,
                              weight=w)
    ref, _, _ = np.histogram2d(y, x, bins=[np.arange(31) * b, np.arange(41) * b], weights=w)
    assert out == 0 and np.array_equal(h, ref.astype(np.int64))
    # weighted epochs: the largest weight per (bin, epoch) by np.maximum.at, summed
    he, _ = oracle.histogram(x, y, e, t, 0, 0, b, "weighted_epochs", 0, 0, 40, 30, weight=w)
    best = np.zeros((30, 40, 7), np.int64)
    np.maximum.at(best, (y // b, x // b, e.astype(np.int64)), w.astype(np.int64))
    assert np.array_equal(he, best.sum(axis=2))
    # and the vote reports exactly the bins of those histograms at a threshold
    for mode, hist in (("weighted_detections", h), ("weighted_epochs", he)):
        c = oracle.vote(x, y, e, t, [[0, 0]], b, 300, mode, weight=w)
        iy, ix = np.nonzero(hist >= 300)
        assert _rows(c) == [(0, int(bx), int(by), int(hist[by, bx]), 0)
                            for by, bx in sorted(zip(iy, ix))]


def test_weights_are_conserved(oracle_lib):
    wl = synth.make_tiny()
    g = grid.build_grid(dataclasses.asdict(wl.grid), grid.spacing_q8(wl.binw_q8, wl.span_q16))
    w = _weights(3, wl.n)
    w[w == 0] = 1  # every detection's bin is then reported at N_min = 1
    c = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, g, wl.binw_q8, 1,
                    "weighted_detections", weight=w)
    sums = np.bincount(c["v_idx"], weights=c["count"], minlength=len(g))
    assert np.all(sums == int(w.astype(np.int64).sum()))


def test_ordering_and_scaling(oracle_lib):
    d = synth.make_random_small(8, n=300, n_epochs=6, n_v=25, dup_frac=0.4)
    args = (d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"])
    w = _weights(8, len(d["x_q8"]), hi=60)
    we = oracle.vote(*args, 1, "weighted_epochs", weight=w + 1)
    wd = oracle.vote(*args, 1, "weighted_detections", weight=w + 1)
    ep = oracle.vote(*args, 1, "epochs")
    # all weights >= 1: the same bins; EPOCHS <= WEIGHTED_EPOCHS <= WEIGHTED_DETECTIONS
    assert np.array_equal(we[["v_idx", "bx", "by"]], ep[["v_idx", "bx", "by"]])
    assert np.array_equal(wd[["v_idx", "bx", "by"]], ep[["v_idx", "bx", "by"]])
    assert np.all(ep["count"] <= we["count"]) and np.all(we["count"] <= wd["count"])
    assert np.any(we["count"] < wd["count"])  # two detections of one epoch in a bin do show
    # scaling every weight by 4 scales every score by 4 (and the threshold with it)
    for mode in ("weighted_epochs", "weighted_detections"):
        a = oracle.vote(*args, 37, mode, weight=w)
        b = oracle.vote(*args, 4 * 37, mode, weight=4 * w)
        assert np.array_equal(a[["v_idx", "bx", "by"]], b[["v_idx", "bx", "by"]])
        assert np.array_equal(4 * a["count"].astype(np.int64), b["count"].astype(np.int64))
    # all weights 0: nothing reaches N_min = 1
    z = np.zeros(len(w), np.uint8)
    assert len(oracle.vote(*args, 1, "weighted_epochs", weight=z)) == 0


def test_weights_checked(oracle_lib):
    with pytest.raises(ValueError):
        oracle.vote([0], [0], [0], [0], [[0, 0]], 256, 1, "weighted_epochs")
    with pytest.raises(ValueError):
        oracle.vote([0], [0], [0], [0], [[0, 0]], 256, 1, "epochs", weight=[1])
    with pytest.raises(ValueError):
        oracle.vote([0], [0], [0], [0], [[0, 0]], 256, 1, "weighted_epochs", weight=[300])

"""Pins of the FP64 feature and label oracle (oracle/features.py) against a
hand-derived example and properties that hold by construction."""
import json
import os

import numpy as np
import pytest

from oracle import CAND_DTYPE
from oracle import features as of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "features_example.json")


def _cand(v_idx, bx, by):
    c = np.zeros(1, CAND_DTYPE)
    c["v_idx"], c["bx"], c["by"] = v_idx, bx, by
    return c


def test_hand_example():
    g = json.load(open(GOLDEN))
    c = g["candidate"]
    f = of.candidate_features(g["x_q8"], g["y_q8"], g["epoch"], g["snr"], g["t_q16"],
                              g["v_q8"], g["binw_q8"], _cand(c["v_idx"], c["bx"], c["by"]),
                              g["vmax_q8"])
    assert f.shape == (1, of.N_FEATURES)
    np.testing.assert_allclose(f[0], g["features"], rtol=0, atol=1e-12)


def _random_case(seed, n=300, E=12, nv=5, b=1024):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 40 * 256, n).astype(np.int32)
    y = rng.integers(0, 40 * 256, n).astype(np.int32)
    e = rng.integers(0, E, n).astype(np.uint8)
    snr = (3 + np.abs(rng.normal(size=n))).astype(np.float32)
    t = np.sort(rng.integers(0, 4 * 65536, E)).astype(np.int64)
    v = rng.integers(-600, 600, (nv, 2)).astype(np.int32)
    return x, y, e, snr, t, v, b


def _some_candidates(x, y, e, t, v, b, k=12, seed=0):
    """Bins that actually hold detections (the candidate definition is any bin)."""
    rng = np.random.default_rng(seed)
    d = of.reference_dt(t, e, len(t))
    out = np.zeros(k, CAND_DTYPE)
    for j in range(k):
        i = rng.integers(0, len(x))
        vi = rng.integers(0, len(v))
        di = int(d[e[i]])
        out[j]["v_idx"] = vi
        out[j]["bx"] = (65536 * int(x[i]) - int(v[vi, 0]) * di) // (65536 * b)
        out[j]["by"] = (65536 * int(y[i]) - int(v[vi, 1]) * di) // (65536 * b)
    return out


@pytest.mark.parametrize("seed", range(3))
def test_translation_by_whole_bins_keeps_features(seed):
    x, y, e, snr, t, v, b = _random_case(seed)
    c = _some_candidates(x, y, e, t, v, b)
    f0 = of.candidate_features(x, y, e, snr, t, v, b, c)
    k, l = 3, -2
    c2 = c.copy()
    c2["bx"] += k
    c2["by"] += l
    f1 = of.candidate_features(x + k * b, y + l * b, e, snr, t, v, b, c2)
    np.testing.assert_allclose(f1, f0, rtol=0, atol=1e-12)
    assert np.all(f0[:, 0] > 0)  # every candidate holds at least one detection


def test_permutation_and_clock_origin():
    x, y, e, snr, t, v, b = _random_case(7)
    c = _some_candidates(x, y, e, t, v, b)
    f0 = of.candidate_features(x, y, e, snr, t, v, b, c)
    p = np.random.default_rng(1).permutation(len(x))
    f1 = of.candidate_features(x[p], y[p], e[p], snr[p], t + 123456, v, b, c)
    np.testing.assert_allclose(f1, f0, rtol=0, atol=1e-12)


def test_noiseless_mover_has_flat_residuals():
    """A mover moving exactly at a trial velocity: its residuals are constant
    up to the Q8 position quantisation (no slope, ~no scatter), every epoch
    is covered once and no epoch holds two detections."""
    E, b = 16, 1024
    t = (np.arange(E) * 65536 // 4).astype(np.int64)        # 15 min apart
    vx, vy = 512, -256                                       # 2, -1 px/h
    x = (100 * 256 + (vx * t) // 65536).astype(np.int32)
    y = (300 * 256 + (vy * t) // 65536).astype(np.int32)
    e = np.arange(E, dtype=np.uint8)
    snr = np.full(E, 4.0, np.float32)
    v = np.array([[vx, vy]], np.int32)
    c = _cand(0, (100 * 256) // b, (300 * 256) // b)
    f = of.candidate_features(x, y, e, snr, t, v, b, c)[0]
    assert f[0] == 1.0 and f[1] == 1.0 and f[4] == 1.0 and f[30] == 0.0
    assert f[14] < 1.0 / b and f[15] < 1.0 / b
    assert abs(f[16]) < 2.0 / b and abs(f[17]) < 2.0 / b
    np.testing.assert_allclose(f[26:30], [4 / 16, 4 / 16, 4 / 16, 4 / 16])
    assert f[5] == pytest.approx(vx / np.hypot(vx, vy))


def test_labels_follow_the_injected_track():
    E, b = 10, 1024
    t = (np.arange(E) * 65536 // 2).astype(np.int64)        # half-hour steps
    truth = {"x_mid": np.array([200.0]), "y_mid": np.array([100.0]),
             "vx": np.array([8.0]), "vy": np.array([-4.0]), "t_mid_h": 2.25,
             "present": np.ones((1, E), bool)}
    v = np.array([[8 * 256, -4 * 256], [0, 0]], np.int32)
    # the mover's position at t0 (first epoch): x_mid + vx (0 - t_mid)
    x0, y0 = 200.0 - 8 * 2.25, 100.0 + 4 * 2.25
    bx, by = int(x0 // 4), int(y0 // 4)
    cand = np.zeros(3, CAND_DTYPE)
    cand[0] = (0, bx, by, 0, 0)         # on the track
    cand[1] = (0, bx + 3, by, 0, 0)     # 3 bins off
    cand[2] = (1, bx, by, 0, 0)         # wrong velocity: leaves the track
    lab = of.label_candidates(cand, v, b, t, int(t[0]), truth, 4.0)
    assert list(lab) == [1, 0, 0]


def test_neighbour_features_by_hand():
    """Three candidates: two adjacent (one lattice step, one bin apart), one far."""
    v = np.array([[0, 0], [256, 0], [256 * 40, 0]], np.int32)      # spacing 256
    cand = np.zeros(3, CAND_DTYPE)
    cand[0] = (0, 10, 10, 20, 0)
    cand[1] = (1, 11, 9, 30, 0)
    cand[2] = (2, 10, 10, 25, 0)
    nf = of.neighbour_features(cand, v, 256)
    np.testing.assert_allclose(nf, [[1 / 80, 30 / 20], [1 / 80, 20 / 30], [0, 0]])
    assert np.all(of.neighbour_features(cand, v, 0) == 0)


def test_neighbour_features_rounding_sharing_and_rows():
    """Lattice rounding half up (v = 1.5 s lands on index 2, -1.5 s on -1),
    two candidates on one lattice index and bin counted once with the larger
    count, the 4095 cap, and rows looked up against the whole list."""
    s = 100
    v = np.array([[150, 0], [200, 0], [-150, 0], [0, 0], [210, 0]], np.int32)
    cand = np.zeros(5, CAND_DTYPE)
    cand[0] = (0, 0, 0, 9000, 0)   # index (2, 0), count capped to 4095
    cand[1] = (3, 1, 1, 50, 0)     # index (0, 0): two lattice steps from 0, no neighbour of it
    cand[2] = (2, 5, 5, 40, 0)     # index (-1, 0), alone
    cand[3] = (1, 1, 1, 60, 0)     # index (2, 0), bin (1, 1): next to cand 0
    cand[4] = (4, 1, 1, 70, 0)     # v = 2.1 s -> index (2, 0), same key as cand 3
    nf = of.neighbour_features(cand, v, s)
    # cand 0 sees the shared key (2, 0, 1, 1) once, with count 70
    np.testing.assert_allclose(nf[0], [1 / 80, 70 / 4095])
    # cand 1 at (0, 0, 1, 1): nothing at lattice index -1..1 except itself
    np.testing.assert_allclose(nf[1], [0, 0])
    np.testing.assert_allclose(nf[2], [0, 0])
    # cands 3 and 4 share a key: each sees cand 0 only (the shared key is its own)
    np.testing.assert_allclose(nf[3], [1 / 80, 4095 / 60])
    np.testing.assert_allclose(nf[4], [1 / 80, 4095 / 70])
    sub = of.neighbour_features(cand, v, s, rows=[4, 0])
    np.testing.assert_allclose(sub, nf[[4, 0]])

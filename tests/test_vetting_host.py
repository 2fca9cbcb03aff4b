"""Host-side vetting logic: mover matching against the oracle's labels,
operating-point choice, balancing and the recall / false-positive count."""
import numpy as np

from oracle import features as of
from paper_2509_26279_amd import sas, synth, vetting

CAND = np.dtype([("v_idx", "<i4"), ("bx", "<i4"), ("by", "<i4"), ("count", "<u2"),
                 ("flags", "<u2")])


def _candidates_near_movers(wl, v, seed, per_mover=6, n_random=400):
    """Candidate records around the movers' t0 positions at grid velocities
    near theirs (some on the track, some a few bins or velocity steps off),
    plus random records."""
    rng = np.random.default_rng(seed)
    t = np.asarray(wl.t_q16, dtype=np.float64)
    present = np.zeros(wl.n_epochs, dtype=bool)
    present[np.asarray(wl.epoch, dtype=np.int64)] = True
    t0 = float(t[present].min())
    t0_h = (t0 - t.min()) / 65536.0
    b = wl.binw_q8 / 256.0
    vv = v.astype(np.float64) / 256.0
    tr = wl.truth
    from scipy.spatial import cKDTree
    _, nearest = cKDTree(vv).query(np.stack([tr["vx"], tr["vy"]], axis=1), k=4)
    recs = []
    for k in range(len(tr["vx"])):
        x0 = tr["x_mid"][k] + tr["vx"][k] * (t0_h - tr["t_mid_h"])
        y0 = tr["y_mid"][k] + tr["vy"][k] * (t0_h - tr["t_mid_h"])
        near = nearest[k]
        for _ in range(per_mover):
            j = int(rng.choice(near))
            ox, oy = rng.integers(-3, 4, 2)
            recs.append((j, int(np.floor(x0 / b)) + ox, int(np.floor(y0 / b)) + oy, 20, 0))
    for _ in range(n_random):
        recs.append((int(rng.integers(len(v))), int(rng.integers(-10, 140)),
                     int(rng.integers(-10, 270)), 20, 0))
    return np.array(recs, dtype=CAND), int(t0)


def test_match_movers_equals_oracle_labels():
    wl = synth.make_fast(7, noise_per_epoch=50)
    v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
    cand, t0 = _candidates_near_movers(wl, v, 1)
    m = vetting.match_movers(cand, v, wl.binw_q8, wl.t_q16, t0, wl.truth, wl.bin_px)
    lab = of.label_candidates(cand, v, wl.binw_q8, wl.t_q16, t0, wl.truth, wl.bin_px)
    assert 0 < int(lab.sum()) < len(cand)
    np.testing.assert_array_equal((m >= 0).astype(np.uint8), lab)
    # the matched index is the smallest qualifying mover (brute force)
    t = np.asarray(wl.t_q16, dtype=np.float64)
    th, tc = (t - t0) / 65536.0, (t - t.min()) / 65536.0
    b = wl.binw_q8 / 256.0
    tr = wl.truth
    for i in np.nonzero(m >= 0)[0][:40]:
        vx, vy = v[cand[i]["v_idx"]] / 256.0
        cx = (cand[i]["bx"] + 0.5) * b + vx * th
        cy = (cand[i]["by"] + 0.5) * b + vy * th
        ok = [np.sum(np.hypot(tr["x_mid"][k] + tr["vx"][k] * (tc - tr["t_mid_h"]) - cx,
                              tr["y_mid"][k] + tr["vy"][k] * (tc - tr["t_mid_h"]) - cy)
                     < wl.bin_px) >= 0.5 * len(t) for k in range(len(tr["vx"]))]
        assert int(np.argmax(ok)) == m[i]


def test_recall_fp_counts():
    matched = np.array([0, 0, 1, -1, -1, 2, 3])
    findable = np.array([True, True, False, True])
    rec, fp = vetting.recall_fp([1, 0, 1, 1, 0, 1, 0], matched, findable)
    # found: movers 0, 1 (not findable), 2; findable 0, 1, 3 -> 0 and ... 2 of 3
    assert fp == 1 and abs(rec - 2 / 3) < 1e-12
    assert vetting.recall_fp(np.zeros(7), matched, findable) == (0.0, 0)
    assert vetting.recall_fp(np.zeros(0), np.zeros(0, int), np.zeros(0, bool)) == (1.0, 0)


def test_superset_tau_keeps_every_plain_mover():
    rng = np.random.default_rng(3)
    n_movers = 40
    matched = np.where(rng.uniform(size=2000) < 0.5, rng.integers(0, n_movers, 2000), -1)
    findable = rng.uniform(size=n_movers) < 0.8
    scores = rng.normal(size=2000) + 2.0 * (matched >= 0)
    plain = rng.uniform(size=2000) < 0.3
    tau = vetting.superset_tau(scores, matched, findable, plain)
    plain_found = set(matched[plain & (matched >= 0)].tolist())
    learned_found = set(matched[(scores >= tau) & (matched >= 0)].tolist())
    need = {k for k in plain_found if findable[k]}
    assert need <= learned_found
    # any larger threshold loses one of them
    above = np.unique(scores[scores > tau])
    if len(above):
        lost = set(matched[(scores >= above[0]) & (matched >= 0)].tolist())
        assert not need <= lost
    rp = vetting.recall_fp(plain, matched, findable)[0]
    assert vetting.recall_fp(scores >= tau, matched, findable)[0] >= rp
    assert vetting.superset_tau(scores, matched, findable, np.zeros(2000, bool)) == float("inf")


def test_balance_caps_each_mover():
    matched = np.array([0] * 20 + [1] * 3 + [-1] * 50)
    keep = vetting.balance(matched, 8, seed=0)
    assert keep[matched == -1].all()
    assert keep[matched == 0].sum() == 8 and keep[matched == 1].sum() == 3
    assert vetting.balance(matched, 0).all()


def test_budget_tau():
    scores = np.array([5.0, 4.0, 3.0, 2.0, 1.0, 0.5], dtype=np.float32)
    matched = np.array([-1, 0, -1, -1, 1, -1])
    # negatives 5, 3, 2, 0.5: at most one false positive -> just above 3
    tau = vetting.budget_tau(scores, matched, 1)
    assert 3.0 < tau <= np.nextafter(np.float32(3.0), np.float32(10))
    assert int(((scores >= tau) & (matched < 0)).sum()) == 1
    assert vetting.budget_tau(scores, matched, 0) > 5.0
    assert vetting.budget_tau(scores, matched, 4) == float("-inf")

"""Pins of the Step-3 greedy extraction oracle (oracle/extract.py): a worked
example by hand, invariants of the loop on adversarial catalogs, agreement of
its contributor counts with the C oracle's vote, and recovery of noiseless
movers with their ghosts suppressed."""
import numpy as np
import pytest

import oracle
from oracle import extract as ox
from paper_2509_26279_amd import synth

CAND = oracle.CAND_DTYPE


def _hand():
    # 4 px bins, epochs at 0, 1 and 2 h; velocities 0, 1 and 2 px/h along x.
    # A: static at (1, 1) px; B: x = 10, 12, 14 px at y = 9 px (2 px/h).
    x = np.array([1, 1, 1, 10, 12, 14]) * 256
    y = np.array([1, 1, 1, 9, 9, 9]) * 256
    e = np.array([0, 1, 2, 0, 1, 2])
    t = np.array([0, 1, 2]) * 65536
    v = np.array([[0, 0], [256, 0], [512, 0]])
    return x, y, e, t, v, 1024


def test_hand_example():
    """By hand (bin = floor((x - v t) / 4 px)):
      v0: A -> (0, 0) x3; B -> (2, 2), (3, 2), (3, 2)
      v1: A -> (0, 0), (0, 0), (-1, 0); B -> (2, 2), (2, 2), (3, 2)
      v2: A -> (0, 0), (-1, 0), (-1, 0); B -> (2, 2) x3
    At N_min = 2 the vote reports six cells; v0 (0, 0) and v2 (2, 2) hold 3
    (the tie goes to the smaller v_idx).  Taking A at v0 empties every cell
    A fed; B at v2 is then the maximum; nothing is left after it."""
    x, y, e, t, v, b = _hand()
    cand = oracle.vote(x, y, e, t, v, b, 2)
    assert len(cand) == 6
    got = ox.extract(x, y, e, t, v, b, cand, 2)
    assert [(c[0], c[1], c[2], c[3]) for c in got] == [(0, 0, 0, 3), (2, 2, 2, 3)]
    assert sorted(got[0][4].tolist()) == [0, 1, 2] and sorted(got[1][4].tolist()) == [3, 4, 5]
    # the same in detection counts; and at N_min = 4 nothing is extracted
    assert [(c[0], c[3]) for c in ox.extract(x, y, e, t, v, b, cand, 2, "detections")] == \
        [(0, 3), (2, 3)]
    assert ox.extract(x, y, e, t, v, b, cand, 4) == []


def test_tie_break_by_then_bx():
    """Two cells of one velocity with equal counts: the smaller by goes first,
    then, at equal by, the smaller bx."""
    x = np.array([1, 1, 9, 9, 9, 9]) * 256
    y = np.array([9, 9, 9, 9, 1, 1]) * 256
    e = np.array([0, 1, 0, 1, 0, 1])
    t = np.array([0, 1]) * 65536
    v = np.array([[0, 0]])
    cand = oracle.vote(x, y, e, t, v, 1024, 2)
    got = ox.extract(x, y, e, t, v, 1024, cand, 2)
    assert [(c[1], c[2]) for c in got] == [(2, 0), (0, 2), (2, 2)]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mode", ["epochs", "detections"])
def test_loop_invariants(seed, mode):
    d = synth.make_random_small(seed, n=120, n_epochs=[4, 6, 9][seed % 3], n_v=12,
                                dup_frac=0.3)
    n_min = 2
    cand = oracle.vote(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"],
                       n_min, mode)
    members = ox.contributors(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"],
                              d["binw_q8"], cand)
    ep = np.asarray(d["epoch"])
    # the contributors of a cell reproduce the C oracle's count of it
    for c, m in zip(cand, members):
        n = len(np.unique(ep[m])) if mode == "epochs" else len(m)
        assert n == int(c["count"])
    got = ox.extract(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], d["v_q8"], d["binw_q8"],
                     cand, n_min, mode)
    taken = np.concatenate([g[4] for g in got]) if got else np.zeros(0, int)
    assert len(taken) == len(np.unique(taken))  # clusters are disjoint
    counts = [g[3] for g in got]
    assert all(a >= b for a, b in zip(counts, counts[1:]))  # the maximum only falls
    for g in got:
        n = len(np.unique(ep[g[4]])) if mode == "epochs" else len(g[4])
        assert n == g[3] >= n_min
    if got:  # the first cluster is the vote's maximum under the tie rule
        k = min(range(len(cand)), key=lambda i: (-int(cand[i]["count"]), int(cand[i]["v_idx"]),
                                                 int(cand[i]["by"]), int(cand[i]["bx"])))
        assert (got[0][0], got[0][1], got[0][2]) == \
            (int(cand[k]["v_idx"]), int(cand[k]["bx"]), int(cand[k]["by"]))
    alive = np.ones(len(ep), bool)
    alive[taken] = False
    for m in members:  # nothing left at or above N_min
        live = m[alive[m]]
        n = len(np.unique(ep[live])) if mode == "epochs" else len(live)
        assert n < n_min


def test_noiseless_movers_one_cluster_each():
    """Movers on lattice velocities, far apart, no noise: the vote reports
    each mover at its own velocity and at many ghost cells; the loop takes
    exactly one cluster per mover, holding all of its detections."""
    t = np.arange(8) * 65536 // 2  # 8 epochs over 3.5 h
    s = 256  # 1 px/h lattice
    v = np.array([[i * s, j * s] for j in range(-3, 4) for i in range(-3, 4)])
    movers = [(40.5, 40.5, 2, -1), (140.5, 60.5, -3, 0), (90.5, 150.5, 1, 3)]
    xs, ys, es = [], [], []
    for (x0, y0, vx, vy) in movers:
        for e in range(len(t)):
            h = t[e] / 65536
            xs.append(int((x0 + vx * h) * 256))
            ys.append(int((y0 + vy * h) * 256))
            es.append(e)
    x, y, e = np.array(xs), np.array(ys), np.array(es)
    cand = oracle.vote(x, y, e, t, v, 1024, 5)
    assert len(cand) > len(movers)
    got = ox.extract(x, y, e, t, v, 1024, cand, 5)
    assert len(got) == len(movers)
    owners = sorted(tuple(sorted(set((g[4] // len(t)).tolist()))) for g in got)
    assert owners == [(0,), (1,), (2,)]
    assert all(len(g[4]) == len(t) for g in got)

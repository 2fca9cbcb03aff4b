"""Pins of the Refine / Gather / iterate oracle (Steps 4-6 of Sec. 2.1,
oracle/refine.py): the regression against numpy's least squares on the
chosen subset, FAST-MCD against the exact MCD by brute force on small sets,
the C-step theorem (the determinant never increases), affine equivariance,
robustness to 40 % outliers, the gather against a plain loop, and the whole
iteration recovering a mover in noise."""
import itertools
import math

import numpy as np
import pytest

from oracle import refine as R
from paper_2509_26279_amd import synth

STARTS = synth.mcd_starts(7, 500)


def _line(n, vx, vy, sig, seed, x0=100.0, y0=50.0, span=4.0):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0, span, n))
    return np.stack([t, x0 + vx * t + rng.normal(0, sig, n), y0 + vy * t + rng.normal(0, sig, n)],
                    axis=1)


def test_regression_is_least_squares_on_the_subset():
    z = _line(60, 12.0, -7.0, 0.4, 1)
    sub, mu, S = R.fast_mcd(z, STARTS)
    B, c, sig = R.regress(mu, S)
    zs = z[sub]
    A = np.stack([zs[:, 0], np.ones(len(zs))], axis=1)
    coef, *_ = np.linalg.lstsq(A, zs[:, 1:], rcond=None)
    assert np.allclose(B, coef[0], rtol=1e-10, atol=1e-10)
    assert np.allclose(c, coef[1], rtol=1e-10, atol=1e-9)
    res = zs[:, 1:] - A @ coef
    assert np.allclose(sig, res.T @ res / len(zs), rtol=1e-8, atol=1e-12)
    assert len(sub) == R.h_of(60) == 32


@pytest.mark.parametrize("seed", range(5))
def test_fast_mcd_finds_the_exact_mcd_on_small_sets(seed):
    rng = np.random.default_rng(seed)
    n = 11
    z = np.stack([rng.uniform(0, 3, n), rng.normal(0, 2, n), rng.normal(0, 2, n)], axis=1)
    z[:3, 1:] += 15.0 * rng.normal(size=(3, 2))  # a few outliers
    h = R.h_of(n)
    best = min(itertools.combinations(range(n), h),
               key=lambda s: np.linalg.det(R.mean_cov(z[list(s)])[1]))
    sub, _, _ = R.fast_mcd(z, STARTS)
    assert list(sub) == list(best)


@pytest.mark.parametrize("seed", range(6))
def test_c_steps_never_raise_the_determinant(seed):
    z = _line(80, 3.0, 1.0, 1.0, seed + 10)
    z[::5, 1:] += np.random.default_rng(seed).uniform(-40, 40, (16, 2))
    h = R.h_of(len(z))
    sub = np.sort(np.random.default_rng(seed).choice(len(z), h, replace=False))
    det = np.linalg.det(R.mean_cov(z[sub])[1])
    for _ in range(8):
        sub = R.c_step(z, sub, h)
        d = np.linalg.det(R.mean_cov(z[sub])[1])
        assert d <= det * (1 + 1e-12)
        det = d


def test_affine_equivariance():
    z = _line(50, 5.0, 2.0, 0.7, 3)
    z[:12, 1:] += 30.0
    sub, mu, S = R.fast_mcd(z, STARTS)
    B, c, _ = R.regress(mu, S)
    # shift and scale the positions: the same subset, the line moves with them
    z2 = z.copy()
    z2[:, 1] = 3.0 * z[:, 1] + 17.0
    z2[:, 2] = 3.0 * z[:, 2] - 4.0
    sub2, mu2, S2 = R.fast_mcd(z2, STARTS)
    B2, c2, _ = R.regress(mu2, S2)
    assert np.array_equal(sub, sub2)
    assert np.allclose(B2, 3.0 * B) and np.allclose(c2, [3.0 * c[0] + 17.0, 3.0 * c[1] - 4.0])


@pytest.mark.parametrize("frac", [0.2, 0.4])
def test_robust_to_outliers(frac):
    n = 100
    z = _line(n, 20.0, -10.0, 0.3, 5)
    k = int(frac * n)
    rng = np.random.default_rng(9)
    bad = rng.choice(n, k, replace=False)
    z[bad, 1:] = rng.uniform(-200, 400, (k, 2))
    sub, mu, S = R.fast_mcd(z, STARTS)
    B, c, _ = R.regress(mu, S)
    assert not set(sub) & set(bad.tolist())
    assert abs(B[0] - 20.0) < 0.5 and abs(B[1] + 10.0) < 0.5
    # plain least squares on all points is pulled away
    A = np.stack([z[:, 0], np.ones(n)], axis=1)
    coef, *_ = np.linalg.lstsq(A, z[:, 1:], rcond=None)
    assert abs(coef[0][0] - 20.0) > 1.0 or abs(coef[0][1] + 10.0) > 1.0


def test_gather_against_a_loop():
    d = synth.make_random_small(3, n=400, n_epochs=7, binw_q8=1024)
    B, c, dx = np.array([1.5, -0.75]), np.array([2.0, -3.0]), 6.0
    got = R.gather(d["x_q8"], d["y_q8"], d["epoch"], d["t_q16"], B, c, dx)
    t = np.asarray(d["t_q16"], dtype=np.int64)
    t0 = min(int(t[e]) for e in d["epoch"])
    want = []
    for i in range(len(d["x_q8"])):
        th = (int(t[d["epoch"][i]]) - t0) / 65536.0
        px, py = c[0] + B[0] * th, c[1] + B[1] * th
        if math.hypot(d["x_q8"][i] / 256.0 - px, d["y_q8"][i] / 256.0 - py) <= dx:
            want.append(i)
    assert got.tolist() == want and len(want) > 0
    # a point exactly at distance dx is gathered
    x = np.array([256 * 10, 256 * 16], np.int32)
    y = np.array([256 * 10, 256 * 10], np.int32)
    g = R.gather(x, y, [0, 0], [0], np.array([0.0, 0.0]), np.array([10.0, 10.0]), 6.0)
    assert g.tolist() == [0, 1]


def test_iteration_recovers_a_mover_in_noise():
    rng = np.random.default_rng(4)
    E, vx, vy = 30, 14.0, 6.0
    t_q16 = (np.arange(E) * 65536 * 4 // (E - 1)).astype(np.int64) + 12345
    th = (t_q16 - t_q16[0]) / 65536.0
    mx = 300.0 + vx * th + rng.normal(0, 0.4, E)
    my = 200.0 + vy * th + rng.normal(0, 0.4, E)
    nn = 3000
    nx, ny, ne = rng.uniform(0, 600, nn), rng.uniform(0, 600, nn), rng.integers(0, E, nn)
    x = np.floor(256 * np.concatenate([mx, nx])).astype(np.int32)
    y = np.floor(256 * np.concatenate([my, ny])).astype(np.int32)
    e = np.concatenate([np.arange(E), ne]).astype(np.uint8)
    # a Step-3 cluster: 20 of the mover's detections and 8 noise points near it
    near = np.nonzero((np.abs(nx - 350) < 40) & (np.abs(ny - 220) < 40))[0][:8] + E
    members = np.concatenate([np.arange(0, 20), near])
    out = R.refine_cluster(x, y, e, t_q16, members, STARTS, 4.0)
    assert out["status"] == R.STATUS_CONVERGED
    assert abs(out["B"][0] - vx) < 0.3 and abs(out["B"][1] - vy) < 0.3
    assert set(range(E)) <= set(out["gathered"].tolist())  # every detection of the mover
    assert len(out["gathered"]) < E + 10


def test_too_small_and_starts_as_input():
    x = np.arange(4, dtype=np.int32) * 256
    out = R.refine_cluster(x, x, np.arange(4), np.arange(4) * 65536, [0, 1, 2, 3], STARTS, 4.0)
    assert out["status"] == R.STATUS_TOO_SMALL
    # every start repeating a point: no start survives
    z = _line(20, 1.0, 1.0, 0.5, 2)
    assert R.fast_mcd(z, np.zeros((8, 4), np.uint32)) is None

"""Pins of the FP64 MLP reference (oracle/mlp_ref.py): its gradient against
finite differences of its own loss in exact FP64, the bf16 rounding against
known values, the loss against its closed form, AdamW against a hand step."""
import numpy as np
import pytest

from oracle import mlp_ref as M


def _case(seed, B=24):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, M.N_PARAMS)
    x = rng.normal(0, 1, (B, M.D_IN))
    y = (rng.uniform(size=B) < 0.3).astype(np.float64)
    mu = rng.normal(0, 0.1, M.D_IN)
    sd = rng.uniform(0.5, 2.0, M.D_IN)
    return p, x, y, mu, sd


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_finite_differences(seed):
    p, x, y, mu, sd = _case(seed)
    loss, g = M.loss_and_grad(p, x, y, mu, sd, pos_weight=2.5, bf16_on=False)
    rng = np.random.default_rng(100 + seed)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    # every block of parameters is probed
    idx = np.union1d(idx, [0, 32 * 128, 32 * 128 + 128 + 5, M.N_PARAMS - 129, M.N_PARAMS - 1])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = M.loss_and_grad(pp, x, y, mu, sd, pos_weight=2.5, bf16_on=False)
        lm, _ = M.loss_and_grad(pm, x, y, mu, sd, pos_weight=2.5, bf16_on=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_bf16_rounding_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, 1.0 + 3 * 2 ** -8,
                     -2.5, 3.14159265, 0.0])
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 4 * 2 ** -8, -2.5, 3.140625, 0.0])
    np.testing.assert_array_equal(M.bf16(vals), exp)   # ties go to even


def test_loss_closed_form_and_zero_network():
    p = np.zeros(M.N_PARAMS)
    x = np.random.default_rng(0).normal(size=(10, M.D_IN))
    y = np.array([1, 0] * 5, np.float64)
    loss, g = M.loss_and_grad(p, x, y, np.zeros(32), np.ones(32), pos_weight=3.0)
    # z = 0 everywhere: softplus(0) = log 2; mean of 3 y + (1 - y) times log 2
    assert loss == pytest.approx(np.log(2) * (3 * 5 + 5) / 10)
    P = M.unpack(g)
    # dz = (0.5 (3 y + 1 - y) - 3 y) / 10: -0.15 for y = 1, 0.05 for y = 0
    assert P["b3"][0] == pytest.approx(M.bf16(np.array([-0.15]))[0] * 5 +
                                       M.bf16(np.array([0.05]))[0] * 5)
    assert np.all(P["W1"] == 0) and np.all(P["W2"] == 0)   # dead ReLUs pass no gradient


def test_adamw_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.1, -0.2, 0.0])
    p1, m, v = M.adamw(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, wd=0.1)
    # step 1: m_hat = g, v_hat = g^2, so the update is lr (sign(g) + wd p) for g != 0
    np.testing.assert_allclose(p1[:2], p[:2] - 0.01 * (np.sign(g[:2]) * (1 / (1 + 1e-8 / np.abs(g[:2]))) + 0.1 * p[:2]))
    assert p1[2] == pytest.approx(0.5 - 0.01 * 0.1 * 0.5)


def test_each_rounding_point_is_resolved_by_the_gpu_tolerance():
    """The GPU comparison (tests/test_gpu_mlp.py) allows a relative L2 error
    of TOL on the logits and on each gradient block.  Leaving out any one
    bf16 rounding point of the reference moves the logits (forward points)
    or some gradient block by more than 5 TOL on every gradient case, so a
    kernel that misses or misplaces a rounding point cannot pass."""
    from mlp_case import BLOCKS, GRAD_CASES, TOL, case, rel_l2
    for B, pw in GRAD_CASES:
        p, x, y, mu, sd = case(100 + B, B)
        z, _ = M.forward(p, x, mu, sd)
        _, g = M.loss_and_grad(p, x, y, mu, sd, pos_weight=pw)
        for pt in M.POINTS:
            keep = tuple(q for q in M.POINTS if q != pt)
            z2, _ = M.forward(p, x, mu, sd, points=keep)
            _, g2 = M.loss_and_grad(p, x, y, mu, sd, pos_weight=pw, points=keep)
            shift = max([rel_l2(z2, z)] + [rel_l2(g2[a:b], g[a:b]) for _, a, b in BLOCKS])
            assert shift > 5 * TOL, (B, pt, shift)
        # and the full set of points is the default
        z3, _ = M.forward(p, x, mu, sd, points=M.POINTS)
        assert np.array_equal(z3, z)

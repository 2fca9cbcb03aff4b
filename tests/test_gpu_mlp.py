"""The vetting MLP's GPU kernels (bf16 MFMA, FP32 accumulation) against the
FP64 reference with the same bf16 rounding points (oracle/mlp_ref.py)."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2509_26279_amd import sas

pytestmark = pytest.mark.gpu

BLOCKS = [("W1", 0, 4096), ("b1", 4096, 4224), ("W2", 4224, 20608), ("b2", 20608, 20736),
          ("W3", 20736, 20864), ("b3", 20864, 20865)]


def _case(seed, B):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.15, M.N_PARAMS).astype(np.float32)
    p[4096:4224] = rng.normal(0, 0.2, 128)      # biases that keep units alive
    p[20608:20736] = rng.normal(0, 0.2, 128)
    x = rng.normal(0.3, 1.5, (B, 32)).astype(np.float32)
    y = (rng.uniform(size=B) < 0.25).astype(np.float32)
    mu = rng.normal(0.3, 0.1, 32).astype(np.float32)
    sd = rng.uniform(1.0, 2.0, 32).astype(np.float32)
    sd[5] = 0.0                                 # a constant feature
    return p, x, y, mu, sd


def _net(p, mu, sd, max_batch=4096):
    net = sas.MLP(max_batch=max_batch, seed=1)
    net.set_params(p)
    net.set_norm(mu, sd)
    return net


@pytest.mark.parametrize("B", [1, 37, 640, 4096])
def test_forward_matches_reference(gpu, B):
    import torch
    p, x, y, mu, sd = _case(B, B)
    net = _net(p, mu, sd)
    z = net.forward(torch.as_tensor(x).cuda()).cpu().numpy()
    ref, _ = M.forward(p, x, mu, sd)
    np.testing.assert_allclose(z, ref, rtol=5e-3, atol=5e-3 * max(1.0, np.abs(ref).max()))
    net.close()


def test_forward_any_n_in_chunks(gpu):
    import torch
    p, x, y, mu, sd = _case(9, 1000)
    net = _net(p, mu, sd, max_batch=256)        # 4 chunks, the last one partial
    z = net.forward(torch.as_tensor(x).cuda()).cpu().numpy()
    ref, _ = M.forward(p, x, mu, sd)
    np.testing.assert_allclose(z, ref, rtol=5e-3, atol=5e-3 * max(1.0, np.abs(ref).max()))
    net.close()


@pytest.mark.parametrize("B,pw", [(64, 1.0), (700, 3.0), (4096, 10.0)])
def test_gradient_matches_reference(gpu, B, pw):
    import torch
    p, x, y, mu, sd = _case(100 + B, B)
    net = _net(p, mu, sd)
    xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    loss, g = net.grad(xt, yt, pw)
    g = g.cpu().numpy().astype(np.float64)
    rl, rg = M.loss_and_grad(p, x, y, mu, sd, pos_weight=pw)
    assert float(loss.cpu()) == pytest.approx(rl, rel=2e-3)
    for name, a, b in BLOCKS:
        err = np.linalg.norm(g[a:b] - rg[a:b]) / max(np.linalg.norm(rg[a:b]), 1e-12)
        assert err < 2e-2, (name, err)
    # determinism: the same batch gives the same gradient bit for bit
    _, g2 = net.grad(xt, yt, pw)
    assert np.array_equal(g2.cpu().numpy().astype(np.float64), g)
    net.close()


def test_adamw_step_matches_reference(gpu):
    import torch
    p, x, y, mu, sd = _case(5, 512)
    net = _net(p, mu, sd)
    xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    _, g = net.grad(xt, yt, 2.0)
    g = g.cpu().numpy().astype(np.float64)
    params, m, v = p.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    for t in (1, 2):
        net.train_step(xt, yt, 2.0, lr=1e-2, weight_decay=0.05)
        _, gt = net.grad(xt, yt, 2.0) if t == 1 else (None, None)
        params, m, v = M.adamw(params, g, m, v, t, lr=1e-2, wd=0.05)
        if t == 1:
            np.testing.assert_allclose(net.params(), params, rtol=1e-5, atol=1e-6)
            g = gt.cpu().numpy().astype(np.float64)   # the gradient at the new point
    np.testing.assert_allclose(net.params(), params, rtol=1e-5, atol=1e-6)
    net.close()


def test_training_separates_a_toy_problem(gpu):
    import torch
    rng = np.random.default_rng(3)
    n = 8192
    x = rng.normal(size=(n, 32)).astype(np.float32)
    y = ((x[:, 0] + 0.5 * x[:, 3] - 0.25 * x[:, 7] ** 2) > 0.3).astype(np.float32)
    net = sas.MLP(max_batch=1024, seed=7)
    net.set_norm(x.mean(0), x.std(0))
    xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    losses = []
    for it in range(300):
        b = (it * 1024) % n
        losses.append(float(net.train_step(xt[b:b + 1024], yt[b:b + 1024], 1.0, lr=3e-3).cpu()))
    acc = ((net.forward(xt).cpu().numpy() > 0) == (y > 0.5)).mean()
    assert losses[-1] < 0.5 * losses[0] and acc > 0.95, (losses[0], losses[-1], acc)
    net.close()

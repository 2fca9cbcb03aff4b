"""The vetting MLP's GPU kernels (bf16 MFMA, FP32 accumulation) against the
FP64 reference with the same bf16 rounding points (oracle/mlp_ref.py).

Both sides round at the same points, so they differ only where an FP32 sum
and the FP64 sum of the same terms round to different bf16 values; the
bound TOL (relative L2 per tensor) is far below the effect of any one
rounding point (tests/test_oracle_mlp.py)."""
import sys

import numpy as np
import pytest

from mlp_case import BLOCKS, GRAD_CASES, TOL, case, rel_l2
from oracle import mlp_ref as M
from paper_2509_26279_amd import sas

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _net(p, mu, sd, max_batch=4096):
    net = sas.MLP(max_batch=max_batch, seed=1)
    net.set_params(p)
    net.set_norm(mu, sd)
    return net


@pytest.mark.parametrize("B", [1, 37, 640, 4096])
def test_forward_matches_reference(gpu, B):
    import torch
    p, x, y, mu, sd = case(B, B)
    net = _net(p, mu, sd)
    z = net.forward(torch.as_tensor(x).cuda()).cpu().numpy()
    ref, _ = M.forward(p, x, mu, sd)
    err = rel_l2(z, ref)
    _say(f"forward B={B}: logits rel-L2 {err:.2e}")
    assert err < TOL, err
    net.close()


def test_forward_any_n_in_chunks(gpu):
    import torch
    p, x, y, mu, sd = case(9, 1000)
    net = _net(p, mu, sd, max_batch=256)        # 4 chunks, the last one partial
    z = net.forward(torch.as_tensor(x).cuda()).cpu().numpy()
    ref, _ = M.forward(p, x, mu, sd)
    assert rel_l2(z, ref) < TOL
    net.close()


@pytest.mark.parametrize("B,pw", GRAD_CASES)
def test_gradient_matches_reference(gpu, B, pw):
    import torch
    p, x, y, mu, sd = case(100 + B, B)
    net = _net(p, mu, sd)
    xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    loss, g = net.grad(xt, yt, pw)
    g = g.cpu().numpy().astype(np.float64)
    rl, rg = M.loss_and_grad(p, x, y, mu, sd, pos_weight=pw)
    errs = {name: rel_l2(g[a:b], rg[a:b]) for name, a, b in BLOCKS}
    _say(f"gradient B={B} pw={pw}: loss rel {abs(float(loss.cpu()) - rl) / abs(rl):.2e}, "
         + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert float(loss.cpu()) == pytest.approx(rl, rel=TOL)
    for name, err in errs.items():
        assert err < TOL, (name, err)
    # determinism: the same batch gives the same gradient bit for bit
    _, g2 = net.grad(xt, yt, pw)
    assert np.array_equal(g2.cpu().numpy().astype(np.float64), g)
    net.close()


def test_adamw_step_matches_reference(gpu):
    import torch
    p, x, y, mu, sd = case(5, 512)
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


def test_checkpoint_resumes_training_bit_for_bit(gpu):
    """Ten AdamW steps in one run against five steps, a checkpoint, and five
    more steps in a fresh network of another seed and batch size restored
    from it: identical parameters and logits, bit for bit."""
    import torch
    rng = np.random.default_rng(11)
    x = rng.normal(size=(4096, 32)).astype(np.float32)
    y = (x[:, 1] - x[:, 2] > 0.2).astype(np.float32)
    xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    batches = [(xt[k * 512:(k + 1) * 512], yt[k * 512:(k + 1) * 512]) for k in range(8)]

    def steps(net, ks):
        for k in ks:
            bx, by = batches[k % len(batches)]
            net.train_step(bx, by, 2.5, lr=3e-3, weight_decay=0.02)

    a = sas.MLP(max_batch=1024, seed=3)
    a.set_norm(x.mean(0), x.std(0))
    steps(a, range(5))
    blob = a.save()
    assert blob.startswith(b'{"format": "sas_mlp",') and b'"step": 5,' in blob[:256]
    steps(a, range(5, 10))
    b = sas.MLP(max_batch=512, seed=99)
    b.load(blob)
    steps(b, range(5, 10))
    assert np.array_equal(a.params(), b.params())
    assert np.array_equal(a.forward(xt).cpu().numpy(), b.forward(xt).cpu().numpy())
    # a corrupted header or a wrong size is refused
    bad = bytearray(blob)
    bad[2:8] = b"XXXXXX"
    with pytest.raises(sas.SasError):
        b.load(bytes(bad))
    with pytest.raises(sas.SasError):
        b.load(blob[:-4])
    a.close()
    b.close()


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

"""FP64 reference of the vetting MLP (TEST INFRASTRUCTURE ONLY, see
oracle/__init__.py).  The paper has no learned component; this is the plain
definition the GPU kernels implement, written with numpy.

Network 32 -> 128 -> 128 -> 1 with ReLU (derivative 0 at 0):
    a0 = q((x - mu) / sd)                       (sd = 0 counts as 1)
    h1 = q(relu(a0 W1 + b1))
    h2 = q(relu(h1 W2 + b2))
    z  = h2 q(W3) + b3                           (logit)
with W1, W2 also used as q(W).  q is rounding to bfloat16 (round to nearest
even of the float32 value); with bf16=False q is the identity and the whole
computation is exact FP64 (used to check the gradient by finite
differences).  The rounding points are named (POINTS); `points` selects
which of them round (all by default), so that a test can show that each of
them is visible at the GPU comparison's tolerance.

Loss: mean over the batch of binary cross-entropy with logits and a weight
pw on positives,  l = pw y softplus(-z) + (1 - y) softplus(z).
Backward (dz = dl/dz = (sigmoid(z) (pw y + 1 - y) - pw y) / B):
    g3 = q(dz);   dW3 = h2^T g3;  db3 = sum g3
    d2 = q((g3 q(W3)^T) * [h2 > 0]);  dW2 = h1^T d2;  db2 = colsum d2
    d1 = q((d2 q(W2)^T) * [h1 > 0]);  dW1 = a0^T d1;  db1 = colsum d1
AdamW (Loshchilov & Hutter 2019), decoupled weight decay on every parameter:
    m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2
    w = w - lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd w)
Parameters are packed W1 (32 x 128, row-major), b1, W2 (128 x 128), b2,
W3 (128), b3: 20865 values.
"""
from __future__ import annotations

import numpy as np

D_IN, D_H = 32, 128
SIZES = [("W1", (D_IN, D_H)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
         ("W3", (D_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16(a):
    """Round to bfloat16 (nearest even) through float32, back to float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(np.isnan(f), np.uint64(0x7FC00000), r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# every bf16 rounding point: the standardised input, the three weight
# matrices, the two hidden activations, the logit gradient and the two
# back-propagated activation gradients
POINTS = ("a0", "W1", "h1", "W2", "h2", "W3", "g3", "d2", "d1")


def _q(a, on):
    return bf16(a) if on else np.asarray(a, dtype=np.float64)


def _on(bf16_on, points, name):
    return bf16_on and (points is None or name in points)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def forward(params, x, mu, sd, bf16_on=True, points=None):
    """Logits and the intermediate activations."""
    P = unpack(params)
    q = lambda a, name: _q(a, _on(bf16_on, points, name))
    sd = np.where(np.asarray(sd, np.float64) == 0, 1.0, np.asarray(sd, np.float64))
    a0 = q((np.asarray(x, np.float64) - np.asarray(mu, np.float64)) / sd, "a0")
    h1 = q(np.maximum(a0 @ q(P["W1"], "W1") + P["b1"], 0.0), "h1")
    h2 = q(np.maximum(h1 @ q(P["W2"], "W2") + P["b2"], 0.0), "h2")
    z = h2 @ q(P["W3"], "W3") + P["b3"][0]
    return z, (a0, h1, h2)


def loss_and_grad(params, x, y, mu, sd, pos_weight=1.0, bf16_on=True, points=None):
    """Mean loss and the gradient (packed like the parameters)."""
    P = unpack(params)
    q = lambda a, name: _q(a, _on(bf16_on, points, name))
    y = np.asarray(y, np.float64)
    z, (a0, h1, h2) = forward(params, x, mu, sd, bf16_on, points)
    B = z.shape[0]
    loss = float(np.mean(pos_weight * y * softplus(-z) + (1 - y) * softplus(z)))
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (sig * (pos_weight * y + 1 - y) - pos_weight * y) / B
    g3 = q(dz, "g3")
    dW3 = h2.T @ g3
    db3 = np.array([g3.sum()])
    d2 = q(np.outer(g3, q(P["W3"], "W3")) * (h2 > 0), "d2")
    dW2 = h1.T @ d2
    db2 = d2.sum(axis=0)
    d1 = q((d2 @ q(P["W2"], "W2").T) * (h1 > 0), "d1")
    dW1 = a0.T @ d1
    db1 = d1.sum(axis=0)
    return loss, pack({"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3})


def adamw(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.01):
    """One AdamW step (t counts from 1); returns new (params, m, v)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    p = np.asarray(params, np.float64)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v

"""Inputs and tolerances shared by the MLP tests (GPU parity against the
FP64 reference, and the CPU check that the tolerance resolves every bf16
rounding point of the reference)."""
import numpy as np

from oracle import mlp_ref as M

BLOCKS = [("W1", 0, 4096), ("b1", 4096, 4224), ("W2", 4224, 20608), ("b2", 20608, 20736),
          ("W3", 20736, 20864), ("b3", 20864, 20865)]

# Relative L2 error allowed between the GPU (FP32 sums, bf16 at the
# reference's rounding points) and the FP64 reference, for the logits and
# for each gradient block.  Dropping any one rounding point from the
# reference moves the logits or some gradient block by 6e-4 or more on the
# cases below (tests/test_oracle_mlp.py checks it), so this bound resolves
# every rounding point.
TOL = 1e-4
# Gradient cases (batch, positive weight).
GRAD_CASES = [(64, 1.0), (700, 3.0), (4096, 10.0)]


def case(seed, B):
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


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

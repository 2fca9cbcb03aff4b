"""Threshold rule of Sec. 2.2 (TEST INFRASTRUCTURE ONLY, see oracle/__init__.py).

N_min is chosen so that the probability that a pure-noise stack reaches it,
times the number of independent stacks N_stacks = |V| * Omega / Delta x^2
(eq. N_stacks), stays at or below an admissible number of false results
N_false (the paper's figure uses 100).

Noise detections form a Poisson process (the Poisson law for N_noise in
Sec. 2.2): with mu detections per bin per epoch, one bin holds at least one
noise detection in a given epoch with probability 1 - exp(-mu).  The number
of distinct epochs of a pure-noise bin is then Binomial(E, 1 - exp(-mu));
the number of detections is Poisson(E mu), the paper's own sum over epochs.
"""
from __future__ import annotations

import math

from scipy.stats import binom, poisson


def expected_noise_candidates(n_min, n_epochs, mu, n_stacks, mode="epochs"):
    """E[# pure-noise stacks with count >= n_min]."""
    if mode == "epochs":
        tail = binom.sf(n_min - 1, n_epochs, 1.0 - math.exp(-mu))
    else:
        tail = poisson.sf(n_min - 1, n_epochs * mu)
    return n_stacks * float(tail)


def choose_n_min(n_epochs, mu, n_stacks, n_false=100.0, mode="epochs"):
    """Smallest N_min with at most n_false expected noise candidates."""
    for n in range(1, 100000):
        if expected_noise_candidates(n, n_epochs, mu, n_stacks, mode) <= n_false:
            return n
    raise ValueError("no threshold reaches the requested false-candidate rate")

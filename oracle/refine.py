"""Refine, Gather and iterate: Steps 4-6 of Sec. 2.1 (TEST INFRASTRUCTURE
ONLY, see oracle/__init__.py).

Step 4 fits a straight trajectory to each cluster by multivariate regression
(Sec. 2, the regression Y = B^T X + c + eps with X = t and Y = (x, y)), made
robust by taking the mean and covariance from the Minimum Covariance
Determinant subset instead of all points.  Step 5 gathers the catalog
detections within Delta x of the fitted line; Step 6 repeats 4 and 5 until
the gathered set no longer changes.

Written out plainly, in FP64:
  * a point is z = (t, x, y): t in hours since the reference epoch t0 of
    Step 1, x and y in pixels (Q8 / 256);
  * MCD: the h-subset of the n points whose covariance has the smallest
    determinant, h = floor((n + 4) / 2) (the maximal-breakdown size for
    three dimensions, about n / 2);
  * FAST-MCD (Rousseeuw and Van Driessen 1999) approximates it: from many
    random 4-point starts, C-steps (mean and covariance of the current
    subset, Mahalanobis distances of all points, the h closest become the
    next subset) never increase the determinant; two C-steps per start,
    the 10 starts with the lowest determinants iterated until the subset
    stops changing, the lowest determinant wins.  The random starts are an
    input (4 uint32 per start, point = value mod n);
  * the regression from the MCD mean mu and covariance S (1/h normalised):
    B = S_tY / S_tt (the velocity), c = mu_Y - B mu_t (the position at t0),
    Sigma_eps = S_YY - B B^T S_tt;
  * Gather: catalog detections whose position lies within Delta x
    (Euclidean, <=) of c + B t at their own epoch's t.

Rules fixed here where the paper is silent (both sides follow them):
  * the points of a set are ordered by catalog index; ties of distances go
    to the lower position, ties of determinants to the earlier start;
  * a start is dropped when its 4 points repeat or their covariance is
    degenerate, det(S) <= 1e-12 S_tt S_xx S_yy; a subset whose covariance is
    degenerate in that sense ends its C-steps (an exact fit);
  * at most 30 C-steps per refined start and 10 refine/gather rounds;
    fewer than 5 points end the iteration (status too_small).
"""
from __future__ import annotations

import numpy as np

from .features import reference_dt

H_EXTRA = 4       # h = (n + H_EXTRA) // 2
N_BEST = 10       # starts refined to convergence
MAX_CSTEPS = 30
MAX_ROUNDS = 10
MIN_POINTS = 5
DEGENERATE = 1e-12

STATUS_CONVERGED = 0
STATUS_MAX_ROUNDS = 1
STATUS_TOO_SMALL = 2
STATUS_NO_START = 3


def h_of(n: int) -> int:
    return (n + H_EXTRA) // 2


def points(x_q8, y_q8, epoch, t_q16, idx):
    """z = (t h since t0, x px, y px) of the catalog detections idx."""
    ea = np.asarray(epoch, dtype=np.int64)
    d = reference_dt(t_q16, ea, len(t_q16))
    idx = np.asarray(idx, dtype=np.int64)
    t = d[ea[idx]].astype(np.float64) / 65536.0
    x = np.asarray(x_q8, dtype=np.float64)[idx] / 256.0
    y = np.asarray(y_q8, dtype=np.float64)[idx] / 256.0
    return np.stack([t, x, y], axis=1)


def mean_cov(z):
    """Mean and covariance (normalised by the number of points)."""
    mu = z.mean(axis=0)
    c = z - mu
    return mu, (c.T @ c) / z.shape[0]


def degenerate(S) -> bool:
    return np.linalg.det(S) <= DEGENERATE * S[0, 0] * S[1, 1] * S[2, 2]


def c_step(z, subset, h):
    """One C-step: from the subset's mean and covariance, the h points of
    smallest Mahalanobis distance (ties to the lower position)."""
    mu, S = mean_cov(z[subset])
    diff = z - mu
    d2 = np.einsum("ij,jk,ik->i", diff, np.linalg.inv(S), diff)
    return np.sort(np.argsort(d2, kind="stable")[:h])


def _run(z, subset, h, steps):
    """C-steps from a subset: (final subset, its determinant)."""
    for _ in range(steps):
        mu, S = mean_cov(z[subset])
        if degenerate(S):  # an exact fit: no further step
            break
        nxt = c_step(z, subset, h)
        if np.array_equal(nxt, subset):
            break
        subset = nxt
    return subset, float(np.linalg.det(mean_cov(z[subset])[1]))


def fast_mcd(z, starts):
    """(subset positions, mean, covariance) of FAST-MCD, or None when no
    start survives."""
    n = z.shape[0]
    h = h_of(n)
    first = []
    for s, r in enumerate(np.asarray(starts, dtype=np.uint64)):
        j = (r % np.uint64(n)).astype(np.int64)
        if len(np.unique(j)) < 4:
            continue
        _, S0 = mean_cov(z[j])
        if degenerate(S0):
            continue
        # the first C-step goes from the 4-point start to h points
        mu0 = z[j].mean(axis=0)
        diff = z - mu0
        d2 = np.einsum("ij,jk,ik->i", diff, np.linalg.inv(S0), diff)
        sub = np.sort(np.argsort(d2, kind="stable")[:h])
        sub, det = _run(z, sub, h, 1)  # the second C-step
        first.append((det, s, sub))
    if not first:
        return None
    first.sort(key=lambda a: (a[0], a[1]))
    best = None
    for det0, s, sub in first[:N_BEST]:
        sub, det = _run(z, sub, h, MAX_CSTEPS)
        if best is None or det < best[0]:
            best = (det, s, sub)
    sub = best[2]
    mu, S = mean_cov(z[sub])
    return sub, mu, S


def regress(mu, S):
    """B (velocity px/h), c (position px at t0), Sigma_eps (2x2)."""
    B = S[0, 1:] / S[0, 0]
    c = mu[1:] - B * mu[0]
    sig = S[1:, 1:] - np.outer(B, B) * S[0, 0]
    return B, c, sig


def gather(x_q8, y_q8, epoch, t_q16, B, c, dx_px):
    """Catalog indices within dx_px of the line c + B t (ascending)."""
    z = points(x_q8, y_q8, epoch, t_q16, np.arange(len(x_q8)))
    px = c[0] + B[0] * z[:, 0]
    py = c[1] + B[1] * z[:, 0]
    r2 = (z[:, 1] - px) ** 2 + (z[:, 2] - py) ** 2
    return np.nonzero(r2 <= dx_px * dx_px)[0]


def refine_cluster(x_q8, y_q8, epoch, t_q16, members, starts, dx_px):
    """Steps 4-6 for one cluster (catalog indices): dict with the fit of the
    last round, the gathered set, the rounds taken and a status."""
    cur = np.sort(np.asarray(members, dtype=np.int64))
    out = {"status": STATUS_TOO_SMALL, "rounds": 0, "gathered": cur, "subset": None,
           "B": None, "c": None, "sigma": None}
    for rnd in range(1, MAX_ROUNDS + 1):
        if len(cur) < MIN_POINTS:
            out["status"] = STATUS_TOO_SMALL
            return out
        z = points(x_q8, y_q8, epoch, t_q16, cur)
        fit = fast_mcd(z, starts)
        if fit is None:
            out["status"] = STATUS_NO_START
            return out
        sub, mu, S = fit
        B, c, sig = regress(mu, S)
        nxt = gather(x_q8, y_q8, epoch, t_q16, B, c, dx_px)
        out.update(rounds=rnd, subset=cur[sub], B=B, c=c, sigma=sig, gathered=nxt)
        if np.array_equal(nxt, cur):
            out["status"] = STATUS_CONVERGED
            return out
        cur = nxt
    out["status"] = STATUS_MAX_ROUNDS
    return out

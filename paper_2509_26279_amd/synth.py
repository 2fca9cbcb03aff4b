"""Seeded synthetic detection catalogs for the catalog shift-and-stack search.

This module only *makes inputs*: noise detections, injected linear movers
(the motion model of Sec. 2, eqs. 1-2) and the search parameters that go
with each workload.  It contains none of the search's own arithmetic (no
projection to the reference epoch, no binning, no counting, no threshold
rule), so that the CPU oracle and the GPU library can both be fed from it
without sharing any of the method.

Input quantisation (the only place floating point meets the integer
catalog):
  * positions: Q8 pixels, ``x_q8 = floor(256 * x_px)`` (int32);
  * times:     Q16 hours, ``t_q16 = round_half_even(65536 * t_hours)`` (int64);
  * velocities handed to a search are Q8 px/h integers (built elsewhere).

Workloads (all detections shuffled with the workload seed):
  * ``tiny``  - 512x512 px, 20 epochs over 2 h, 2000 uniform noise
    detections, 5 movers |v| <= 20 px/h present in exactly 16 of 20 epochs,
    0.5 px jitter; 4 px bins; threshold 12; 21x21 box grid over +-20 px/h.
  * ``wide``  - 2048x4096 px, 100 epochs over 4 h, 3000 noise detections per
    epoch, 200 movers with speed U(20,400) px/h heading within 30 deg of -x,
    per-mover detection probability U(0.3,0.8); 4 px bins; threshold 25;
    sector grid (20..400 px/h, 180 +- 30 deg).
  * ``fast``  - same chip and noise law, 60 epochs over 2 h, 500 movers with
    speed U(20,5000) px/h in any direction; 16 px bins; disk grid to
    5000 px/h; threshold from the false-positive rule of Sec. 2.2.
  * ``night`` - 64 chips with log-uniform detection counts 5e4..5e5 and
    epoch counts U{40..120}, each chip drawn as a ``wide``- or
    ``fast``-style search (seeded coin).
  * ``faint`` - the fast chip's noise law with 400 faint movers whose
    detections come from their flux: true SNR mu ~ U(1.5, 4), each epoch's
    measured SNR ~ N(mu, 1), kept when it reaches 3; noise SNR follows the
    standard normal tail above 3 (a detector's false peaks); speeds
    U(20, 600) px/h, disk grid to 600 px/h, 16 px bins.

Detection SNR follows 3 + |N(0,1)| for noise and movers alike in every
workload but ``faint``, so that SNR alone cannot separate them there.
``likelihood_weights`` turns SNRs into the integer weights of a weighted
vote (an input, like the catalog itself).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Q_POS = 256          # Q8 pixels
Q_TIME = 65536       # Q16 hours
T_ORIGIN_H = 1000.0  # arbitrary clock origin: the search must not assume t=0 at the first epoch


@dataclass
class GridSpec:
    """Search-region description handed to the grid builder (px/h, degrees)."""
    shape: str                      # "box" | "disk" | "annulus" | "sector"
    vmin: float = 0.0               # box: vx min; disk/annulus/sector: min speed
    vmax: float = 0.0               # box: vx max; disk/annulus/sector: max speed
    vy_min: float = 0.0             # box only
    vy_max: float = 0.0             # box only
    angle_deg: float = 0.0          # sector centre direction
    half_width_deg: float = 0.0     # sector half opening


@dataclass
class Workload:
    name: str
    seed: int
    width_px: int
    height_px: int
    n_epochs: int
    span_h: float
    bin_px: float
    n_min: int
    count_dtype: str                # "u8" | "u16"
    grid: GridSpec
    x_q8: np.ndarray = field(repr=False, default=None)
    y_q8: np.ndarray = field(repr=False, default=None)
    epoch: np.ndarray = field(repr=False, default=None)
    snr: np.ndarray = field(repr=False, default=None)
    t_q16: np.ndarray = field(repr=False, default=None)
    is_mover: np.ndarray = field(repr=False, default=None)   # per detection: mover id or -1
    truth: dict = field(repr=False, default=None)

    @property
    def n(self) -> int:
        return int(self.x_q8.shape[0])

    @property
    def binw_q8(self) -> int:
        return int(round(self.bin_px * Q_POS))

    @property
    def span_q16(self) -> int:
        return int(self.t_q16.max() - self.t_q16.min())

    @property
    def extent_q8(self) -> tuple:
        """Declared detector footprint [x0, x1) x [y0, y1) in Q8."""
        return (0, self.width_px * Q_POS, 0, self.height_px * Q_POS)


def quantize_pos(px: np.ndarray) -> np.ndarray:
    return np.floor(np.asarray(px, dtype=np.float64) * Q_POS).astype(np.int32)


def quantize_time(hours: np.ndarray) -> np.ndarray:
    return np.rint(np.asarray(hours, dtype=np.float64) * Q_TIME).astype(np.int64)


def _epoch_hours(n_epochs: int, span_h: float) -> np.ndarray:
    if n_epochs == 1:
        return np.zeros(1)
    return np.arange(n_epochs, dtype=np.float64) * (span_h / (n_epochs - 1))


def _movers(rng, n_movers, speed_law, angle_law, presence_law, width, height,
            t_h, jitter_px):
    """Linear movers x(t) = x_mid + v (t - t_mid) (Sec. 2, eqs. 1-2)."""
    n_ep = t_h.shape[0]
    t_mid = 0.5 * (t_h[0] + t_h[-1])
    xs, ys, es, ids = [], [], [], []
    truth = {"x_mid": [], "y_mid": [], "t_mid_h": t_mid, "vx": [], "vy": [],
             "present": []}
    for m in range(n_movers):
        speed = speed_law(rng)
        ang = angle_law(rng)
        vx, vy = speed * math.cos(ang), speed * math.sin(ang)
        xm, ym = rng.uniform(0, width), rng.uniform(0, height)
        present = presence_law(rng, n_ep)
        jx = rng.normal(0.0, jitter_px, n_ep)
        jy = rng.normal(0.0, jitter_px, n_ep)
        px = xm + vx * (t_h - t_mid) + jx
        py = ym + vy * (t_h - t_mid) + jy
        on = present & (px >= 0) & (px < width) & (py >= 0) & (py < height)
        e_on = np.nonzero(on)[0]
        xs.append(px[e_on]); ys.append(py[e_on]); es.append(e_on)
        ids.append(np.full(e_on.shape[0], m))
        truth["x_mid"].append(xm); truth["y_mid"].append(ym)
        truth["vx"].append(vx); truth["vy"].append(vy)
        truth["present"].append(on)
    for k in ("x_mid", "y_mid", "vx", "vy"):
        truth[k] = np.asarray(truth[k], dtype=np.float64)
    truth["present"] = (np.asarray(truth["present"], dtype=bool)
                        if n_movers else np.zeros((0, n_ep), dtype=bool))
    cat = lambda a, dt: (np.concatenate(a).astype(dt) if a else np.zeros(0, dt))
    return cat(xs, np.float64), cat(ys, np.float64), cat(es, np.int64), \
        cat(ids, np.int64), truth


def _assemble(rng, wl: Workload, noise_x, noise_y, noise_e, mov, snr=None):
    mx, my, me, mid, truth = mov
    x = np.concatenate([noise_x, mx])
    y = np.concatenate([noise_y, my])
    e = np.concatenate([noise_e, me])
    ids = np.concatenate([np.full(noise_x.shape[0], -1, np.int64), mid])
    if snr is None:
        snr = 3.0 + np.abs(rng.normal(0.0, 1.0, x.shape[0]))
    perm = rng.permutation(x.shape[0])
    wl.x_q8 = quantize_pos(x[perm])
    wl.y_q8 = quantize_pos(y[perm])
    wl.epoch = e[perm].astype(np.uint8)
    wl.snr = snr[perm].astype(np.float32)
    wl.is_mover = ids[perm].astype(np.int32)
    wl.truth = truth
    return wl


def _presence_fixed(k):
    def law(rng, n_ep):
        on = np.zeros(n_ep, dtype=bool)
        on[rng.choice(n_ep, size=k, replace=False)] = True
        return on
    return law


def _presence_bernoulli(lo, hi):
    def law(rng, n_ep):
        p = rng.uniform(lo, hi)
        return rng.uniform(0.0, 1.0, n_ep) < p
    return law


def _disk_speed(vmax):
    return lambda rng: vmax * math.sqrt(rng.uniform(0.0, 1.0))


def _uniform(lo, hi):
    return lambda rng: rng.uniform(lo, hi)


# Threshold of the fast-mover workload: the smallest N_min whose expected number
# of pure-noise candidates over the realised grid is at most 100 (Sec. 2.2,
# eq. for N_stacks with Poisson noise per epoch).  Fixed here as a number; the
# rule that produces it lives with the search parameters and is checked by tests.
FAST_N_MIN = 23


def make_tiny(seed: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    wl = Workload("tiny", seed, 512, 512, 20, 2.0, 4.0, 12, "u8",
                  GridSpec("box", -20.0, 20.0, -20.0, 20.0))
    t_h = _epoch_hours(wl.n_epochs, wl.span_h)
    wl.t_q16 = quantize_time(T_ORIGIN_H + t_h)
    nx = rng.uniform(0, wl.width_px, 2000)
    ny = rng.uniform(0, wl.height_px, 2000)
    ne = rng.integers(0, wl.n_epochs, 2000)
    mov = _movers(rng, 5, _disk_speed(20.0), _uniform(0.0, 2 * math.pi),
                  _presence_fixed(16), wl.width_px, wl.height_px, t_h, 0.5)
    return _assemble(rng, wl, nx, ny, ne, mov)


def _chip(rng, wl: Workload, noise_per_epoch, n_movers, speed_law, angle_law):
    t_h = _epoch_hours(wl.n_epochs, wl.span_h)
    wl.t_q16 = quantize_time(T_ORIGIN_H + t_h)
    if np.ndim(noise_per_epoch) == 0:
        counts = np.full(wl.n_epochs, int(noise_per_epoch))
    else:
        counts = np.asarray(noise_per_epoch)
    tot = int(counts.sum())
    nx = rng.uniform(0, wl.width_px, tot)
    ny = rng.uniform(0, wl.height_px, tot)
    ne = np.repeat(np.arange(wl.n_epochs), counts)
    mov = _movers(rng, n_movers, speed_law, angle_law,
                  _presence_bernoulli(0.3, 0.8), wl.width_px, wl.height_px,
                  t_h, 0.5)
    return _assemble(rng, wl, nx, ny, ne, mov)


def make_wide(seed: int = 2, n_epochs: int = 100, noise_per_epoch=3000,
              n_min: int = 25) -> Workload:
    rng = np.random.default_rng(seed)
    wl = Workload("wide", seed, 2048, 4096, n_epochs, 4.0, 4.0, n_min, "u8",
                  GridSpec("sector", 20.0, 400.0, angle_deg=180.0,
                           half_width_deg=30.0))
    return _chip(rng, wl, noise_per_epoch, 200, _uniform(20.0, 400.0),
                 _uniform(math.pi - math.pi / 6, math.pi + math.pi / 6))


def make_fast(seed: int = 3, n_epochs: int = 60, noise_per_epoch=3000,
              n_min: int = FAST_N_MIN) -> Workload:
    rng = np.random.default_rng(seed)
    wl = Workload("fast", seed, 2048, 4096, n_epochs, 2.0, 16.0, n_min, "u16",
                  GridSpec("disk", 0.0, 5000.0))
    return _chip(rng, wl, noise_per_epoch, 500, _uniform(20.0, 5000.0),
                 _uniform(0.0, 2 * math.pi))


def make_faint(seed: int = 500, n_epochs: int = 60, noise_per_epoch: int = 3000,
               n_movers: int = 400, snr_lo: float = 1.5, snr_hi: float = 4.0) -> Workload:
    """Faint movers whose detections follow from their flux (see the module
    header).  truth["snr"] holds each mover's true SNR; n_min is left at 0
    for the search to set."""
    from scipy.stats import norm
    rng = np.random.default_rng(seed)
    wl = Workload("faint", seed, 2048, 4096, n_epochs, 2.0, 16.0, 0, "u16",
                  GridSpec("disk", 0.0, 600.0))
    t_h = _epoch_hours(wl.n_epochs, wl.span_h)
    wl.t_q16 = quantize_time(T_ORIGIN_H + t_h)
    tot = noise_per_epoch * n_epochs
    nx = rng.uniform(0, wl.width_px, tot)
    ny = rng.uniform(0, wl.height_px, tot)
    ne = np.repeat(np.arange(n_epochs), noise_per_epoch)
    # the standard normal tail above 3, by its inverse survival function
    noise_snr = norm.isf(rng.uniform(0.0, 1.0, tot) * norm.sf(3.0))
    drawn = []  # per mover: true SNR and the measured SNR of every epoch

    def presence(r, n_ep):
        mu = r.uniform(snr_lo, snr_hi)
        s = mu + r.normal(0.0, 1.0, n_ep)
        drawn.append((mu, s))
        return s >= 3.0
    mov = _movers(rng, n_movers, _uniform(20.0, 600.0), _uniform(0.0, 2 * math.pi), presence,
                  wl.width_px, wl.height_px, t_h, 0.5)
    mids, mes = mov[3], mov[2]
    mover_snr = np.array([drawn[m][1][e] for m, e in zip(mids, mes)], dtype=np.float64)
    wl = _assemble(rng, wl, nx, ny, ne, mov, snr=np.concatenate([noise_snr, mover_snr]))
    wl.truth["snr"] = np.array([d[0] for d in drawn], dtype=np.float64)
    return wl


def likelihood_weights(snr, scale: float = 4.0) -> np.ndarray:
    """Integer weights for a weighted vote: the log-likelihood ratio of a
    detection of measured SNR s against noise, maximised over the source's
    flux (s^2 / 2), times `scale`, rounded and capped at 255."""
    s = np.asarray(snr, dtype=np.float64)
    return np.minimum(np.rint(scale * s * s / 2.0), 255).astype(np.uint8)


def mcd_starts(seed: int = 7, n_starts: int = 500) -> np.ndarray:
    """The random draws of FAST-MCD's starting subsets, as an input: 4
    uint32 per start (a start takes the points value mod n)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 32, (n_starts, 4), dtype=np.uint64).astype(np.uint32)


def night_chip_params(seed: int = 4, n_chips: int = 64):
    """Per-chip draws of the batched night: style, detection count, epochs."""
    out = []
    for c in range(n_chips):
        rng = np.random.default_rng(seed * 1000 + c)
        style = "wide" if rng.uniform() < 0.5 else "fast"
        n_det = int(math.floor(math.exp(rng.uniform(math.log(5e4), math.log(5e5)))))
        n_ep = int(rng.integers(40, 121))
        out.append({"chip": c, "seed": seed * 1000 + c, "style": style,
                    "n_det": n_det, "n_epochs": n_ep})
    return out


def make_night_chip(p: dict, fast_n_min: int) -> Workload:
    """One chip of the batched night (noise spread evenly over its epochs)."""
    n_ep = p["n_epochs"]
    base, rem = divmod(p["n_det"], n_ep)
    per = np.full(n_ep, base)
    per[:rem] += 1
    if p["style"] == "wide":
        wl = make_wide(p["seed"], n_ep, per, n_min=int(round(0.25 * n_ep)))
    else:
        wl = make_fast(p["seed"], n_ep, per, n_min=fast_n_min)
    wl.name = f"night{p['chip']}-{p['style']}"
    return wl


def make_random_small(seed: int, n: int = 60, n_epochs: int = 6,
                      extent_q8: int = 40 * 256, vmax_q8: int = 6 * 256,
                      n_v: int = 9, binw_q8: int = 3 * 256,
                      allow_negative: bool = True, dup_frac: float = 0.2):
    """Tiny adversarial catalog for brute-force checks.

    Negative coordinates and velocities, detections exactly on bin edges and
    same-epoch duplicates are all drawn on purpose.  Returns a dict of plain
    arrays (x_q8, y_q8, epoch, t_q16, v_q8 [n_v,2], binw_q8).
    """
    rng = np.random.default_rng(seed)
    lo = -extent_q8 if allow_negative else 0
    x = rng.integers(lo, extent_q8, n).astype(np.int64)
    y = rng.integers(lo, extent_q8, n).astype(np.int64)
    # a fraction exactly on bin edges
    k = n // 5
    x[:k] = (x[:k] // binw_q8) * binw_q8
    y[k:2 * k] = (y[k:2 * k] // binw_q8) * binw_q8
    e = rng.integers(0, n_epochs, n)
    # duplicates: copy some detections to the same epoch and position
    nd = int(dup_frac * n)
    src = rng.integers(0, n, nd)
    dst = rng.integers(0, n, nd)
    x[dst], y[dst], e[dst] = x[src], y[src], e[src]
    t = np.sort(rng.integers(0, 3 * Q_TIME, n_epochs)).astype(np.int64)
    t += rng.integers(-10 ** 6, 10 ** 6)
    v = rng.integers(-vmax_q8, vmax_q8 + 1, (n_v, 2)).astype(np.int64)
    v[0] = 0
    return {"x_q8": x.astype(np.int32), "y_q8": y.astype(np.int32),
            "epoch": e.astype(np.uint8), "t_q16": t, "v_q8": v.astype(np.int32),
            "binw_q8": int(binw_q8)}

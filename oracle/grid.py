"""Velocity-grid oracle (NumPy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 2 shows that a trial velocity keeps an object's projected detections
inside one cluster of size Delta x whenever each velocity component is off
by at most Delta x / Delta t (the tolerance derived right after
Delta x = Delta t Delta v).  A complete blind search therefore tests a
lattice of velocities with that spacing; eq. (v_size) counts it.

Reading used here (all integers in Q8 px/h):
  * spacing s = floor(binw_q8 * 65536 / span_q16), span = Delta t in Q16 h;
  * lattice points p = (i s, j s) for integers i, j;
  * p is kept when its closed cell [p - s/2, p + s/2]^2 meets the search
    region, so every velocity of the region lies within s/2 per axis of a
    kept point;
  * order: by (j, i), i.e. vy ascending then vx ascending (row-major).

Region tests are done in doubled Q8 units (cell corners 2 p +- s are
integers) and in IEEE double for the region's own parameters.
Regions: box, disk (|v| <= vmax), annulus (vmin <= |v| <= vmax) and sector
(annulus intersected with directions angle +- half_width, half_width < 90 deg).
For the sector the cell must meet the annulus and meet the wedge; the wedge
test is exact for a convex cone (a corner inside, the apex inside, or one of
the two boundary rays crossing the cell).
"""
from __future__ import annotations

import math

import numpy as np


def spacing_q8(binw_q8: int, span_q16: int) -> int:
    return (int(binw_q8) * 65536) // int(span_q16)


def _nearest_sq(a1, a2):
    """Squared distance from 0 to the interval [a1, a2], elementwise."""
    d = np.where(a1 > 0, a1, np.where(a2 < 0, -a2, 0.0))
    return d * d


def _farthest_sq(a1, a2):
    d = np.maximum(np.abs(a1), np.abs(a2))
    return d * d


def _in_cone(qx, qy, d1, d2):
    c1 = d1[0] * qy - d1[1] * qx          # cross(d1, q)
    c2 = qx * d2[1] - qy * d2[0]          # cross(q, d2)
    return (c1 >= 0.0) & (c2 >= 0.0)


def _ray_hits(d, a1, a2, b1, b2):
    """Does the ray t*d, t >= 0, meet the box [a1,a2]x[b1,b2]? (slab test)"""
    n = a1.shape[0]
    t_in = np.zeros(n)
    t_out = np.full(n, np.inf)
    ok = np.ones(n, dtype=bool)
    for dc, lo, hi in ((d[0], a1, a2), (d[1], b1, b2)):
        if dc == 0.0:
            ok &= (lo <= 0.0) & (hi >= 0.0)
        else:
            t1 = lo / dc
            t2 = hi / dc
            t_in = np.maximum(t_in, np.minimum(t1, t2))
            t_out = np.minimum(t_out, np.maximum(t1, t2))
    return ok & (t_in <= t_out)


def cell_meets(shape, spec, a1, a2, b1, b2):
    """Vectorised region test on cells [a1,a2]x[b1,b2] in doubled Q8 units."""
    k = 512.0  # px/h -> doubled Q8
    if shape == "box":
        return ((a1 <= k * spec["vmax"]) & (a2 >= k * spec["vmin"])
                & (b1 <= k * spec["vy_max"]) & (b2 >= k * spec["vy_min"]))
    near = _nearest_sq(a1, a2) + _nearest_sq(b1, b2)
    rmax = k * spec["vmax"]
    ok = near <= rmax * rmax
    if shape == "disk":
        return ok
    far = _farthest_sq(a1, a2) + _farthest_sq(b1, b2)
    rmin = k * spec["vmin"]
    ok &= far >= rmin * rmin
    if shape == "annulus":
        return ok
    if shape != "sector":
        raise ValueError(shape)
    th = math.radians(spec["angle_deg"])
    hw = math.radians(spec["half_width_deg"])
    d1 = (math.cos(th - hw), math.sin(th - hw))
    d2 = (math.cos(th + hw), math.sin(th + hw))
    wedge = np.zeros(a1.shape[0], dtype=bool)
    for cx, cy in ((a1, b1), (a2, b1), (a1, b2), (a2, b2)):
        wedge |= _in_cone(cx, cy, d1, d2)
    wedge |= (a1 <= 0) & (a2 >= 0) & (b1 <= 0) & (b2 >= 0)
    wedge |= _ray_hits(d1, a1, a2, b1, b2)
    wedge |= _ray_hits(d2, a1, a2, b1, b2)
    return ok & wedge


def build_grid(spec: dict, s_q8: int) -> np.ndarray:
    """Kept lattice points as int32 [n, 2] (vx, vy) in Q8 px/h, row-major (vy, vx)."""
    shape = spec["shape"]
    if shape == "box":
        lo_x, hi_x = spec["vmin"], spec["vmax"]
        lo_y, hi_y = spec["vy_min"], spec["vy_max"]
    else:
        lo_x = lo_y = -spec["vmax"]
        hi_x = hi_y = spec["vmax"]
    s = int(s_q8)
    i0 = int(math.floor(lo_x * 256.0 / s)) - 2
    i1 = int(math.ceil(hi_x * 256.0 / s)) + 2
    j0 = int(math.floor(lo_y * 256.0 / s)) - 2
    j1 = int(math.ceil(hi_y * 256.0 / s)) + 2
    ii, jj = np.meshgrid(np.arange(i0, i1 + 1, dtype=np.int64),
                         np.arange(j0, j1 + 1, dtype=np.int64))  # rows = j
    ii = ii.ravel()
    jj = jj.ravel()
    a1 = (2 * ii * s - s).astype(np.float64)
    a2 = (2 * ii * s + s).astype(np.float64)
    b1 = (2 * jj * s - s).astype(np.float64)
    b2 = (2 * jj * s + s).astype(np.float64)
    keep = cell_meets(shape, spec, a1, a2, b1, b2)
    out = np.stack([ii[keep] * s, jj[keep] * s], axis=1)
    return out.astype(np.int32)

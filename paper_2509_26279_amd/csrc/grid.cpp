// Velocity grid of the blind search (Sec. 2): an object's projected
// detections stay within one cluster of size Delta x when each velocity
// component is off by at most Delta x / Delta t, so the search tests a square
// lattice with that spacing; eq. (v_size) gives its size for a box.
//
// A lattice point p = (i s, j s) is kept when its closed cell
// [p - s/2, p + s/2]^2 meets the search region: then every velocity of the
// region lies within s/2 per axis of a kept point.  Cell corners are handled
// in doubled Q8 units (2 p +- s, exact integers held in doubles); the region's
// own parameters are doubles.  Build with floating-point contraction off so
// that every comparison is the plain IEEE result.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sas.h"

namespace sas {
void set_error(const std::string &msg);
}

namespace {

constexpr double kDoubledQ8 = 512.0;  // px/h -> doubled Q8 px/h

struct Cell {
    double a1, a2, b1, b2;  // x and y extents, doubled Q8
};

double sq_nearest(double lo, double hi) {
    const double d = lo > 0.0 ? lo : (hi < 0.0 ? -hi : 0.0);
    return d * d;
}

double sq_farthest(double lo, double hi) {
    const double d = std::fabs(lo) > std::fabs(hi) ? std::fabs(lo) : std::fabs(hi);
    return d * d;
}

bool inside_cone(double qx, double qy, const double d1[2], const double d2[2]) {
    const double c1 = d1[0] * qy - d1[1] * qx;  // d1 x q
    const double c2 = qx * d2[1] - qy * d2[0];  // q x d2
    return c1 >= 0.0 && c2 >= 0.0;
}

// Slab test of the ray t d (t >= 0) against the cell.
bool ray_meets(const double d[2], const Cell &c) {
    double t_in = 0.0, t_out = INFINITY;
    const double lo[2] = {c.a1, c.b1}, hi[2] = {c.a2, c.b2};
    for (int ax = 0; ax < 2; ++ax) {
        if (d[ax] == 0.0) {
            if (!(lo[ax] <= 0.0 && hi[ax] >= 0.0)) return false;
        } else {
            const double t1 = lo[ax] / d[ax], t2 = hi[ax] / d[ax];
            const double tn = t1 < t2 ? t1 : t2, tf = t1 < t2 ? t2 : t1;
            if (tn > t_in) t_in = tn;
            if (tf < t_out) t_out = tf;
        }
    }
    return t_in <= t_out;
}

struct Region {
    int shape;
    double vmin, vmax, vy_min, vy_max;
    double d1[2], d2[2];

    bool meets(const Cell &c) const {
        if (shape == SAS_GRID_BOX)
            return c.a1 <= kDoubledQ8 * vmax && c.a2 >= kDoubledQ8 * vmin &&
                   c.b1 <= kDoubledQ8 * vy_max && c.b2 >= kDoubledQ8 * vy_min;
        const double rmax = kDoubledQ8 * vmax;
        if (!(sq_nearest(c.a1, c.a2) + sq_nearest(c.b1, c.b2) <= rmax * rmax)) return false;
        if (shape == SAS_GRID_DISK) return true;
        const double rmin = kDoubledQ8 * vmin;
        if (!(sq_farthest(c.a1, c.a2) + sq_farthest(c.b1, c.b2) >= rmin * rmin)) return false;
        if (shape == SAS_GRID_ANNULUS) return true;
        // sector: the cell must also meet the wedge between the two rays
        const double cx[4] = {c.a1, c.a2, c.a1, c.a2}, cy[4] = {c.b1, c.b1, c.b2, c.b2};
        for (int k = 0; k < 4; ++k)
            if (inside_cone(cx[k], cy[k], d1, d2)) return true;
        if (c.a1 <= 0.0 && c.a2 >= 0.0 && c.b1 <= 0.0 && c.b2 >= 0.0) return true;
        return ray_meets(d1, c) || ray_meets(d2, c);
    }
};

}  // namespace

extern "C" sas_status sas_grid_spacing(int32_t binw_q8, int64_t span_q16, int32_t *spacing_out) {
    if (!spacing_out || binw_q8 <= 0 || span_q16 <= 0) {
        sas::set_error("sas_grid_spacing: need binw_q8 > 0, span_q16 > 0 and an output pointer");
        return SAS_E_INVALID;
    }
    const int64_t s = ((int64_t)binw_q8 * 65536) / span_q16;
    if (s < 1 || s > (int64_t)1 << 30) {
        sas::set_error("sas_grid_spacing: spacing outside [1, 2^30] Q8 px/h");
        return SAS_E_INVALID;
    }
    *spacing_out = (int32_t)s;
    return SAS_OK;
}

extern "C" sas_status sas_build_grid(const sas_grid_spec *spec, int32_t *v_out_host, int64_t cap,
                                     int64_t *n_out) {
    if (!spec || !n_out || cap < 0) {
        sas::set_error("sas_build_grid: null spec/n_out or negative cap");
        return SAS_E_INVALID;
    }
    int32_t s = spec->spacing_q8;
    if (s == 0) {
        const sas_status st = sas_grid_spacing(spec->binw_q8, spec->span_q16, &s);
        if (st != SAS_OK) return st;
    }
    if (s < 1) {
        sas::set_error("sas_build_grid: spacing must be >= 1");
        return SAS_E_INVALID;
    }
    Region r{};
    r.shape = spec->shape;
    r.vmin = spec->vmin;
    r.vmax = spec->vmax;
    r.vy_min = spec->vy_min;
    r.vy_max = spec->vy_max;
    double xlo, xhi, ylo, yhi;
    switch (spec->shape) {
    case SAS_GRID_BOX:
        if (!(spec->vmin <= spec->vmax && spec->vy_min <= spec->vy_max)) {
            sas::set_error("sas_build_grid: box needs vmin <= vmax and vy_min <= vy_max");
            return SAS_E_INVALID;
        }
        xlo = spec->vmin; xhi = spec->vmax; ylo = spec->vy_min; yhi = spec->vy_max;
        break;
    case SAS_GRID_DISK:
    case SAS_GRID_ANNULUS:
    case SAS_GRID_SECTOR:
        if (!(spec->vmax >= 0.0 && spec->vmin >= 0.0 && spec->vmin <= spec->vmax)) {
            sas::set_error("sas_build_grid: need 0 <= vmin <= vmax");
            return SAS_E_INVALID;
        }
        if (spec->shape == SAS_GRID_SECTOR &&
            !(spec->half_width_deg > 0.0 && spec->half_width_deg < 90.0)) {
            sas::set_error("sas_build_grid: sector half width must be in (0, 90) degrees");
            return SAS_E_INVALID;
        }
        xlo = ylo = -spec->vmax;
        xhi = yhi = spec->vmax;
        break;
    default:
        sas::set_error("sas_build_grid: unknown shape");
        return SAS_E_INVALID;
    }
    if (!(std::fabs(xlo) < 4.0e6 && std::fabs(xhi) < 4.0e6 && std::fabs(ylo) < 4.0e6 &&
          std::fabs(yhi) < 4.0e6)) {
        sas::set_error("sas_build_grid: speeds must stay below 4e6 px/h");
        return SAS_E_INVALID;
    }
    if (spec->shape == SAS_GRID_SECTOR) {
        const double deg = M_PI / 180.0;
        const double th = spec->angle_deg * deg, hw = spec->half_width_deg * deg;
        r.d1[0] = std::cos(th - hw);
        r.d1[1] = std::sin(th - hw);
        r.d2[0] = std::cos(th + hw);
        r.d2[1] = std::sin(th + hw);
    }
    const int64_t i0 = (int64_t)std::floor(xlo * 256.0 / s) - 2;
    const int64_t i1 = (int64_t)std::ceil(xhi * 256.0 / s) + 2;
    const int64_t j0 = (int64_t)std::floor(ylo * 256.0 / s) - 2;
    const int64_t j1 = (int64_t)std::ceil(yhi * 256.0 / s) + 2;
    if ((i1 - i0 + 1) * (j1 - j0 + 1) > ((int64_t)1 << 34)) {
        sas::set_error("sas_build_grid: lattice too large");
        return SAS_E_INVALID;
    }
    int64_t count = 0;
    const bool write = v_out_host != nullptr;
    for (int64_t j = j0; j <= j1; ++j) {
        for (int64_t i = i0; i <= i1; ++i) {
            const Cell c{(double)(2 * i * s - s), (double)(2 * i * s + s), (double)(2 * j * s - s),
                         (double)(2 * j * s + s)};
            if (!r.meets(c)) continue;
            if (write && count < cap) {
                v_out_host[2 * count] = (int32_t)(i * s);
                v_out_host[2 * count + 1] = (int32_t)(j * s);
            }
            ++count;
        }
    }
    *n_out = count;
    if (!write) return cap == 0 ? SAS_OK : SAS_E_OVERFLOW;
    if (count > cap) {
        sas::set_error("sas_build_grid: output capacity too small; *n_out holds the count");
        return SAS_E_OVERFLOW;
    }
    return SAS_OK;
}

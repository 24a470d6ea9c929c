// One entry of the completed double-layer operator, evaluated on the device.
// Section 2.1 gives the double-layer kernel (1/pi)(r.n) r r^T / rho^4;
// Section 2.2 the Nystrom weights; the jump -1/2, the smooth diagonal limit
// w kappa/(2 pi) t t^T, the wall's rank-one flux term and the pore
// Stokeslet/rotlet completion with its constraint rows remove the double
// layer's null space (Section 2.1 notes that it can be removed).
#pragma once

#include "common.hpp"

namespace sbie {

struct GeomView {
  int64_t nn;
  int32_t m;
  int64_t wall_start;
  const double *x, *y, *nx, *ny, *w, *kappa, *cx, *cy, *rad;
  const int64_t *off;        // device curve offsets
  const double *wall_len;    // device scalar |Gamma_0|
};

inline GeomView make_view(const sbie_geom *g, const double *wall_len) {
  GeomView v;
  v.nn = g->n_nodes;
  v.m = g->n_pores;
  v.wall_start = g->curve_off[g->n_pores];
  v.x = g->x; v.y = g->y; v.nx = g->nx; v.ny = g->ny; v.w = g->w;
  v.kappa = g->kappa; v.cx = g->cx; v.cy = g->cy; v.rad = g->radius;
  v.off = g->curve_off_dev;
  v.wall_len = wall_len;
  return v;
}

__device__ inline double op_entry(const GeomView &g, int64_t r, int64_t c) {
  const int64_t nn = g.nn;
  if (r < 2 * nn) {
    const int64_t i = r < nn ? r : r - nn;
    const int a = r < nn ? 0 : 1;
    if (c < 2 * nn) {
      const int64_t j = c < nn ? c : c - nn;
      const int b = c < nn ? 0 : 1;
      double v;
      if (j != i) {
        const double rx = g.x[i] - g.x[j], ry = g.y[i] - g.y[j];
        const double r2 = rx * rx + ry * ry;
        const double rn = rx * g.nx[j] + ry * g.ny[j];
        const double base = g.w[j] * rn / (kPi * r2 * r2);
        v = base * (a ? ry : rx) * (b ? ry : rx);
      } else {
        const double ta = a ? g.nx[i] : -g.ny[i];
        const double tb = b ? g.nx[i] : -g.ny[i];
        v = g.w[i] * g.kappa[i] * (0.5 / kPi) * ta * tb - (a == b ? 0.5 : 0.0);
      }
      if (i >= g.wall_start && j >= g.wall_start) {
        const double na = a ? g.ny[i] : g.nx[i];
        const double nb = b ? g.ny[j] : g.nx[j];
        v += na * g.w[j] * nb / *g.wall_len;
      }
      return v;
    }
    const int64_t q = c - 2 * nn;
    const int64_t k = q / 3;
    const int comp = (int)(q - 3 * k);
    const double qx = g.x[i] - g.cx[k], qy = g.y[i] - g.cy[k];
    const double q2 = qx * qx + qy * qy;
    if (comp < 2) {
      const double lg = 0.5 * log(q2);
      const double qa = a ? qy : qx;
      const double qb = comp ? qy : qx;
      return (0.25 / kPi) * ((a == comp ? -lg : 0.0) + qa * qb / q2);
    }
    // rotlet column scaled by the pore radius: r_k (q_y, -q_x) / (4 pi q^2)
    const double perp = a ? -qx : qy;
    return (0.25 / kPi) * g.rad[k] * perp / q2;
  }
  const int64_t q = r - 2 * nn;
  const int64_t k = q / 3;
  const int comp = (int)(q - 3 * k);
  if (c >= 2 * nn) return c == r ? -1.0 : 0.0;
  const int64_t j = c < nn ? c : c - nn;
  const int b = c < nn ? 0 : 1;
  if (j < g.off[k] || j >= g.off[k + 1]) return 0.0;
  const double rk = g.rad[k];
  if (comp < 2) return comp == b ? g.w[j] / (2.0 * kPi * rk) : 0.0;
  // (x_j - c_k)_perp = (y_j - cy, -(x_j - cx))
  const double perp = b ? -(g.x[j] - g.cx[k]) : (g.y[j] - g.cy[k]);
  return g.w[j] * perp / (2.0 * kPi * rk * rk);
}

}  // namespace sbie

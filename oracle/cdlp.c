/* Oracle: the completed double-layer operator applied to a vector, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the tests, by the script that writes
 * the stored reference solutions and by the CPU-baseline leg of the
 * benchmark; nothing in the product path may load it.  It shares no code with
 * the GPU library.
 *
 * It is the same operator as the NumPy oracle (oracle/dlp.py), written as a
 * plain double loop so that the large workloads (1e4..1e5 nodes) can be
 * applied on the host's cores in seconds.  One target row at a time, the sum
 * over all sources in index order; no blocking or reordering.
 *
 * Operator (Section 2.1 double-layer kernel, Section 2.2 trapezoid/Nystrom
 * rule; completion and wall rank-one term as in the NumPy oracle):
 *   node rows, component a, with r = x_i - x_j, rho = |r|:
 *     -1/2 sigma_i
 *     + sum_{j != i} w_j / pi * (r . n_j) * r_a * (r . sigma_j) / rho^4
 *     + w_i kappa_i / (2 pi) * t_a (t_i . sigma_i)              (smooth limit)
 *     + [i on wall] n_a,i / |Gamma_0| * sum_{j on wall} w_j n_j . sigma_j
 *     + sum_k [ S(x_i - c_k) lambda_k + r_k R(x_i - c_k) mu_k ]_a
 *   S(r) = (-log rho I + r r^T / rho^2) / (4 pi),  R(r) = (r_y, -r_x) / (4 pi rho^2)
 *   pore rows (pore k):
 *     lambda_a row: 1/(2 pi r_k) sum_{j in k} w_j sigma_a,j - lambda_a,k
 *     mu row:       1/(2 pi r_k^2) sum_{j in k} w_j ((y_j - cy_k) sigma_x,j
 *                                                   - (x_j - cx_k) sigma_y,j) - mu_k
 *
 * Two precisions of the same formulas: REAL = double (plain) and
 * REAL = long double (x87 80-bit: every difference, product and sum carried
 * with a 64-bit significand), the second used to evaluate residuals f - A u
 * whose size is far below |A| |u| (the density on long pipes is ~1e3 times
 * the boundary data, so plain sums cannot resolve a residual of 1e-10 |f|).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define PI_L 3.141592653589793238462643383279502884L

#define DEFINE_APPLY(NAME, REAL, LOG, SIMD, ATTR)                                  \
  ATTR void NAME(int64_t nn, int32_t m, const int64_t *curve_off, const double *x,         \
            const double *y, const double *nx, const double *ny, const double *tx,    \
            const double *ty, const double *w, const double *kappa,                   \
            const double *cx, const double *cy, const double *radius,                 \
            const double *u, double *out) {                                           \
    const double *sx = u, *sy = u + nn, *comp = u + 2 * nn;                           \
    const int64_t w0 = curve_off[m], w1 = curve_off[m + 1];                           \
    const REAL pi = (REAL)PI_L;                                                       \
    REAL wall_len = 0, flux = 0;                                                      \
    for (int64_t j = w0; j < w1; ++j) {                                               \
      wall_len += (REAL)w[j];                                                         \
      flux += (REAL)w[j] * ((REAL)nx[j] * sx[j] + (REAL)ny[j] * sy[j]);               \
    }                                                                                 \
    _Pragma("omp parallel for schedule(dynamic, 64)")                                 \
    for (int64_t i = 0; i < nn; ++i) {                                                \
      REAL ax = 0, ay = 0;                                                            \
      _Pragma(SIMD)                                                                   \
      for (int64_t j = 0; j < nn; ++j) {                                              \
        if (j == i) continue;                                                         \
        REAL rx = (REAL)x[i] - (REAL)x[j];                                            \
        REAL ry = (REAL)y[i] - (REAL)y[j];                                            \
        REAL rho2 = rx * rx + ry * ry;                                                \
        REAL rn = rx * nx[j] + ry * ny[j];                                            \
        REAL rs = rx * sx[j] + ry * sy[j];                                            \
        REAL c = (REAL)w[j] / pi * rn * rs / (rho2 * rho2);                           \
        ax += c * rx;                                                                 \
        ay += c * ry;                                                                 \
      }                                                                               \
      /* jump and smooth diagonal limit */                                            \
      REAL ts = (REAL)tx[i] * sx[i] + (REAL)ty[i] * sy[i];                            \
      REAL d = (REAL)w[i] * kappa[i] / (2 * pi);                                      \
      ax += d * tx[i] * ts - (REAL)0.5 * sx[i];                                       \
      ay += d * ty[i] * ts - (REAL)0.5 * sy[i];                                       \
      /* rank-one wall term */                                                        \
      if (i >= w0 && i < w1) {                                                        \
        ax += (REAL)nx[i] / wall_len * flux;                                          \
        ay += (REAL)ny[i] / wall_len * flux;                                          \
      }                                                                               \
      /* Stokeslet and rotlet completion */                                           \
      for (int32_t k = 0; k < m; ++k) {                                               \
        REAL qx = (REAL)x[i] - (REAL)cx[k];                                           \
        REAL qy = (REAL)y[i] - (REAL)cy[k];                                           \
        REAL q2 = qx * qx + qy * qy;                                                  \
        REAL lg = (REAL)0.5 * LOG(q2);                                                \
        REAL lx = comp[3 * k], ly = comp[3 * k + 1], mu = comp[3 * k + 2];            \
        REAL dot = (qx * lx + qy * ly) / q2;                                          \
        REAL rot = (REAL)radius[k] * mu / q2;                                         \
        ax += (-lg * lx + qx * dot + rot * qy) / (4 * pi);                            \
        ay += (-lg * ly + qy * dot - rot * qx) / (4 * pi);                            \
      }                                                                               \
      out[i] = (double)ax;                                                            \
      out[nn + i] = (double)ay;                                                       \
    }                                                                                 \
    /* pore constraint rows */                                                        \
    for (int32_t k = 0; k < m; ++k) {                                                 \
      REAL lx = 0, ly = 0, mo = 0;                                                    \
      for (int64_t j = curve_off[k]; j < curve_off[k + 1]; ++j) {                     \
        lx += (REAL)w[j] * sx[j];                                                     \
        ly += (REAL)w[j] * sy[j];                                                     \
        mo += (REAL)w[j] * (((REAL)y[j] - (REAL)cy[k]) * sx[j]                        \
                            - ((REAL)x[j] - (REAL)cx[k]) * sy[j]);                    \
      }                                                                               \
      REAL rk = radius[k];                                                            \
      out[2 * nn + 3 * k] = (double)(lx / (2 * pi * rk) - (REAL)comp[3 * k]);         \
      out[2 * nn + 3 * k + 1] = (double)(ly / (2 * pi * rk) - (REAL)comp[3 * k + 1]); \
      out[2 * nn + 3 * k + 2] =                                                       \
          (double)(mo / (2 * pi * rk * rk) - (REAL)comp[3 * k + 2]);                  \
    }                                                                                 \
  }

/* The double version lets the compiler vectorise the sum over sources (the
   order of the additions is then by vector lane; any order is a valid
   rounding of the same sum) and picks the widest vector unit at load time. */
DEFINE_APPLY(oracle_apply_f64, double, log, "omp simd reduction(+ : ax, ay)",
             __attribute__((target_clones("avx512f", "avx2", "default"))))
DEFINE_APPLY(oracle_apply_f80, long double, logl, "GCC unroll 1", )

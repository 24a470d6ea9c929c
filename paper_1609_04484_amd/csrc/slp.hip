// Single-layer (first-kind) formulation of Section 2.1, equation
// "stokesBIE": f(x_i) = 1/(4 pi) int_Gamma G(x_i - y) sigma(y) ds, with
// G(r) = -log|r| I + r r^T / |r|^2, collocated at the nodes and integrated
// by the corrected trapezoid rule of Section 2.2 (Kapur-Rokhlin, sixth
// order): the node i itself is left out, and the weights of the six nodes on
// either side of it on its own curve are multiplied by (1 + gamma_k).  The
// correction weights are derived below from the error expansion of the
// punctured trapezoid rule (the paper does not print them).  Unknowns are
// [sigma_x (Nn) | sigma_y (Nn)] (no completion: 2 Nn unknowns).
//
// Matvec launches:
//   slp_pack      source records (x, y, w sigma_x / 4pi, w sigma_y / 4pi)
//   slp_pairs<T>  the O(Nn^2) punctured sum, same layout as the double
//                 layer's pair kernel: T targets per lane, four waves split a
//                 source chunk and add their sums in LDS
//   slp_epilogue  sums the chunk partials and adds the 12 corrections of
//                 each node (its curve neighbours at distance 1..6)
// The velocity in the fluid (equation "stokesSLP_discretized") reuses the
// pack and pair kernels with the points as targets and no corrections.
#include <algorithm>
#include <cmath>
#include <utility>

#include "pairmath.hpp"
#include "slp.hpp"

namespace sbie {

namespace {

constexpr int kSlpBlock = 256;
constexpr int kSlpWaves = kSlpBlock / 64;
constexpr int kSlpCorr = 6;   // corrected neighbours on each side

// ---------------------------------------------------------------------------
// Correction weights.  For f(t) = phi(t) log|t - t_i| + psi(t) with phi, psi
// smooth on a periodic grid of step h, the generalised Euler-Maclaurin
// expansion gives
//   int f - h sum_{j != i} f_j = h phi_i log(h / 2 pi) + h psi_i
//                               + 2 sum_{p >= 1} zeta'(-2p) h^{2p+1} phi_i^{(2p)} / (2p)!.
// The corrections h sum_{0 < |k| <= 6} gamma_|k| f_{i+k} reproduce it up to
// O(h^7 log h) when, with the sums over k = 1..6,
//   2 sum gamma_k k^{2p} = [p == 0]   and   2 sum gamma_k k^{2p} log k =
//   -log(2 pi) (p = 0), 2 zeta'(-2p) (p = 1, 2);
// zeta'(-2p) = (-1)^p (2p)! zeta(2p + 1) / (2 (2 pi)^{2p}) (functional
// equation).  zeta(3), zeta(5) are summed directly with an Euler-Maclaurin
// tail.  The 6 x 6 system is solved once on the host.
// ---------------------------------------------------------------------------
long double zeta_odd(int s) {
  const int n = 64;
  long double acc = 0.0L;
  for (int k = n; k >= 1; --k) acc += powl((long double)k, -(long double)s);
  const long double N = n;
  // tail sum_{k > N} k^-s = N^{1-s}/(s-1) - N^-s/2 + s N^{-s-1}/12 - s(s+1)(s+2) N^{-s-3}/720 + ...
  acc += powl(N, 1.0L - s) / (s - 1) - powl(N, -(long double)s) / 2 +
         s * powl(N, -(long double)s - 1) / 12 -
         (long double)s * (s + 1) * (s + 2) * powl(N, -(long double)s - 3) / 720;
  return acc;
}

struct Weights {
  double g[kSlpCorr];
};

Weights derive_weights() {
  const long double pi = 3.141592653589793238462643383279502884L;
  long double a[kSlpCorr][kSlpCorr + 1];
  const long double zp1 = -2.0L * zeta_odd(3) / (2.0L * powl(2 * pi, 2));   // zeta'(-2)
  const long double zp2 = 24.0L * zeta_odd(5) / (2.0L * powl(2 * pi, 4));   // zeta'(-4)
  const long double rhs[kSlpCorr] = {1.0L, 0.0L, 0.0L, -logl(2 * pi), 2 * zp1, 2 * zp2};
  for (int p = 0; p < 3; ++p)
    for (int k = 1; k <= kSlpCorr; ++k) {
      a[p][k - 1] = 2.0L * powl((long double)k, 2 * p);
      a[3 + p][k - 1] = 2.0L * powl((long double)k, 2 * p) * logl((long double)k);
    }
  for (int r = 0; r < kSlpCorr; ++r) a[r][kSlpCorr] = rhs[r];
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < kSlpCorr; ++c) {
    int piv = c;
    for (int r = c + 1; r < kSlpCorr; ++r)
      if (fabsl(a[r][c]) > fabsl(a[piv][c])) piv = r;
    for (int q = 0; q <= kSlpCorr; ++q) std::swap(a[c][q], a[piv][q]);
    for (int r = 0; r < kSlpCorr; ++r) {
      if (r == c) continue;
      const long double f = a[r][c] / a[c][c];
      for (int q = c; q <= kSlpCorr; ++q) a[r][q] -= f * a[c][q];
    }
  }
  Weights w;
  for (int k = 0; k < kSlpCorr; ++k) w.g[k] = (double)(a[k][kSlpCorr] / a[k][k]);
  return w;
}

const Weights &weights() {
  static const Weights w = derive_weights();
  return w;
}

__device__ __forceinline__ int curve_of(const int64_t *__restrict__ off, int ncurves, int64_t i) {
  int lo = 0, hi = ncurves - 1;   // largest k with off[k] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void slp_pack(int64_t nn, const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ w, const double *__restrict__ u,
                         double *__restrict__ src) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nn) return;
  const double s = w[j] * (0.25 / kPi);
  double2 *d = reinterpret_cast<double2 *>(src + 4 * j);
  d[0] = make_double2(x[j], y[j]);
  d[1] = make_double2(s * u[j], s * u[nn + j]);
}

// One (target tile, source chunk) workgroup: T targets per lane (64 T per
// tile), the chunk split into quarters over the four waves.  The pair with
// r = 0 (a target on a source node) is left out, which is the punctured rule
// for the node rows.  Per pair: r (2), rho^2 (2), its reciprocal (4), log
// (one library call), the two components (6).
template <int T, bool ACC>
__global__ __launch_bounds__(kSlpBlock) void slp_pairs(const double *__restrict__ src,
                                                       const double *__restrict__ xs,
                                                       const double *__restrict__ ys, int64_t nt,
                                                       int64_t ns, int64_t chunk,
                                                       double *__restrict__ part, int tiles) {
  constexpr int NV = ACC ? 4 : 2;
  const int tile = blockIdx.x % tiles;
  const int64_t ch = blockIdx.x / tiles;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tile0 = (int64_t)tile * (64 * T) + lane;
  double xi[T], yi[T], ax[T], ay[T], ex[T], ey[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int64_t i = tile0 + (int64_t)t * 64;
    xi[t] = i < nt ? xs[i] : xs[nt - 1] + 1.0e3 * (double)(t + 1);
    yi[t] = i < nt ? ys[i] : ys[nt - 1];
    ax[t] = ay[t] = ex[t] = ey[t] = 0.0;
  }
  const int c0 = (int)(ch * chunk);
  const int c1 = (int)(ch * chunk + chunk < ns ? ch * chunk + chunk : ns);
  const int qlen = c1 > c0 ? (c1 - c0 + kSlpWaves - 1) / kSlpWaves : 0;
  const int j0 = __builtin_amdgcn_readfirstlane(c0 + wv * qlen < c1 ? c0 + wv * qlen : c1);
  const int j1 = __builtin_amdgcn_readfirstlane(j0 + qlen < c1 ? j0 + qlen : c1);
  for (int j = j0; j < j1; ++j) {
    const double *s = src + 4 * (int64_t)j;   // wave-uniform: scalar loads
    const double sx = s[0], sy = s[1], qx = s[2], qy = s[3];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const double rx = xi[t] - sx, ry = yi[t] - sy;
      const double r2 = fma(ry, ry, rx * rx);
      const bool self = r2 == 0.0;
      const double inv = self ? 0.0 : recip(r2);
      const double hl = self ? 0.0 : 0.5 * log(r2);
      const double d = fma(ry, qy, rx * qx) * inv;
      const double vx = fma(rx, d, -hl * qx);
      const double vy = fma(ry, d, -hl * qy);
      if (ACC) {
        two_sum_acc(ax[t], ex[t], vx);
        two_sum_acc(ay[t], ey[t], vy);
      } else {
        ax[t] += vx;
        ay[t] += vy;
      }
    }
  }
  __shared__ double red[kSlpWaves - 1][NV * T][64];
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      red[wv - 1][NV * t][lane] = ax[t];
      red[wv - 1][NV * t + 1][lane] = ay[t];
      if (ACC) {
        red[wv - 1][NV * t + 2][lane] = ex[t];
        red[wv - 1][NV * t + 3][lane] = ey[t];
      }
    }
  }
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int o = 0; o < kSlpWaves - 1; ++o)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if (ACC) {
        two_sum_acc(ax[t], ex[t], red[o][NV * t][lane]);
        two_sum_acc(ay[t], ey[t], red[o][NV * t + 1][lane]);
        ex[t] += red[o][NV * t + 2][lane];
        ey[t] += red[o][NV * t + 3][lane];
      } else {
        ax[t] += red[o][NV * t][lane];
        ay[t] += red[o][NV * t + 1][lane];
      }
    }
  double *px = part + ch * NV * nt;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int64_t i = tile0 + (int64_t)t * 64;
    if (i < nt) {
      px[i] = ax[t];
      px[nt + i] = ay[t];
      if (ACC) {
        px[2 * nt + i] = ex[t];
        px[3 * nt + i] = ey[t];
      }
    }
  }
}

struct Gamma {
  double g[kSlpCorr];
};

// y_i = sum of the chunk partials + the corrections gamma_k w_j G(x_i - x_j)
// sigma_j / (4 pi) over the six curve neighbours j = i +- k (periodic on the
// curve of i).
__global__ void slp_epilogue(int64_t nn, int ncurves, const int64_t *__restrict__ off, int nchunks, int acc,
                             const double *__restrict__ part, const double *__restrict__ src,
                             Gamma gam, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int64_t stride = (acc ? 4 : 2) * nn;
  double vx = 0.0, vy = 0.0, ex = 0.0, ey = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    const double *p = part + (int64_t)c * stride;
    if (acc) {
      two_sum_acc(vx, ex, p[i]);
      two_sum_acc(vy, ey, p[nn + i]);
      ex += p[2 * nn + i];
      ey += p[3 * nn + i];
    } else {
      vx += p[i];
      vy += p[nn + i];
    }
  }
  const int k = curve_of(off, ncurves, i);
  const int64_t a = off[k], n = off[k + 1] - a;
  const double xi = src[4 * i], yi = src[4 * i + 1];
  for (int d = 1; d <= kSlpCorr; ++d)
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int64_t q = (i - a) + sgn * d;
      q = ((q % n) + n) % n;
      const double *s = src + 4 * (a + q);
      const double rx = xi - s[0], ry = yi - s[1];
      const double r2 = fma(ry, ry, rx * rx);
      const double dd = fma(ry, s[3], rx * s[2]) / r2;
      const double hl = 0.5 * log(r2);
      const double g = gam.g[d - 1];
      const double cx = g * fma(rx, dd, -hl * s[2]);
      const double cy = g * fma(ry, dd, -hl * s[3]);
      if (acc) {
        two_sum_acc(vx, ex, cx);
        two_sum_acc(vy, ey, cy);
      } else {
        vx += cx;
        vy += cy;
      }
    }
  out[i] = vx + ex;
  out[nn + i] = vy + ey;
}

__global__ void slp_velocity_epilogue(int64_t np, int nchunks, const double *__restrict__ part,
                                      double *__restrict__ ux, double *__restrict__ uy,
                                      const double *__restrict__ rx, const double *__restrict__ ry,
                                      double *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double vx = 0.0, vy = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    vx += part[(int64_t)c * 2 * np + i];
    vy += part[(int64_t)c * 2 * np + np + i];
  }
  ux[i] = vx;
  uy[i] = vy;
  if (err) {
    const double a = sqrt(vx * vx + vy * vy), b = sqrt(rx[i] * rx[i] + ry[i] * ry[i]);
    err[i] = fabs(a - b) / b;
  }
}

// A[rows, cols] of the corrected single-layer matrix (column-major).
__global__ void slp_assemble_kernel(int64_t nn, int ncurves, const int64_t *__restrict__ off,
                                    const double *__restrict__ x, const double *__restrict__ y,
                                    const double *__restrict__ w, Gamma gam,
                                    const int64_t *__restrict__ rows, int64_t nr,
                                    const int64_t *__restrict__ cols, int64_t nc,
                                    double *__restrict__ out, int64_t ld) {
  const int64_t ri = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ci = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  if (ri >= nr || ci >= nc) return;
  const int64_t R = rows[ri], C = cols[ci];
  const int64_t i = R < nn ? R : R - nn, j = C < nn ? C : C - nn;
  const int a = R < nn ? 0 : 1, b = C < nn ? 0 : 1;
  double v = 0.0;
  if (i != j) {
    const double rx = x[i] - x[j], ry = y[i] - y[j];
    const double r2 = rx * rx + ry * ry;
    const double ra = a ? ry : rx, rb = b ? ry : rx;
    double gab = ra * rb / r2;
    if (a == b) gab -= 0.5 * log(r2);
    double fac = 1.0;
    const int ki = curve_of(off, ncurves, i), kj = curve_of(off, ncurves, j);
    if (ki == kj) {
      const int64_t n = off[ki + 1] - off[ki];
      int64_t d = i > j ? i - j : j - i;
      if (n - d < d) d = n - d;
      if (d >= 1 && d <= kSlpCorr) fac += gam.g[d - 1];
    }
    v = w[j] * (0.25 / kPi) * fac * gab;
  }
  out[ri + ci * ld] = v;
}

// Square diagonal blocks: block b uses indices idx[ioff[b] .. ioff[b] + sz[b])
// for rows and columns and writes a column-major sz x sz matrix at
// out + ooff[b].
__global__ void slp_assemble_diag_kernel(int64_t nn, int ncurves, const int64_t *__restrict__ off,
                                         const double *__restrict__ x, const double *__restrict__ y,
                                         const double *__restrict__ w, Gamma gam,
                                         const int64_t *__restrict__ idx, const int64_t *__restrict__ ioff,
                                         const int32_t *__restrict__ sz, const int64_t *__restrict__ ooff,
                                         double *__restrict__ out) {
  const int b = blockIdx.z;
  const int n = sz[b];
  const int ri = blockIdx.x * blockDim.x + threadIdx.x;
  const int ci = blockIdx.y * blockDim.y + threadIdx.y;
  if (ri >= n || ci >= n) return;
  const int64_t *ix = idx + ioff[b];
  const int64_t R = ix[ri], C = ix[ci];
  const int64_t i = R < nn ? R : R - nn, j = C < nn ? C : C - nn;
  const int a = R < nn ? 0 : 1, bb = C < nn ? 0 : 1;
  double v = 0.0;
  if (i != j) {
    const double rx = x[i] - x[j], ry = y[i] - y[j];
    const double r2 = rx * rx + ry * ry;
    const double ra = a ? ry : rx, rb = bb ? ry : rx;
    double gab = ra * rb / r2;
    if (a == bb) gab -= 0.5 * log(r2);
    double fac = 1.0;
    const int ki = curve_of(off, ncurves, i), kj = curve_of(off, ncurves, j);
    if (ki == kj) {
      const int64_t nc = off[ki + 1] - off[ki];
      int64_t d = i > j ? i - j : j - i;
      if (nc - d < d) d = nc - d;
      if (d >= 1 && d <= kSlpCorr) fac += gam.g[d - 1];
    }
    v = w[j] * (0.25 / kPi) * fac * gab;
  }
  out[ooff[b] + ri + (int64_t)ci * n] = v;
}

int pair_chunks(int64_t ns, int64_t tiles) {
  int per_cu = 0, cus = 0, dev = 0;
  SBIE_HIP(hipGetDevice(&dev));
  SBIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&slp_pairs<4, false>), kSlpBlock, 0));
  SBIE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t resident = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>((ns + 255) / 256, 1024));
  return (int)std::max<int64_t>(1, std::min<int64_t>((8 * resident + tiles - 1) / tiles, cap));
}

Gamma gamma_arg() {
  Gamma g;
  for (int k = 0; k < kSlpCorr; ++k) g.g[k] = weights().g[k];
  return g;
}

}  // namespace

void slp_check_geom(const sbie_geom *g) {
  for (int k = 0; k <= g->n_pores; ++k) {
    const int64_t n = g->curve_off[k + 1] - g->curve_off[k];
    if (n > 0 && n <= 2 * kSlpCorr)
      fail(SBIE_UNSUPPORTED, "curve %d has %lld nodes: the corrected rule needs more than %d", k,
           (long long)n, 2 * kSlpCorr);
  }
}

void slp_matvec_run(const sbie_geom *g, const double *x, double *y, bool accurate, hipStream_t s) {
  const int64_t nn = g->n_nodes;
  const int T = accurate ? 1 : 4;
  const int tiles = (int)ceil_div(nn, (int64_t)64 * T);
  const int chunks = pair_chunks(nn, tiles);
  const int nv = accurate ? 4 : 2;
  StreamBuf<double> scratch((size_t)4 * nn + (size_t)chunks * nv * nn, s);
  double *src = scratch.p, *part = src + 4 * nn;
  slp_pack<<<ceil_div(nn, 256), 256, 0, s>>>(nn, g->x, g->y, g->w, x, src);
  SBIE_LAUNCH_CHECK();
  const int64_t chunk = (nn + chunks - 1) / chunks;
  const unsigned grid = (unsigned)((int64_t)tiles * chunks);
  if (accurate)
    slp_pairs<1, true><<<grid, kSlpBlock, 0, s>>>(src, g->x, g->y, nn, nn, chunk, part, tiles);
  else
    slp_pairs<4, false><<<grid, kSlpBlock, 0, s>>>(src, g->x, g->y, nn, nn, chunk, part, tiles);
  SBIE_LAUNCH_CHECK();
  slp_epilogue<<<ceil_div(nn, 256), 256, 0, s>>>(nn, g->n_pores + 1, g->curve_off_dev, chunks,
                                                 accurate ? 1 : 0, part, src, gamma_arg(), y);
  SBIE_LAUNCH_CHECK();
}

void slp_assemble(const sbie_geom *g, const int64_t *rows, int64_t nr, const int64_t *cols, int64_t nc,
                  double *out, int64_t ld, hipStream_t s) {
  if (nr == 0 || nc == 0) return;
  dim3 blk(64, 4);
  const int64_t step = (int64_t)65535 * 4;
  for (int64_t c0 = 0; c0 < nc; c0 += step) {
    const int64_t cn = nc - c0 < step ? nc - c0 : step;
    dim3 grid(ceil_div(nr, 64), ceil_div(cn, 4));
    slp_assemble_kernel<<<grid, blk, 0, s>>>(g->n_nodes, g->n_pores + 1, g->curve_off_dev, g->x, g->y, g->w,
                                             gamma_arg(), rows, nr, cols + c0, cn, out + c0 * ld, ld);
    SBIE_LAUNCH_CHECK();
  }
}

void slp_assemble_diag_batched(const sbie_geom *g, const int64_t *idx, const int64_t *ioff, const int32_t *sz,
                               const int64_t *ooff, int nblocks, int max_n, double *out, hipStream_t s) {
  if (nblocks == 0) return;
  dim3 blk(64, 4);
  dim3 grid(ceil_div(max_n, 64), ceil_div(max_n, 4), nblocks);
  slp_assemble_diag_kernel<<<grid, blk, 0, s>>>(g->n_nodes, g->n_pores + 1, g->curve_off_dev, g->x, g->y, g->w,
                                                gamma_arg(), idx, ioff, sz, ooff, out);
  SBIE_LAUNCH_CHECK();
}

void slp_velocity_run(const sbie_geom *g, const double *sigma, const double *px, const double *py,
                      int64_t np, double *ux, double *uy, const double *rx, const double *ry, double *err,
                      hipStream_t s) {
  const int64_t nn = g->n_nodes;
  const int tiles = (int)ceil_div(np, (int64_t)64 * 4);
  const int chunks = pair_chunks(nn, tiles);
  StreamBuf<double> scratch((size_t)4 * nn + (size_t)chunks * 2 * np, s);
  double *src = scratch.p, *part = src + 4 * nn;
  slp_pack<<<ceil_div(nn, 256), 256, 0, s>>>(nn, g->x, g->y, g->w, sigma, src);
  SBIE_LAUNCH_CHECK();
  const int64_t chunk = (nn + chunks - 1) / chunks;
  slp_pairs<4, false><<<(unsigned)((int64_t)tiles * chunks), kSlpBlock, 0, s>>>(src, px, py, np, nn, chunk,
                                                                                part, tiles);
  SBIE_LAUNCH_CHECK();
  slp_velocity_epilogue<<<ceil_div(np, 256), 256, 0, s>>>(np, chunks, part, ux, uy, rx, ry, err);
  SBIE_LAUNCH_CHECK();
}

void slp_weights(double *out) {
  for (int k = 0; k < kSlpCorr; ++k) out[k] = weights().g[k];
}

}  // namespace sbie

extern "C" int stokes_slp_weights(double *gamma) {
  return sbie::guarded([&]() {
    if (!gamma) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    sbie::slp_weights(gamma);
    return SBIE_OK;
  });
}

extern "C" int stokes_slp_matvec(const sbie_geom *g, const double *x, double *y, int mode, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!x || !y) sbie::fail(SBIE_INVALID_ARGUMENT, "null vector");
    if (mode != SBIE_MV_FULL && mode != SBIE_MV_FULL_ACCURATE)
      sbie::fail(SBIE_INVALID_ARGUMENT, "single-layer matvec mode must be SBIE_MV_FULL or SBIE_MV_FULL_ACCURATE");
    const int64_t n = 2 * g->n_nodes;
    if (x < y + n && y < x + n) sbie::fail(SBIE_INVALID_ARGUMENT, "x and y overlap");
    sbie::slp_check_geom(g);
    sbie::slp_matvec_run(g, x, y, mode == SBIE_MV_FULL_ACCURATE, (hipStream_t)stream);
    return SBIE_OK;
  });
}

extern "C" int stokes_slp_assemble(const sbie_geom *g, const int64_t *rows, int64_t nr, const int64_t *cols,
                                   int64_t nc, double *out, int64_t ld, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (nr < 0 || nc < 0 || ld < nr) sbie::fail(SBIE_INVALID_ARGUMENT, "bad block shape");
    if ((nr > 0 && !rows) || (nc > 0 && !cols) || (nr > 0 && nc > 0 && !out))
      sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    sbie::slp_check_geom(g);
    sbie::slp_assemble(g, rows, nr, cols, nc, out, ld, (hipStream_t)stream);
    return SBIE_OK;
  });
}

extern "C" int stokes_slp_velocity(const sbie_geom *g, const double *sigma, const double *px, const double *py,
                                   int64_t np, double *ux, double *uy, const double *uref_x,
                                   const double *uref_y, double *err, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (np < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "np < 0");
    if (np == 0) return SBIE_OK;
    if (!sigma || !px || !py || !ux || !uy) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if ((err != nullptr) != (uref_x != nullptr) || (uref_x != nullptr) != (uref_y != nullptr))
      sbie::fail(SBIE_INVALID_ARGUMENT, "uref_x, uref_y and err go together");
    if (np > (int64_t)0x7fffffff) sbie::fail(SBIE_INVALID_ARGUMENT, "too many points");
    sbie::slp_velocity_run(g, sigma, px, py, np, ux, uy, uref_x, uref_y, err, (hipStream_t)stream);
    return SBIE_OK;
  });
}

// Matrix-free application of the completed double-layer operator
// (Section 2.1 double-layer kernel, Section 2.2 Nystrom discretisation).
//
// Launch structure of one y = A x:
//   pack_sources      SoA node data + current density -> 64-byte source records
//                     (x, y, q_xx, q_xy, q_yy) with q the symmetric part of
//                     a sigma^T, a = w n / pi, so that the pair factor
//                     (r.a)(r.sigma) = r^T q r; pore records
//                     (cx, cy, lambda_x, lambda_y, r mu)
//   wall_flux         flux functional sum_wall w n.sigma and |Gamma_0|
//   dlp_pairs<T>      the O(Nn^2) pair sum, split into (target tile, source
//                     chunk) workgroups; each lane owns T targets and the
//                     four waves of a workgroup share the tile and split the
//                     chunk, then add their sums in LDS (one partial sum per
//                     workgroup); source records are wave-uniform so they
//                     are read through the scalar data path and broadcast
//   completion_pairs  Stokeslet/rotlet columns, (target tile, pore chunk)
//   epilogue          sums the partials, adds the jump, the smooth diagonal
//                     limit and the wall rank-one term
//   pore_rows         the three constraint rows per pore (one wave per pore)
#include <algorithm>
#include <map>
#include <mutex>

#include "common.hpp"
#include "pairmath.hpp"

namespace sbie {

namespace {

constexpr int kBlock = 256;
constexpr int kPoreChunk = 64;

int g_tpt = 4;        // targets per thread
int g_chunks = 0;     // source chunks (0 = automatic)
int g_batch_queue = 1;   // batched pair stage: persistent work queue (1) or one workgroup per item (0)
int g_sym_mode = 1;      // symmetric pair evaluation: 0 never, 1 where it pays, 2 always (plain modes)

// optional event bracketing of the pair kernel
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

__device__ __forceinline__ void pack_body(int64_t j, int64_t nn, int m, const double *__restrict__ x,
                                          const double *__restrict__ y, const double *__restrict__ nx,
                                          const double *__restrict__ ny, const double *__restrict__ w,
                                          const double *__restrict__ rad, const double *__restrict__ cx,
                                          const double *__restrict__ cy, const double *__restrict__ u,
                                          double *__restrict__ src, double *__restrict__ psrc) {
  if (j < nn) {
    const double s = w[j] * (1.0 / kPi);
    const double ax = s * nx[j], ay = s * ny[j], sx = u[j], sy = u[nn + j];
    double2 *d = reinterpret_cast<double2 *>(src + 8 * j);
    d[0] = make_double2(x[j], y[j]);
    d[1] = make_double2(ax * sx, fma(ax, sy, ay * sx));
    d[2] = make_double2(ay * sy, 0.0);
    d[3] = make_double2(0.0, 0.0);
  }
  if (j < m) {
    const double *lam = u + 2 * nn + 3 * j;
    double2 *d = reinterpret_cast<double2 *>(psrc + 8 * j);
    d[0] = make_double2(cx[j], cy[j]);
    d[1] = make_double2(lam[0], lam[1]);
    d[2] = make_double2(rad[j] * lam[2], 0.0);
    d[3] = make_double2(0.0, 0.0);
  }
}

__global__ void pack_sources(int64_t nn, int m, const double *__restrict__ x,
                             const double *__restrict__ y,
                             const double *__restrict__ nx,
                             const double *__restrict__ ny,
                             const double *__restrict__ w,
                             const double *__restrict__ rad,
                             const double *__restrict__ cx,
                             const double *__restrict__ cy,
                             const double *__restrict__ u,
                             double *__restrict__ src,
                             double *__restrict__ psrc) {
  pack_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, nn, m, x, y, nx, ny, w, rad, cx, cy, u, src,
            psrc);
}

// scal[0] = sum over wall nodes of w (n . sigma); scal[1] = sum of w.
// 1024 threads.
__device__ __forceinline__ void wall_flux_body(int64_t wall_start, int64_t nn, const double *__restrict__ nx,
                                               const double *__restrict__ ny, const double *__restrict__ w,
                                               const double *__restrict__ u, double *scal, int with_flux) {
  __shared__ double sb[1024], sl[1024];
  double b = 0.0, l = 0.0;
  for (int64_t i = wall_start + threadIdx.x; i < nn; i += blockDim.x) {
    l += w[i];
    if (with_flux) b += w[i] * (nx[i] * u[i] + ny[i] * u[nn + i]);
  }
  sb[threadIdx.x] = b;
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sb[threadIdx.x] += sb[threadIdx.x + s];
      sl[threadIdx.x] += sl[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal[0] = sb[0];
    scal[1] = sl[0];
  }
}

__global__ void wall_flux(int64_t wall_start, int64_t nn,
                          const double *__restrict__ nx,
                          const double *__restrict__ ny,
                          const double *__restrict__ w,
                          const double *__restrict__ u, double *scal,
                          int with_flux) {
  wall_flux_body(wall_start, nn, nx, ny, w, u, scal, with_flux);
}

// Reciprocals of T positive numbers with one hardware reciprocal: the
// product of all of them is inverted (and refined) once, and each 1/d_t is
// recovered as that inverse times the product of the others (Montgomery's
// batch-inversion trick).  The d_t are squared distances between nodes (at
// least 1e-100), so a product of up to eight stays far inside the FP64
// range for any domain smaller than about 1e18.
template <int T>
__device__ __forceinline__ void batch_recip(const double *d, double *out) {
  if constexpr (T == 1) {
    out[0] = recip(d[0]);
  } else if constexpr (T == 2) {
    const double r = recip(d[0] * d[1]);
    out[0] = r * d[1];
    out[1] = r * d[0];
  } else if constexpr (T == 4) {
    const double p01 = d[0] * d[1], p23 = d[2] * d[3];
    const double r = recip(p01 * p23);
    const double r01 = r * p23, r23 = r * p01;
    out[0] = r01 * d[1];
    out[1] = r01 * d[0];
    out[2] = r23 * d[3];
    out[3] = r23 * d[2];
  } else if constexpr (T == 8) {
    // product tree over eight values, one refined reciprocal, then the
    // partial products recover every 1/d_t
    const double p01 = d[0] * d[1], p23 = d[2] * d[3], p45 = d[4] * d[5], p67 = d[6] * d[7];
    const double p03 = p01 * p23, p47 = p45 * p67;
    const double r = recip(p03 * p47);
    const double r03 = r * p47, r47 = r * p03;
    const double r01 = r03 * p23, r23 = r03 * p01, r45 = r47 * p67, r67 = r47 * p45;
    out[0] = r01 * d[1];
    out[1] = r01 * d[0];
    out[2] = r23 * d[3];
    out[3] = r23 * d[2];
    out[4] = r45 * d[5];
    out[5] = r45 * d[4];
    out[6] = r67 * d[7];
    out[7] = r67 * d[6];
  } else {
#pragma unroll
    for (int h = 0; h < T; h += 8) batch_recip<8>(d + h, out + h);
  }
}

// The contribution of one source record to T targets, with the
// reciprocals of S consecutive sources batched together (S * T values).
// Per pair: r (2), r_y^2 and rho^2 (2), its share of the batched
// reciprocal, r^T q r = r_x (q_xx r_x + q_xy r_y) + q_yy r_y^2 (4),
// 1/rho^4 (1), the coefficient (1) and two accumulating FMAs.
template <int T, int S, bool ACC>
__device__ __forceinline__ void pair_step(const double *__restrict__ src, int j, const double *xi,
                                          const double *yi, double *ax, double *ay, double *cxa,
                                          double *cya) {
  double sx[S], sy[S], qxx[S], qxy[S], qyy[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const double *s = src + 8 * (int64_t)(j + q);  // wave-uniform: scalar loads
    sx[q] = s[0];
    sy[q] = s[1];
    qxx[q] = s[2];
    qxy[q] = s[3];
    qyy[q] = s[4];
  }
  double rx[S * T], ry[S * T], ryy[S * T], r2[S * T], inv[S * T];
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int u = q * T + t;
      rx[u] = xi[t] - sx[q];
      ry[u] = yi[t] - sy[q];
      // the self pair has r = 0 exactly: the 1e-100 added inside the fused
      // multiply-add keeps 1/rho^4 finite there (the pair's factor r^T q r
      // is then q_yy 1e-100, times r = 0) and is below half an ulp of
      // r_y^2 and rho^2 for every pair of distinct nodes
      ryy[u] = fma(ry[u], ry[u], 1e-100);
      r2[u] = fma(rx[u], rx[u], ryy[u]);
    }
  batch_recip<S * T>(r2, inv);
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int u = q * T + t;
      const double h = fma(qxy[q], ry[u], qxx[q] * rx[u]);
      const double pq = fma(h, rx[u], qyy[q] * ryy[u]);
      const double c = pq * (inv[u] * inv[u]);
      if (ACC) {
        two_sum_acc(ax[t], cxa[t], c * rx[u]);
        two_sum_acc(ay[t], cya[t], c * ry[u]);
      } else {
        ax[t] = fma(c, rx[u], ax[t]);
        ay[t] = fma(c, ry[u], ay[t]);
      }
    }
}

// One workgroup of the pair sum: target tile `tile` (64 T targets, lane l
// owning targets tile * 64 T + l + 64 t) against source chunk `ch` (sources
// [ch * chunk, (ch + 1) * chunk)), the chunk split into four consecutive
// quarters, one per wave.  The plain kernel takes two sources per step for
// T <= 4 (eight or fewer reciprocals share one hardware reciprocal); the
// compensated one takes one.  The four waves' sums are added in LDS in a
// fixed order and one partial sum per target is written:
// part[ch][0..1 or 0..3][nn] (value x, y and, compensated, their errors).
constexpr int kWaves = kBlock / 64;
constexpr int kTileLanes = 64;

template <int T, bool ACC>
__device__ __forceinline__ void dlp_pairs_body(const double *__restrict__ src, const double *__restrict__ xs,
                                               const double *__restrict__ ys, int64_t nt, int64_t ns,
                                               int64_t chunk, double *__restrict__ part, int64_t tile,
                                               int64_t ch) {
  constexpr int S = (!ACC && T <= 4) ? 2 : 1;
  constexpr int NV = ACC ? 4 : 2;    // values per target in a partial sum
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tile0 = tile * (kTileLanes * T) + lane;
  double xi[T], yi[T], ax[T], ay[T], cxa[T], cya[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int64_t i = tile0 + (int64_t)t * kTileLanes;
    // padding targets of the last tile sit far away from every node and at
    // distinct places, so at most one target per thread can coincide with a
    // source (the batched reciprocal multiplies the squared distances)
    xi[t] = i < nt ? xs[i] : xs[nt - 1] + 1.0e3 * (double)(t + 1);
    yi[t] = i < nt ? ys[i] : ys[nt - 1];
    ax[t] = 0.0;
    ay[t] = 0.0;
    cxa[t] = 0.0;
    cya[t] = 0.0;
  }
  // uniform 32-bit loop bounds kept in scalar registers (node counts are
  // below 2^31), so the loop test is a scalar compare; this wave's quarter
  // of the chunk
  const int c0 = (int)(ch * chunk);
  const int c1 = (int)(ch * chunk + chunk < ns ? ch * chunk + chunk : ns);
  const int qlen = c1 > c0 ? (c1 - c0 + kWaves - 1) / kWaves : 0;
  const int j0 = __builtin_amdgcn_readfirstlane(c0 + wv * qlen < c1 ? c0 + wv * qlen : c1);
  const int j1 = __builtin_amdgcn_readfirstlane(j0 + qlen < c1 ? j0 + qlen : c1);
  const int js = j1 > j0 ? j0 + ((j1 - j0) / S) * S : j0;
  for (int j = j0; j < js; j += S) pair_step<T, S, ACC>(src, j, xi, yi, ax, ay, cxa, cya);
  for (int j = js; j < j1; ++j) pair_step<T, 1, ACC>(src, j, xi, yi, ax, ay, cxa, cya);
  // waves 1..3 hand their sums to wave 0 through LDS
  __shared__ double red[kWaves - 1][NV * T][kTileLanes];
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      red[wv - 1][NV * t][lane] = ax[t];
      red[wv - 1][NV * t + 1][lane] = ay[t];
      if (ACC) {
        red[wv - 1][NV * t + 2][lane] = cxa[t];
        red[wv - 1][NV * t + 3][lane] = cya[t];
      }
    }
  }
  __syncthreads();
  // wave 0 adds the other waves' sums and writes (no early exit for the
  // other waves: the persistent batch kernel runs this body in a loop)
  if (wv == 0) {
#pragma unroll
    for (int o = 0; o < kWaves - 1; ++o)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (ACC) {
          two_sum_acc(ax[t], cxa[t], red[o][NV * t][lane]);
          two_sum_acc(ay[t], cya[t], red[o][NV * t + 1][lane]);
          cxa[t] += red[o][NV * t + 2][lane];
          cya[t] += red[o][NV * t + 3][lane];
        } else {
          ax[t] += red[o][NV * t][lane];
          ay[t] += red[o][NV * t + 1][lane];
        }
      }
    double *px = part + ch * NV * nt;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t i = tile0 + (int64_t)t * kTileLanes;
      if (i < nt) {
        px[i] = ax[t];
        px[nt + i] = ay[t];
        if (ACC) {
          px[2 * nt + i] = cxa[t];
          px[3 * nt + i] = cya[t];
        }
      }
    }
  }
}

// One-dimensional grid of tiles x chunks workgroups.  Workgroups are handed
// to the eight XCDs round robin (workgroup b to XCD b % 8); when the chunk
// count is a multiple of 8 (xcd != 0), XCD x takes the chunks ch = x (mod 8),
// so each XCD's L2 only ever holds an eighth of the source records.
template <int T, bool ACC>
__global__ __launch_bounds__(kBlock) void dlp_pairs(
    const double *__restrict__ src, const double *__restrict__ xs,
    const double *__restrict__ ys, int64_t nt, int64_t nn, int64_t chunk,
    double *__restrict__ part, int tiles, int xcd) {
  int tile, ch;
  if (xcd) {
    const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
    ch = x + 8 * (k / tiles);
    tile = k % tiles;
  } else {
    tile = blockIdx.x % tiles;
    ch = blockIdx.x / tiles;
  }
  dlp_pairs_body<T, ACC>(src, xs, ys, nt, nn, chunk, part, tile, ch);
}

// ---------------------------------------------------------------------------
// Symmetric evaluation of the pair sum.  The contributions of node j to node
// i and of node i to node j share r = x_i - x_j (up to its sign), rho^2 and
// 1/rho^4: for q_i, q_j the records' tensors,
//   to i:  r (r^T q_j r) / rho^4,      to j:  -r (r^T q_i r) / rho^4,
// so one evaluation of the shared part serves both, and every unordered
// pair of distinct tiles is visited once.  Work unit: a superblock pair
// (Kr <= Kc) of SB x SB tiles of 256 nodes.  Each lane owns 4 targets of the
// current row tile and one node of its wave's quarter of the column tile;
// the column nodes are passed round the wave by DPP rotations (one lane per
// step, 64 steps), each carrying its own sum, so no cross-lane reduction is
// needed: the row tile's sums stay in registers, the column nodes' sums go
// to LDS (one slot per node) until the superblock is done.  Diagonal tiles (I = J) are
// summed one way only, the self pair included (zero as in dlp_pairs).
// Partial sums: for the targets of superblock K, R + 1 slots of 2 x SB x 256
// doubles, slot Kc - K for the row part of superblock pair (K, Kc) and slot
// R - K + Kr for the column part of (Kr, K); every slot is written once per
// product, then sym_reduce adds each target's slots in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kSymT = 4;                          // targets per lane
constexpr int kSymTile = kTileLanes * kSymT;      // 256 nodes per tile
constexpr int kSymSB = 4;                         // tiles per superblock side
constexpr int kSymSBN = kSymSB * kSymTile;        // nodes per superblock

// The value of the previous lane (lane l receives lane l - 1, lane 0 lane
// 63): a DPP whole-wave rotation (wave_ror:1), two VALU moves per double
// and no trip through LDS.  (Measured at the 1000-pore pipe: 1.82 ms per
// product against 1.98 ms when the ring goes through the LDS crossbar.)
__device__ __forceinline__ double ring_next(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x13C, 0xF, 0xF, false),
                          __builtin_amdgcn_mov_dpp(lo, 0x13C, 0xF, 0xF, false));
}

// This lane's T targets (positions xi, yi; tensors qa = q_xx, qb = q_xy +
// q_yx, qc = q_yy) against the node this lane currently holds (position xj,
// yj, tensor ja, jb, jc): the targets' sums into ax, ay, the node's sum
// (before its sign) into bx, by.  One batched reciprocal for the T pairs.
template <int T>
__device__ __forceinline__ void sym_pairs(const double *xi, const double *yi, const double *qa, const double *qb,
                                          const double *qc, double xj, double yj, double ja, double jb, double jc,
                                          double *ax, double *ay, double &bx, double &by) {
  double rx[T], ry[T], ryy[T], r2[T], inv[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    rx[t] = xi[t] - xj;
    ry[t] = yi[t] - yj;
    ryy[t] = fma(ry[t], ry[t], 1e-100);
    r2[t] = fma(rx[t], rx[t], ryy[t]);
  }
  batch_recip<T>(r2, inv);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const double i2 = inv[t] * inv[t];
    const double h = fma(jb, ry[t], ja * rx[t]);
    const double c = fma(h, rx[t], jc * ryy[t]) * i2;
    ax[t] = fma(c, rx[t], ax[t]);
    ay[t] = fma(c, ry[t], ay[t]);
    const double h2 = fma(qb[t], ry[t], qa[t] * rx[t]);
    const double c2 = fma(h2, rx[t], qc[t] * ryy[t]) * i2;
    bx = fma(c2, rx[t], bx);
    by = fma(c2, ry[t], by);
  }
}

__global__ __launch_bounds__(kBlock) void dlp_pairs_sym(const double *__restrict__ src,
                                                        const double *__restrict__ xs,
                                                        const double *__restrict__ ys, int64_t nn, int ntiles,
                                                        int R, double *__restrict__ P) {
  constexpr int T = kSymT;
  // superblock pair of this workgroup, row-major over the upper triangle:
  // row k starts at k R - k (k - 1) / 2
  const int64_t b = blockIdx.x;
  auto start = [&](int64_t k) { return k * R - k * (k - 1) / 2; };
  const double tr = 2.0 * R + 1.0;
  int Kr = (int)floor(0.5 * (tr - sqrt(fmax(0.0, tr * tr - 8.0 * (double)b))));
  Kr = Kr < 0 ? 0 : (Kr > R - 1 ? R - 1 : Kr);
  while (Kr > 0 && start(Kr) > b) --Kr;
  while (Kr + 1 < R && start(Kr + 1) <= b) ++Kr;
  const int Kc = Kr + (int)(b - start(Kr));
  Kr = __builtin_amdgcn_readfirstlane(Kr);
  const int Kcu = __builtin_amdgcn_readfirstlane(Kc);

  __shared__ double rev[kSymSB][2][kSymTile];
  __shared__ double red[kWaves - 1][2 * T][kTileLanes];
  for (int e = threadIdx.x; e < kSymSB * 2 * kSymTile; e += blockDim.x) (&rev[0][0][0])[e] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t slot_doubles = 2 * (int64_t)kSymSBN;
  for (int ti = 0; ti < kSymSB; ++ti) {
    const int I = Kr * kSymSB + ti;
    if (I >= ntiles) break;
    double xi[T], yi[T], qa[T], qb[T], qc[T], ax[T], ay[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t i = (int64_t)I * kSymTile + lane + (int64_t)t * kTileLanes;
      if (i < nn) {
        xi[t] = xs[i];
        yi[t] = ys[i];
        qa[t] = src[8 * i + 2];
        qb[t] = src[8 * i + 3];
        qc[t] = src[8 * i + 4];
      } else {
        // padding targets: far from every node, at distinct places, no
        // tensor (their column contributions vanish)
        xi[t] = xs[nn - 1] + 1.0e3 * (double)(t + 1);
        yi[t] = ys[nn - 1];
        qa[t] = qb[t] = qc[t] = 0.0;
      }
      ax[t] = 0.0;
      ay[t] = 0.0;
    }
    const int tj0 = (Kr == Kcu) ? ti : 0;
    for (int tj = tj0; tj < kSymSB; ++tj) {
      const int J = Kcu * kSymSB + tj;
      if (J >= ntiles) break;
      const int64_t jb = (int64_t)J * kSymTile;
      // this wave's quarter of tile J: 16 T consecutive nodes
      constexpr int kQuarter = kSymTile / kWaves;
      const int64_t q0 = jb + (int64_t)wv * kQuarter;
      if (J == I) {
        const int j0 = (int)q0;
        const int j1 = (int)(q0 + kQuarter < nn ? q0 + kQuarter : nn);
        double cxa[T], cya[T];
        int j = j0;
        for (; j + 1 < j1; j += 2) pair_step<T, 2, false>(src, j, xi, yi, ax, ay, cxa, cya);
        for (; j < j1; ++j) pair_step<T, 1, false>(src, j, xi, yi, ax, ay, cxa, cya);
      } else {
        // the quarter in rings of 64 nodes, one per lane, each passed round
        // the wave one lane per step: after 64 steps every lane has met
        // every node of the ring and each node (with its sum) is back in
        // its own lane
        for (int sub = 0; sub < kQuarter / kTileLanes; ++sub) {
          const int jl = wv * kQuarter + sub * kTileLanes + lane;
          const int64_t jn = jb + jl;
          double xj, yj, ja, jbq, jc;
          if (jn < nn) {
            xj = xs[jn];
            yj = ys[jn];
            ja = src[8 * jn + 2];
            jbq = src[8 * jn + 3];
            jc = src[8 * jn + 4];
          } else {
            // padding nodes (only in the last tile, which never meets
            // padding targets here): far below every node, no tensor
            xj = xs[nn - 1];
            yj = ys[nn - 1] - 1.0e3 * (double)(lane + 1);
            ja = jbq = jc = 0.0;
          }
          double bx = 0.0, by = 0.0;
          for (int k = 0; k < kTileLanes; ++k) {
            sym_pairs<T>(xi, yi, qa, qb, qc, xj, yj, ja, jbq, jc, ax, ay, bx, by);
            xj = ring_next(xj);
            yj = ring_next(yj);
            ja = ring_next(ja);
            jbq = ring_next(jbq);
            jc = ring_next(jc);
            bx = ring_next(bx);
            by = ring_next(by);
          }
          rev[tj][0][jl] -= bx;
          rev[tj][1][jl] -= by;
        }
      }
    }
    // the row tile's sums: waves 1..3 through LDS to wave 0, in a fixed order
    if (wv > 0) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        red[wv - 1][2 * t][lane] = ax[t];
        red[wv - 1][2 * t + 1][lane] = ay[t];
      }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int o = 0; o < kWaves - 1; ++o)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          ax[t] += red[o][2 * t][lane];
          ay[t] += red[o][2 * t + 1][lane];
        }
      double *po = P + ((int64_t)Kr * (R + 1) + (Kcu - Kr)) * slot_doubles + (int64_t)ti * kSymTile;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        po[lane + t * kTileLanes] = ax[t];
        po[kSymSBN + lane + t * kTileLanes] = ay[t];
      }
    }
    __syncthreads();
  }
  // the column tiles' sums
  double *pc = P + ((int64_t)Kcu * (R + 1) + (R - Kcu) + Kr) * slot_doubles;
  for (int tj = 0; tj < kSymSB; ++tj) {
    if (Kcu * kSymSB + tj >= ntiles) break;
    for (int e = threadIdx.x; e < kSymTile; e += blockDim.x) {
      pc[(int64_t)tj * kSymTile + e] = rev[tj][0][e];
      pc[kSymSBN + (int64_t)tj * kSymTile + e] = rev[tj][1][e];
    }
  }
}

// part[i], part[nn + i] = the R + 1 slots of node i, added in slot order.
__global__ void sym_reduce(const double *__restrict__ P, int64_t nn, int R, double *__restrict__ part) {
  constexpr int sbn = kSymSBN;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int64_t K = i / sbn, il = i - K * sbn;
  const double *p = P + K * (R + 1) * 2 * (int64_t)sbn + il;
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s <= R; ++s) {
    sx += p[(int64_t)s * 2 * sbn];
    sy += p[(int64_t)s * 2 * sbn + sbn];
  }
  part[i] = sx;
  part[nn + i] = sy;
}

// Stokeslet + rotlet columns: sum over pores of S(x_i - c_k) lambda_k
// + r_k R(x_i - c_k) mu_k, without the 1/(4 pi) (applied in the epilogue).
template <bool ACC>
__device__ __forceinline__ void completion_body(const double *__restrict__ psrc, const double *__restrict__ xs,
                                                const double *__restrict__ ys, int64_t nn, int m,
                                                double *__restrict__ part, int64_t tile, int pc) {
  const int64_t i0 = tile * kBlock + threadIdx.x;
  const int64_t i = i0 < nn ? i0 : nn - 1;
  const double xi = xs[i], yi = ys[i];
  double ax = 0.0, ay = 0.0, cxa = 0.0, cya = 0.0;
  const int k0 = pc * kPoreChunk;
  const int k1 = k0 + kPoreChunk < m ? k0 + kPoreChunk : m;
  for (int k = k0; k < k1; ++k) {
    const double *p = psrc + 8 * k;
    const double qx = xi - p[0], qy = yi - p[1];
    const double lx = p[2], ly = p[3], rmu = p[4];
    const double q2 = fma(qy, qy, qx * qx);
    const double inv = 1.0 / q2;
    const double lg = 0.5 * log(q2);
    const double dot = fma(qy, ly, qx * lx) * inv;
    const double tx = -lg * lx + qx * dot + rmu * qy * inv;
    const double ty = -lg * ly + qy * dot - rmu * qx * inv;
    if (ACC) {
      two_sum_acc(ax, cxa, tx);
      two_sum_acc(ay, cya, ty);
    } else {
      ax += tx;
      ay += ty;
    }
  }
  if (i0 < nn) {
    double *px = part + (int64_t)pc * (ACC ? 4 : 2) * nn;
    px[i0] = ax;
    px[nn + i0] = ay;
    if (ACC) {
      px[2 * nn + i0] = cxa;
      px[3 * nn + i0] = cya;
    }
  }
}

template <bool ACC>
__global__ __launch_bounds__(kBlock) void completion_pairs(
    const double *__restrict__ psrc, const double *__restrict__ xs,
    const double *__restrict__ ys, int64_t nn, int m,
    double *__restrict__ part) {
  completion_body<ACC>(psrc, xs, ys, nn, m, part, blockIdx.x, blockIdx.y);
}

__device__ __forceinline__ void epilogue_body(int64_t i, int64_t nn, int64_t wall_start, int nchunks,
                                              int npchunks, int full, int acc,
                                              const double *__restrict__ part,
                                              const double *__restrict__ nx,
                                              const double *__restrict__ ny,
                                              const double *__restrict__ w,
                                              const double *__restrict__ kappa,
                                              const double *__restrict__ u,
                                              const double *__restrict__ scal,
                                              double *__restrict__ out) {
  if (i >= nn) return;
  // (value, error) pairs; the error parts are only used in the compensated
  // mode, where every addition below is a two-sum
  double vx = 0.0, vy = 0.0, ex = 0.0, ey = 0.0;
  auto add = [&](double &v, double &e, double a) {
    if (acc) two_sum_acc(v, e, a); else v += a;
  };
  const int64_t stride = (acc ? 4 : 2) * nn;   // doubles per partial sum
  for (int c = 0; c < nchunks; ++c) {
    const double *p = part + (int64_t)c * stride;
    add(vx, ex, p[i]);
    add(vy, ey, p[nn + i]);
    if (acc) {
      ex += p[2 * nn + i];
      ey += p[3 * nn + i];
    }
  }
  const double sx = u[i], sy = u[nn + i];
  const double tx = -ny[i], ty = nx[i];
  const double d = w[i] * kappa[i] * (0.5 / kPi) * (tx * sx + ty * sy);
  add(vx, ex, d * tx);
  add(vy, ey, d * ty);
  if (full) {
    double cx = 0.0, cy = 0.0, ecx = 0.0, ecy = 0.0;
    for (int c = 0; c < npchunks; ++c) {
      const double *p = part + (int64_t)(nchunks + c) * stride;
      add(cx, ecx, p[i]);
      add(cy, ecy, p[nn + i]);
      if (acc) {
        ecx += p[2 * nn + i];
        ecy += p[3 * nn + i];
      }
    }
    add(vx, ex, cx * (0.25 / kPi));
    add(vx, ex, ecx * (0.25 / kPi));
    add(vy, ey, cy * (0.25 / kPi));
    add(vy, ey, ecy * (0.25 / kPi));
    add(vx, ex, -0.5 * sx);
    add(vy, ey, -0.5 * sy);
    if (i >= wall_start) {
      const double f = scal[0] / scal[1];
      add(vx, ex, nx[i] * f);
      add(vy, ey, ny[i] * f);
    }
  }
  out[i] = vx + ex;
  out[nn + i] = vy + ey;
}

__global__ void epilogue(int64_t nn, int64_t wall_start, int nchunks,
                         int npchunks, int full, int acc,
                         const double *__restrict__ part,
                         const double *__restrict__ nx,
                         const double *__restrict__ ny,
                         const double *__restrict__ w,
                         const double *__restrict__ kappa,
                         const double *__restrict__ u,
                         const double *__restrict__ scal,
                         double *__restrict__ out) {
  epilogue_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, nn, wall_start, nchunks, npchunks, full, acc,
                part, nx, ny, w, kappa, u, scal, out);
}

// One wave per pore: the constraint rows lambda_k and mu_k.
__device__ __forceinline__ void pore_rows_body(int k, int64_t nn, int m, const int64_t *__restrict__ off,
                                               const double *__restrict__ x,
                                               const double *__restrict__ y,
                                               const double *__restrict__ w,
                                               const double *__restrict__ cx,
                                               const double *__restrict__ cy,
                                               const double *__restrict__ rad,
                                               const double *__restrict__ u, int full,
                                               double *__restrict__ out) {
  if (k >= m) return;
  double sx = 0.0, sy = 0.0, sm = 0.0;
  if (full) {
    const int64_t a = off[k], b = off[k + 1];
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      const double ux = u[j], uy = u[nn + j];
      sx += w[j] * ux;
      sy += w[j] * uy;
      // (x_j - c_k)_perp . sigma = (y_j - cy) ux - (x_j - cx) uy
      sm += w[j] * ((y[j] - cy[k]) * ux - (x[j] - cx[k]) * uy);
    }
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_down(sx, o, 64);
      sy += __shfl_down(sy, o, 64);
      sm += __shfl_down(sm, o, 64);
    }
  }
  if (threadIdx.x == 0) {
    double *o = out + 2 * nn + 3 * (int64_t)k;
    if (full) {
      const double *lam = u + 2 * nn + 3 * (int64_t)k;
      const double r = rad[k];
      o[0] = sx / (2.0 * kPi * r) - lam[0];
      o[1] = sy / (2.0 * kPi * r) - lam[1];
      o[2] = sm / (2.0 * kPi * r * r) - lam[2];
    } else {
      o[0] = o[1] = o[2] = 0.0;
    }
  }
}

__global__ void pore_rows(int64_t nn, int m, const int64_t *__restrict__ off,
                          const double *__restrict__ x,
                          const double *__restrict__ y,
                          const double *__restrict__ w,
                          const double *__restrict__ cx,
                          const double *__restrict__ cy,
                          const double *__restrict__ rad,
                          const double *__restrict__ u, int full,
                          double *__restrict__ out) {
  pore_rows_body(blockIdx.x, nn, m, off, x, y, w, cx, cy, rad, u, full, out);
}

__global__ void wall_length_kernel(int64_t wall_start, int64_t nn,
                                   const double *__restrict__ w, double *out) {
  __shared__ double sl[256];
  double l = 0.0;
  for (int64_t i = wall_start + threadIdx.x; i < nn; i += blockDim.x) l += w[i];
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sl[threadIdx.x] += sl[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sl[0];
}

}  // namespace

size_t MatvecWork::doubles() const { return 0; }

// Workgroups of the plain pair kernel (targets per thread tpt) that the whole
// device holds at once: occupancy per compute unit times the unit count.
int64_t resident_pair_blocks(int tpt) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int64_t> cache;
  int dev = 0;
  SBIE_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({dev, tpt});
  if (it != cache.end()) return it->second;
  const void *fn = nullptr;
  switch (tpt) {
    case 1: fn = reinterpret_cast<const void *>(&dlp_pairs<1, false>); break;
    case 2: fn = reinterpret_cast<const void *>(&dlp_pairs<2, false>); break;
    case 4: fn = reinterpret_cast<const void *>(&dlp_pairs<4, false>); break;
    default: fn = reinterpret_cast<const void *>(&dlp_pairs<8, false>); break;
  }
  int per_cu = 0, cus = 0;
  SBIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0));
  SBIE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t r = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  cache[{dev, tpt}] = r;
  return r;
}

// Source chunks for the pair kernel.  All (tile, chunk) workgroups cost the
// same; with few of them per resident slot the last, partly filled round of
// workgroups is a large share of the run.  About eight rounds of the
// device's resident workgroups keep that share small; the partial sums (2 nn
// doubles per chunk, re-read by the epilogue) are then a few percent of the
// pair time.  Chunks hold at least 256 sources (64 per wave).
int choose_chunks(int64_t nn, int64_t tiles, int tpt) {
  const int64_t resident = resident_pair_blocks(tpt);
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>((nn + 255) / 256, 1024));
  const int64_t want = (8 * resident + tiles - 1) / tiles;
  int64_t c = std::max<int64_t>(1, std::min(want, cap));
  if (c >= 16) c &= ~int64_t(7);   // a multiple of 8 for the XCD-aware order
  return (int)c;
}

MatvecWork plan_matvec(const sbie_geom *g, bool allow_sym) {
  MatvecWork w;
  w.tpt = g_tpt;
  const int64_t nn = g->n_nodes;
  // symmetric evaluation: one superblock pair per workgroup needs enough
  // pairs to fill the device (from about 16k nodes), and its partial sums
  // grow as nn^2 / 1024 doubles (bounded here by 128 superblocks, 131,072
  // nodes, 270 MB); the explicit chunk count of the launch-shape hook asks
  // for the chunked kernel
  const int64_t ntiles = (nn + kSymTile - 1) / kSymTile;
  const int64_t R = (ntiles + kSymSB - 1) / kSymSB;
  if (allow_sym && g_chunks == 0 && R <= 128 &&
      (g_sym_mode == 2 || (g_sym_mode == 1 && nn >= 16384))) {
    w.sym = 1;
    w.sym_R = (int)R;
    w.chunks = 1;
    w.pchunks = g->n_pores > 0 ? (int)ceil_div(g->n_pores, kPoreChunk) : 0;
    return w;
  }
  const int64_t tiles = ceil_div(nn, (int64_t)kTileLanes * w.tpt);
  if (g_chunks > 0) {
    w.chunks = g_chunks;
  } else {
    w.chunks = choose_chunks(nn, tiles, w.tpt);
  }
  if ((int64_t)w.chunks > nn) w.chunks = (int)nn;
  w.pchunks = g->n_pores > 0 ? (int)ceil_div(g->n_pores, kPoreChunk) : 0;
  return w;
}

size_t matvec_scratch_doubles(const MatvecWork &w, const sbie_geom *g) {
  const int64_t nn = g->n_nodes;
  return (size_t)8 * nn + (size_t)8 * (g->n_pores + 1) +
         (size_t)(w.chunks + w.pchunks) * 4 * nn + 8 +
         (w.sym ? (size_t)w.sym_R * (w.sym_R + 1) * 2 * kSymSBN : 0);
}

void bind_matvec_scratch(MatvecWork &w, const sbie_geom *g, double *base) {
  const int64_t nn = g->n_nodes;
  // records, then the two scalars, then the partial sums (their size
  // depends on the mode and is last so that a smaller mode needs less)
  w.src = base;
  w.psrc = w.src + 8 * nn;
  w.scal = w.psrc + 8 * (g->n_pores + 1);
  w.part = w.scal + 8;
  w.sym_buf = w.sym ? w.part + (size_t)(w.chunks + w.pchunks) * 4 * nn : nullptr;
}

void matvec_run(const sbie_geom *g, const double *x, double *y, int mode,
                MatvecWork &w, hipStream_t s, const PairSum *pairs) {
  const int64_t nn = g->n_nodes;
  const int m = g->n_pores;
  const int full = mode == SBIE_MV_FULL || mode == SBIE_MV_FULL_ACCURATE;
  const bool acc = mode == SBIE_MV_FULL_ACCURATE;
  if (pairs && (acc || w.chunks != 1))
    fail(SBIE_UNSUPPORTED, "the fast multipole pair sum has no compensated mode");
  const int64_t wall_start = g->curve_off[m];
  const int64_t packn = nn > m ? nn : m;
  pack_sources<<<ceil_div(packn, 256), 256, 0, s>>>(
      nn, m, g->x, g->y, g->nx, g->ny, g->w, g->radius, g->cx, g->cy, x,
      w.src, w.psrc);
  SBIE_LAUNCH_CHECK();
  if (full) {
    wall_flux<<<1, 1024, 0, s>>>(wall_start, nn, g->nx, g->ny, g->w, x, w.scal, 1);
    SBIE_LAUNCH_CHECK();
  }
  const int64_t chunk = (nn + w.chunks - 1) / w.chunks;
  const int tiles = (int)ceil_div(nn, (int64_t)kTileLanes * w.tpt);
  if (w.sym && acc)
    fail(SBIE_INVALID_ARGUMENT, "the compensated product needs a chunked plan (plan_matvec with allow_sym off)");
  const int xcd = (w.chunks % 8 == 0) ? 1 : 0;
  const unsigned grid = (unsigned)((int64_t)tiles * w.chunks);
  const int tiles1 = (int)ceil_div(nn, kTileLanes);
  const unsigned grid1 = (unsigned)((int64_t)tiles1 * w.chunks);
  const int64_t stride = (acc ? 4 : 2) * nn;   // doubles per partial sum
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // only the plain pair kernel is timed (the compensated one is a
  // different kernel, launched for true residuals)
  if (g_timing && !acc) {
    SBIE_HIP(hipEventCreate(&ev0));
    SBIE_HIP(hipEventCreate(&ev1));
    SBIE_HIP(hipEventRecord(ev0, s));
  }
  if (pairs) {
    pairs->run(w.src, w.part, s);
  } else if (w.sym && !acc) {
    const int ntiles = (int)ceil_div(nn, kSymTile);
    const int R = w.sym_R;
    if ((int64_t)R * kSymSB < ntiles || w.chunks != 1 || !w.sym_buf)
      fail(SBIE_INVALID_ARGUMENT, "symmetric pair plan does not match the geometry");
    dlp_pairs_sym<<<(unsigned)((int64_t)R * (R + 1) / 2), kBlock, 0, s>>>(w.src, g->x, g->y, nn, ntiles, R,
                                                                          w.sym_buf);
    SBIE_LAUNCH_CHECK();
    sym_reduce<<<ceil_div(nn, 256), 256, 0, s>>>(w.sym_buf, nn, R, w.part);
  } else if (acc) {
    dlp_pairs<1, true><<<grid1, kBlock, 0, s>>>(w.src, g->x, g->y, nn, nn, chunk, w.part, tiles1, xcd);
  } else {
    switch (w.tpt) {
      case 1: dlp_pairs<1, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, nn, chunk, w.part, tiles, xcd); break;
      case 2: dlp_pairs<2, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, nn, chunk, w.part, tiles, xcd); break;
      case 4: dlp_pairs<4, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, nn, chunk, w.part, tiles, xcd); break;
      case 8: dlp_pairs<8, false><<<grid, kBlock, 0, s>>>(w.src, g->x, g->y, nn, nn, chunk, w.part, tiles, xcd); break;
      default: fail(SBIE_INVALID_ARGUMENT, "targets per thread must be 1, 2, 4 or 8");
    }
  }
  SBIE_LAUNCH_CHECK();
  if (g_timing && !acc) {
    SBIE_HIP(hipEventRecord(ev1, s));
    g_events.emplace_back(ev0, ev1);
  }
  if (full && m > 0) {
    dim3 pg(ceil_div(nn, kBlock), w.pchunks);
    if (acc)
      completion_pairs<true><<<pg, kBlock, 0, s>>>(w.psrc, g->x, g->y, nn, m,
                                                   w.part + (size_t)w.chunks * stride);
    else
      completion_pairs<false><<<pg, kBlock, 0, s>>>(w.psrc, g->x, g->y, nn, m,
                                                    w.part + (size_t)w.chunks * stride);
    SBIE_LAUNCH_CHECK();
  }
  epilogue<<<ceil_div(nn, 256), 256, 0, s>>>(nn, wall_start, w.chunks,
                                             full ? w.pchunks : 0, full, acc ? 1 : 0, w.part,
                                             g->nx, g->ny, g->w, g->kappa, x,
                                             w.scal, y);
  SBIE_LAUNCH_CHECK();
  if (m > 0) {
    pore_rows<<<m, 64, 0, s>>>(nn, m, g->curve_off_dev, g->x, g->y, g->w,
                               g->cx, g->cy, g->radius, x, full, y);
    SBIE_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// Velocity at points of the fluid from a solved density: the same source
// records, pair and completion kernels with the points as targets (no self
// pair, no jump, no diagonal limit, no wall term), then one epilogue.
// ---------------------------------------------------------------------------
namespace {

__global__ void velocity_epilogue(int64_t np, int nchunks, int npchunks, const double *__restrict__ part,
                                  double *__restrict__ ux, double *__restrict__ uy,
                                  const double *__restrict__ rx, const double *__restrict__ ry,
                                  double *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double vx = 0.0, vy = 0.0, cx = 0.0, cy = 0.0;
  for (int c = 0; c < nchunks; ++c) {
    const double *p = part + (int64_t)c * 2 * np;
    vx += p[i];
    vy += p[np + i];
  }
  for (int c = 0; c < npchunks; ++c) {
    const double *p = part + (int64_t)(nchunks + c) * 2 * np;
    cx += p[i];
    cy += p[np + i];
  }
  vx += cx * (0.25 / kPi);
  vy += cy * (0.25 / kPi);
  ux[i] = vx;
  uy[i] = vy;
  if (err) {
    // relative error of the velocity magnitude against a reference field
    const double a = sqrt(vx * vx + vy * vy), b = sqrt(rx[i] * rx[i] + ry[i] * ry[i]);
    err[i] = fabs(a - b) / b;
  }
}

}  // namespace

void velocity_run(const sbie_geom *g, const double *sigma, const double *px, const double *py, int64_t np,
                  double *ux, double *uy, const double *rx, const double *ry, double *err, hipStream_t s) {
  const int64_t nn = g->n_nodes;
  const int m = g->n_pores;
  const int tpt = 4;
  const int tiles = (int)ceil_div(np, (int64_t)kTileLanes * tpt);
  int chunks = g_chunks > 0 ? g_chunks : choose_chunks(nn, tiles, tpt);
  if ((int64_t)chunks > nn) chunks = (int)nn;
  const int pchunks = m > 0 ? (int)ceil_div(m, kPoreChunk) : 0;
  StreamBuf<double> scratch((size_t)8 * nn + (size_t)8 * (m + 1) + (size_t)(chunks + pchunks) * 2 * np, s);
  double *src = scratch.p, *psrc = src + 8 * nn, *part = psrc + 8 * (m + 1);
  pack_sources<<<ceil_div(nn > m ? nn : m, 256), 256, 0, s>>>(nn, m, g->x, g->y, g->nx, g->ny, g->w, g->radius,
                                                             g->cx, g->cy, sigma, src, psrc);
  SBIE_LAUNCH_CHECK();
  const int64_t chunk = (nn + chunks - 1) / chunks;
  const int xcd = (chunks % 8 == 0) ? 1 : 0;
  dlp_pairs<4, false><<<(unsigned)((int64_t)tiles * chunks), kBlock, 0, s>>>(src, px, py, np, nn, chunk, part,
                                                                            tiles, xcd);
  SBIE_LAUNCH_CHECK();
  if (m > 0) {
    dim3 pg(ceil_div(np, kBlock), pchunks);
    completion_pairs<false><<<pg, kBlock, 0, s>>>(psrc, px, py, np, m, part + (size_t)chunks * 2 * np);
    SBIE_LAUNCH_CHECK();
  }
  velocity_epilogue<<<ceil_div(np, 256), 256, 0, s>>>(np, chunks, pchunks, part, ux, uy, rx, ry, err);
  SBIE_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched matvec
// ---------------------------------------------------------------------------
namespace {

struct BMember {
  const double *x, *y, *nx, *ny, *w, *kappa, *cx, *cy, *rad;
  const int64_t *off;
  int64_t nn, wall_start, chunk, tiles, ctiles;
  int m, chunks, pchunks, pad;
  double *src, *psrc, *part, *scal;
  const double *u;
  double *out;
};

enum { kStPack = 0, kStPair, kStComp, kStNode, kStPore, kStages };

// Largest b with st[b] <= unit (members with no units in a stage share the
// start of the next one and are skipped).
__device__ __forceinline__ int find_member(const int64_t *__restrict__ st, int nb, int64_t unit) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st[mid] <= unit) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void pack_b(const BMember *__restrict__ d, const int64_t *__restrict__ st, int nb) {
  const int b = find_member(st, nb, blockIdx.x);
  const BMember &M = d[b];
  const int64_t j = ((int64_t)blockIdx.x - st[b]) * blockDim.x + threadIdx.x;
  pack_body(j, M.nn, M.m, M.x, M.y, M.nx, M.ny, M.w, M.rad, M.cx, M.cy, M.u, M.src, M.psrc);
}

__global__ void wall_flux_b(const BMember *__restrict__ d) {
  const BMember &M = d[blockIdx.x];
  wall_flux_body(M.wall_start, M.nn, M.nx, M.ny, M.w, M.u, M.scal, 1);
}

template <int T, bool ACC>
__global__ __launch_bounds__(kBlock) void dlp_pairs_b(const BMember *__restrict__ d,
                                                      const int64_t *__restrict__ st, int nb) {
  const int b = find_member(st, nb, blockIdx.x);
  const BMember &M = d[b];
  const int64_t u = (int64_t)blockIdx.x - st[b];
  dlp_pairs_body<T, ACC>(M.src, M.x, M.y, M.nn, M.nn, M.chunk, M.part, u % M.tiles, u / M.tiles);
}

// The same work items as dlp_pairs_b (every (member, tile, chunk) of the
// batch) taken from a device work queue by a persistent grid sized to the
// device's resident workgroups: each workgroup draws the next item index
// with one atomic add until the queue is exhausted, so members of any size
// mix freely and no workgroup waits on another.  Results are identical to
// dlp_pairs_b (the same body on the same items).
template <int T, bool ACC>
__global__ __launch_bounds__(kBlock) void dlp_pairs_bq(const BMember *__restrict__ d,
                                                       const int64_t *__restrict__ st, int nb,
                                                       unsigned long long *queue, int64_t total) {
  __shared__ int64_t item;
  for (;;) {
    // the barrier also orders the previous item's LDS reduction before the
    // next item's writes to it
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t u0 = item;
    __syncthreads();
    if (u0 >= total) return;   // uniform over the workgroup
    const int b = find_member(st, nb, u0);
    const BMember &M = d[b];
    const int64_t u = u0 - st[b];
    dlp_pairs_body<T, ACC>(M.src, M.x, M.y, M.nn, M.nn, M.chunk, M.part, u % M.tiles, u / M.tiles);
  }
}

__global__ void reset_queue(unsigned long long *queue) { *queue = 0ull; }

template <bool ACC>
__global__ __launch_bounds__(kBlock) void completion_b(const BMember *__restrict__ d,
                                                       const int64_t *__restrict__ st, int nb) {
  const int b = find_member(st, nb, blockIdx.x);
  const BMember &M = d[b];
  const int64_t u = (int64_t)blockIdx.x - st[b];
  completion_body<ACC>(M.psrc, M.x, M.y, M.nn, M.m, M.part + (int64_t)M.chunks * (ACC ? 4 : 2) * M.nn,
                       u % M.ctiles, (int)(u / M.ctiles));
}

__global__ void epilogue_b(const BMember *__restrict__ d, const int64_t *__restrict__ st, int nb, int full,
                           int acc) {
  const int b = find_member(st, nb, blockIdx.x);
  const BMember &M = d[b];
  const int64_t i = ((int64_t)blockIdx.x - st[b]) * blockDim.x + threadIdx.x;
  epilogue_body(i, M.nn, M.wall_start, M.chunks, full ? M.pchunks : 0, full, acc, M.part, M.nx, M.ny, M.w,
                M.kappa, M.u, M.scal, M.out);
}

__global__ void pore_rows_b(const BMember *__restrict__ d, const int64_t *__restrict__ st, int nb, int full) {
  const int b = find_member(st, nb, blockIdx.x);
  const BMember &M = d[b];
  pore_rows_body((int)(blockIdx.x - st[b]), M.nn, M.m, M.off, M.x, M.y, M.w, M.cx, M.cy, M.rad, M.u, full,
                 M.out);
}

}  // namespace

BatchMatvec::BatchMatvec(const sbie_geom *const *g, int count) {
  tpt = g_tpt;
  size_t total = 0;
  std::vector<size_t> offs;
  for (int b = 0; b < count; ++b) {
    geoms.push_back(g[b]);
    work.push_back(plan_matvec(g[b], false));
    work.back().tpt = tpt;
    offs.push_back(total);
    total += (matvec_scratch_doubles(work.back(), g[b]) + 31) & ~size_t(31);
  }
  scratch.alloc(total);
  for (int b = 0; b < count; ++b) bind_matvec_scratch(work[b], g[b], scratch.p + offs[b]);
  desc_cap = (size_t)count * sizeof(BMember) + (size_t)kStages * (count + 1) * sizeof(int64_t) + 256;
  desc.alloc(desc_cap);
  SBIE_HIP(hipHostMalloc((void **)&hdesc, desc_cap, hipHostMallocDefault));
  SBIE_HIP(hipEventCreateWithFlags(&staged, hipEventDisableTiming));
  queue.alloc(1);
}

BatchMatvec::~BatchMatvec() {
  if (staged) {
    (void)hipEventSynchronize(staged);
    (void)hipEventDestroy(staged);
  }
  if (hdesc) (void)hipHostFree(hdesc);
}

void BatchMatvec::run(const std::vector<int> &members, const std::vector<const double *> &u,
                      const std::vector<double *> &y, int mode, hipStream_t s) {
  std::vector<int> mem = members;
  if (mem.empty())
    for (int b = 0; b < (int)geoms.size(); ++b) mem.push_back(b);
  const int nb = (int)mem.size();
  if (nb == 0) return;
  if ((int)u.size() != nb || (int)y.size() != nb) fail(SBIE_INVALID_ARGUMENT, "batched matvec: vector count");
  const int full = mode == SBIE_MV_FULL || mode == SBIE_MV_FULL_ACCURATE;
  const bool acc = mode == SBIE_MV_FULL_ACCURATE;
  const int T = acc ? 1 : tpt;
  // the previous table must have reached the device before it is rewritten
  SBIE_HIP(hipEventSynchronize(staged));
  BMember *hd = reinterpret_cast<BMember *>(hdesc);
  int64_t *hst = reinterpret_cast<int64_t *>(hdesc + (size_t)nb * sizeof(BMember));
  int64_t acc_st[kStages] = {0, 0, 0, 0, 0};
  for (int a = 0; a < nb; ++a) {
    const sbie_geom *g = geoms[mem[a]];
    const MatvecWork &w = work[mem[a]];
    BMember &M = hd[a];
    M.x = g->x; M.y = g->y; M.nx = g->nx; M.ny = g->ny; M.w = g->w; M.kappa = g->kappa;
    M.cx = g->cx; M.cy = g->cy; M.rad = g->radius; M.off = g->curve_off_dev;
    M.nn = g->n_nodes;
    M.m = g->n_pores;
    M.wall_start = g->curve_off[g->n_pores];
    M.chunks = w.chunks;
    M.pchunks = w.pchunks;
    M.pad = 0;
    M.chunk = (M.nn + w.chunks - 1) / w.chunks;
    M.tiles = ceil_div(M.nn, (int64_t)kTileLanes * T);
    M.ctiles = ceil_div(M.nn, kBlock);
    M.src = w.src; M.psrc = w.psrc; M.part = w.part; M.scal = w.scal;
    M.u = u[a];
    M.out = y[a];
    const int64_t units[kStages] = {
        (int64_t)ceil_div(M.nn > M.m ? M.nn : M.m, 256), M.tiles * M.chunks,
        (full && M.m > 0) ? M.ctiles * M.pchunks : 0, (int64_t)ceil_div(M.nn, 256), (int64_t)M.m};
    for (int q = 0; q < kStages; ++q) {
      hst[(size_t)q * (nb + 1) + a] = acc_st[q];
      acc_st[q] += units[q];
    }
  }
  for (int q = 0; q < kStages; ++q) hst[(size_t)q * (nb + 1) + nb] = acc_st[q];
  const size_t bytes = (size_t)nb * sizeof(BMember) + (size_t)kStages * (nb + 1) * sizeof(int64_t);
  SBIE_HIP(hipMemcpyAsync(desc.p, hdesc, bytes, hipMemcpyHostToDevice, s));
  SBIE_HIP(hipEventRecord(staged, s));
  const BMember *dd = reinterpret_cast<const BMember *>(desc.p);
  const int64_t *dst = reinterpret_cast<const int64_t *>(desc.p + (size_t)nb * sizeof(BMember));
  auto stt = [&](int q) { return dst + (size_t)q * (nb + 1); };
  auto grid = [&](int q) -> unsigned {
    if (acc_st[q] > (int64_t)0x7fffffff) fail(SBIE_INVALID_ARGUMENT, "batch too large for one launch");
    return (unsigned)acc_st[q];
  };
  pack_b<<<grid(kStPack), 256, 0, s>>>(dd, stt(kStPack), nb);
  SBIE_LAUNCH_CHECK();
  if (full) {
    wall_flux_b<<<nb, 1024, 0, s>>>(dd);
    SBIE_LAUNCH_CHECK();
  }
  if (g_batch_queue && acc_st[kStPair] > 0) {
    // persistent grid: as many workgroups as the device holds at once (the
    // occupancy of the plain kernel with this shape), at most one per item
    const int64_t items = acc_st[kStPair];
    const unsigned pg = (unsigned)std::min<int64_t>(items, resident_pair_blocks(T));
    reset_queue<<<1, 1, 0, s>>>(queue.p);
    SBIE_LAUNCH_CHECK();
    if (acc) {
      dlp_pairs_bq<1, true><<<pg, kBlock, 0, s>>>(dd, stt(kStPair), nb, queue.p, items);
    } else {
      switch (T) {
        case 1: dlp_pairs_bq<1, false><<<pg, kBlock, 0, s>>>(dd, stt(kStPair), nb, queue.p, items); break;
        case 2: dlp_pairs_bq<2, false><<<pg, kBlock, 0, s>>>(dd, stt(kStPair), nb, queue.p, items); break;
        case 4: dlp_pairs_bq<4, false><<<pg, kBlock, 0, s>>>(dd, stt(kStPair), nb, queue.p, items); break;
        case 8: dlp_pairs_bq<8, false><<<pg, kBlock, 0, s>>>(dd, stt(kStPair), nb, queue.p, items); break;
        default: fail(SBIE_INVALID_ARGUMENT, "targets per thread must be 1, 2, 4 or 8");
      }
    }
  } else if (acc) {
    dlp_pairs_b<1, true><<<grid(kStPair), kBlock, 0, s>>>(dd, stt(kStPair), nb);
  } else {
    switch (T) {
      case 1: dlp_pairs_b<1, false><<<grid(kStPair), kBlock, 0, s>>>(dd, stt(kStPair), nb); break;
      case 2: dlp_pairs_b<2, false><<<grid(kStPair), kBlock, 0, s>>>(dd, stt(kStPair), nb); break;
      case 4: dlp_pairs_b<4, false><<<grid(kStPair), kBlock, 0, s>>>(dd, stt(kStPair), nb); break;
      case 8: dlp_pairs_b<8, false><<<grid(kStPair), kBlock, 0, s>>>(dd, stt(kStPair), nb); break;
      default: fail(SBIE_INVALID_ARGUMENT, "targets per thread must be 1, 2, 4 or 8");
    }
  }
  SBIE_LAUNCH_CHECK();
  if (acc_st[kStComp] > 0) {
    if (acc)
      completion_b<true><<<grid(kStComp), kBlock, 0, s>>>(dd, stt(kStComp), nb);
    else
      completion_b<false><<<grid(kStComp), kBlock, 0, s>>>(dd, stt(kStComp), nb);
    SBIE_LAUNCH_CHECK();
  }
  epilogue_b<<<grid(kStNode), 256, 0, s>>>(dd, stt(kStNode), nb, full, acc ? 1 : 0);
  SBIE_LAUNCH_CHECK();
  if (acc_st[kStPore] > 0) {
    pore_rows_b<<<grid(kStPore), 64, 0, s>>>(dd, stt(kStPore), nb, full);
    SBIE_LAUNCH_CHECK();
  }
}

void wall_length(const sbie_geom *g, double *out, hipStream_t s) {
  wall_length_kernel<<<1, 256, 0, s>>>(g->curve_off[g->n_pores], g->n_nodes,
                                       g->w, out);
  SBIE_LAUNCH_CHECK();
}

}  // namespace sbie

extern "C" int stokes_dlp_matvec(const sbie_geom *g, const double *x, double *y,
                                 int mode, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!x || !y) sbie::fail(SBIE_INVALID_ARGUMENT, "null vector");
    if (mode != SBIE_MV_FULL && mode != SBIE_MV_DLP_ONLY && mode != SBIE_MV_FULL_ACCURATE)
      sbie::fail(SBIE_INVALID_ARGUMENT, "unknown matvec mode %d", mode);
    const int64_t n = sbie::n_unknowns(g);
    if (x < y + n && y < x + n)
      sbie::fail(SBIE_INVALID_ARGUMENT, "x and y overlap");
    hipStream_t s = (hipStream_t)stream;
    sbie::MatvecWork w = sbie::plan_matvec(g, mode != SBIE_MV_FULL_ACCURATE);
    sbie::StreamBuf<double> scratch(sbie::matvec_scratch_doubles(w, g), s);
    sbie::bind_matvec_scratch(w, g, scratch.p);
    sbie::matvec_run(g, x, y, mode, w, s);
    return SBIE_OK;
  });
}

// ---------------------------------------------------------------------------
// Matvec without allocation: the same kernels with their scratch in a fixed
// device array of the library.  Its name is a host-side stand-in in host
// code; the device address of each GPU's copy is looked up once per device
// and only that address is passed to kernels.
// ---------------------------------------------------------------------------
namespace sbie {
namespace {

constexpr size_t kNoAllocDoubles = size_t(64) << 17;   // 64 MiB of FP64
__device__ __align__(256) double g_noalloc_scratch[kNoAllocDoubles];

std::mutex g_noalloc_mu;
std::vector<double *> g_noalloc_ptr;   // per device, looked up on first use

double *noalloc_scratch() {
  int dev = 0;
  SBIE_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if ((int)g_noalloc_ptr.size() <= dev) g_noalloc_ptr.resize(dev + 1, nullptr);
  if (!g_noalloc_ptr[dev]) {
    void *ptr = nullptr;
    SBIE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch)));
    if (!ptr) fail(SBIE_HIP_ERROR, "no device address for the matvec scratch array");
    g_noalloc_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_noalloc_ptr[dev];
}

}  // namespace
}  // namespace sbie

extern "C" int stokes_dlp_matvec_noalloc(const sbie_geom *g, const double *x, double *y, int mode,
                                         void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!x || !y) sbie::fail(SBIE_INVALID_ARGUMENT, "null vector");
    if (mode != SBIE_MV_FULL && mode != SBIE_MV_DLP_ONLY && mode != SBIE_MV_FULL_ACCURATE)
      sbie::fail(SBIE_INVALID_ARGUMENT, "unknown matvec mode %d", mode);
    const int64_t n = sbie::n_unknowns(g);
    if (x < y + n && y < x + n) sbie::fail(SBIE_INVALID_ARGUMENT, "x and y overlap");
    sbie::MatvecWork w = sbie::plan_matvec(g, false);
    // fit the source chunks into the fixed array: records and scalars, then
    // one partial sum (2 or 4 doubles per node) per pair and pore chunk
    const int64_t nn = g->n_nodes;
    const int64_t per = (mode == SBIE_MV_FULL_ACCURATE ? 4 : 2) * nn;
    const int64_t fixed = 8 * nn + 8 * ((int64_t)g->n_pores + 1) + 8;
    const int64_t room = (int64_t)sbie::kNoAllocDoubles - fixed;
    const int64_t max_chunks = room > 0 ? room / per - w.pchunks : 0;
    if (max_chunks < 1)
      sbie::fail(SBIE_INVALID_ARGUMENT,
                 "problem too large for the %zu MiB no-allocation scratch (%lld nodes, %d pores)",
                 sbie::kNoAllocDoubles * sizeof(double) >> 20, (long long)nn, (int)g->n_pores);
    if (w.chunks > max_chunks) {
      int64_t c = max_chunks;
      if (c >= 16) c &= ~int64_t(7);
      w.chunks = (int)c;
    }
    sbie::bind_matvec_scratch(w, g, sbie::noalloc_scratch());
    sbie::matvec_run(g, x, y, mode, w, (hipStream_t)stream);
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_batched(const sbie_geom *geoms, int32_t count, const double *const *x,
                                         double *const *y, int mode, void *stream) {
  return sbie::guarded([&]() {
    if (count < 0 || (count > 0 && (!geoms || !x || !y))) sbie::fail(SBIE_INVALID_ARGUMENT, "bad batch");
    if (mode != SBIE_MV_FULL && mode != SBIE_MV_DLP_ONLY && mode != SBIE_MV_FULL_ACCURATE)
      sbie::fail(SBIE_INVALID_ARGUMENT, "unknown matvec mode %d", mode);
    if (count == 0) return SBIE_OK;
    std::vector<const sbie_geom *> gp;
    std::vector<const double *> u;
    std::vector<double *> out;
    for (int b = 0; b < count; ++b) {
      sbie::validate_geom(&geoms[b]);
      if (!x[b] || !y[b]) sbie::fail(SBIE_INVALID_ARGUMENT, "null vector for member %d", b);
      const int64_t n = sbie::n_unknowns(&geoms[b]);
      if (x[b] < y[b] + n && y[b] < x[b] + n) sbie::fail(SBIE_INVALID_ARGUMENT, "x and y overlap (member %d)", b);
      gp.push_back(&geoms[b]);
      u.push_back(x[b]);
      out.push_back(y[b]);
    }
    sbie::BatchMatvec bm(gp.data(), count);
    bm.run({}, u, out, mode, (hipStream_t)stream);
    // the batch's scratch is freed on return: wait for its kernels
    SBIE_HIP(hipStreamSynchronize((hipStream_t)stream));
    return SBIE_OK;
  });
}

extern "C" int stokes_velocity(const sbie_geom *g, const double *sigma, const double *px, const double *py,
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
    sbie::velocity_run(g, sigma, px, py, np, ux, uy, uref_x, uref_y, err, (hipStream_t)stream);
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_set_shape(int targets_per_thread,
                                           int source_chunks) {
  return sbie::guarded([&]() {
    if (targets_per_thread != 1 && targets_per_thread != 2 &&
        targets_per_thread != 4 && targets_per_thread != 8)
      sbie::fail(SBIE_INVALID_ARGUMENT, "targets per thread must be 1, 2, 4 or 8");
    if (source_chunks < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "source_chunks < 0");
    sbie::g_tpt = targets_per_thread;
    sbie::g_chunks = source_chunks;
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_describe_plan(const sbie_geom *g, int mode, int32_t *symmetric, int32_t *chunks,
                                              int32_t *targets_per_thread) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!symmetric || !chunks || !targets_per_thread) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    const sbie::MatvecWork w = sbie::plan_matvec(g, mode != SBIE_MV_FULL_ACCURATE);
    *symmetric = w.sym;
    *chunks = w.chunks;
    *targets_per_thread = w.sym ? sbie::kSymT : (mode == SBIE_MV_FULL_ACCURATE ? 1 : w.tpt);
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_set_symmetric(int mode) {
  return sbie::guarded([&]() {
    if (mode < 0 || mode > 2) sbie::fail(SBIE_INVALID_ARGUMENT, "mode must be 0, 1 or 2");
    sbie::g_sym_mode = mode;
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_batched_set_schedule(int persistent) {
  return sbie::guarded([&]() {
    if (persistent != 0 && persistent != 1) sbie::fail(SBIE_INVALID_ARGUMENT, "persistent must be 0 or 1");
    sbie::g_batch_queue = persistent;
    return SBIE_OK;
  });
}

extern "C" int sbie_kernel_timing(int enable) {
  return sbie::guarded([&]() {
    sbie::g_timing = enable != 0;
    return SBIE_OK;
  });
}

extern "C" int sbie_kernel_time(double *total_ms, int64_t *launches) {
  return sbie::guarded([&]() {
    if (!total_ms || !launches) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    double tot = 0.0;
    for (auto &e : sbie::g_events) {
      SBIE_HIP(hipEventSynchronize(e.second));
      float ms = 0.0f;
      SBIE_HIP(hipEventElapsedTime(&ms, e.first, e.second));
      tot += ms;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    *total_ms = tot;
    *launches = (int64_t)sbie::g_events.size();
    sbie::g_events.clear();
    return SBIE_OK;
  });
}

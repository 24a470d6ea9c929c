// Fast multipole evaluation of the double-layer pair sum: the products of
// GMRES evaluated in O(N) work instead of O(N^2) (Section 2.2 notes that the
// matrix-vector products can be accelerated by a fast multipole method; the
// far field is approximated by Chebyshev interpolation, the construction of
// the H^2 operators of Section 3.1).
//
// The pair sum at node x_i is  sum_j r (r^T q_j r) / rho^4,  r = x_i - y_j,
// with q_j = (w_j / pi) n_j sigma_j^T (only its symmetric part matters): a
// kernel that is smooth away from r = 0 and linear in q.  For a target box
// X and a well-separated source box Y it is interpolated in both boxes on
// p x p tensor Chebyshev grids (nodes t_k = cos((2k+1) pi / (2p))):
//   K(x, y) ~ sum_a sum_b S_a(x) K(xbar_a, ybar_b) S_b(y),
//   S_k(t) = 1/p + 2/p sum_{m=1}^{p-1} T_m(t_k) T_m(t)  (per direction),
// so each box carries p^2 multipole tensors Qbar_b = sum_j S_b(y_j) q_j
// (3 numbers each) and p^2 local velocities L_a (2 numbers each).
//
// Tree: the bounding square of all nodes, subdivided uniformly to depth L
// (only non-empty boxes are kept), Morton order.  Per matvec:
//   fmm_gather   source records in leaf order (SoA)
//   fmm_p2m      leaf multipoles from the sources
//   fmm_m2m      parent multipoles from the children (exact: a parent's
//                interpolant is a polynomial the child grids reproduce)
//   fmm_m2l      every box at level >= 2: kernel between its grid and the
//                grids of its interaction list (children of the parent's
//                neighbours that are not neighbours of the box)
//   fmm_l2l      children's locals += parent's local, interpolated
//   fmm_leaf     per leaf: the local expansion at every target plus the
//                direct sum over the neighbouring leaves (itself included)
// The output is the pair sum in node order, which the matvec's epilogue
// completes (jump, diagonal limit, Stokeslet/rotlet columns, wall term).
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "common.hpp"
#include "fmm_tree.hpp"
#include "pairmath.hpp"

struct sbie_fmm;

namespace sbie {
namespace {

constexpr int kFmmThreads = 256;
constexpr int kLeafThreads = 64;

// S_k(t), k = 0..P-1, for one coordinate t in [-1, 1]; tm[k * P + m] =
// T_m(t_k).
template <int P>
__device__ __forceinline__ void cheb_interp(const double *__restrict__ tm, double t, double *s) {
  double T[P];
  T[0] = 1.0;
  if (P > 1) T[1] = t;
#pragma unroll
  for (int m = 2; m < P; ++m) T[m] = 2.0 * t * T[m - 1] - T[m - 2];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int m = 1; m < P; ++m) acc = fma(tm[k * P + m], T[m], acc);
    s[k] = (1.0 + 2.0 * acc) * (1.0 / P);
  }
}

// One pair of the double-layer sum: source at (sx, sy) with tensor
// (qa, qb, qc) = (q_xx, q_xy + q_yx, q_yy), target at (xi, yi).  The self
// pair (r = 0) contributes zero: the 1e-100 inside the fused multiply-add
// keeps 1/rho^4 finite and the contribution is a multiple of r = 0.
__device__ __forceinline__ void dl_pair(double xi, double yi, double sx, double sy, double qa, double qb,
                                        double qc, double &ax, double &ay) {
  const double rx = xi - sx, ry = yi - sy;
  const double ryy = fma(ry, ry, 1e-100);
  const double r2 = fma(rx, rx, ryy);
  const double inv = recip(r2);
  const double h = fma(qb, ry, qa * rx);
  const double pq = fma(h, rx, qc * ryy);
  const double c = pq * (inv * inv);
  ax = fma(c, rx, ax);
  ay = fma(c, ry, ay);
}

__global__ void fmm_gather(int64_t nn, const int *__restrict__ perm, const double *__restrict__ src,
                           double *__restrict__ srt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const double *r = src + 8 * (int64_t)perm[k];
  srt[k] = r[0];
  srt[nn + k] = r[1];
  srt[2 * nn + k] = r[2];
  srt[3 * nn + k] = r[3];
  srt[4 * nn + k] = r[4];
}

// One workgroup per leaf; thread b < P^2 owns multipole node b = by P + bx.
template <int P>
__global__ __launch_bounds__(kFmmThreads) void fmm_p2m(int64_t nn, const int *__restrict__ leaf_box,
                                                       const int *__restrict__ leaf_start,
                                                       const double *__restrict__ ctr, const double *__restrict__ hb,
                                                       const double *__restrict__ tm, const double *__restrict__ srt,
                                                       double *__restrict__ Q) {
  constexpr int kChunk = 64;
  __shared__ double stm[P * P];
  __shared__ double sx[kChunk][P], sy[kChunk][P];
  __shared__ double sq[3][kChunk];
  const int leaf = blockIdx.x, box = leaf_box[leaf], tid = threadIdx.x;
  for (int e = tid; e < P * P; e += blockDim.x) stm[e] = tm[e];
  const double cx = ctr[2 * box], cy = ctr[2 * box + 1], ih = 1.0 / hb[box];
  const int s0 = leaf_start[leaf], s1 = leaf_start[leaf + 1];
  const int bx = tid % P, by = tid / P;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  __syncthreads();
  for (int j0 = s0; j0 < s1; j0 += kChunk) {
    const int n = min(kChunk, s1 - j0);
    if (tid < 2 * kChunk) {
      const int j = tid >> 1, d = tid & 1;
      if (j < n) {
        double s[P];
        const double t = d ? (srt[nn + j0 + j] - cy) * ih : (srt[j0 + j] - cx) * ih;
        cheb_interp<P>(stm, t, s);
#pragma unroll
        for (int k = 0; k < P; ++k) (d ? sy : sx)[j][k] = s[k];
      }
    } else if (tid < 3 * kChunk) {
      const int j = tid - 2 * kChunk;
      if (j < n) {
        sq[0][j] = srt[2 * nn + j0 + j];
        sq[1][j] = srt[3 * nn + j0 + j];
        sq[2][j] = srt[4 * nn + j0 + j];
      }
    }
    __syncthreads();
    if (tid < P * P)
      for (int j = 0; j < n; ++j) {
        const double w = sx[j][bx] * sy[j][by];
        q0 = fma(w, sq[0][j], q0);
        q1 = fma(w, sq[1][j], q1);
        q2 = fma(w, sq[2][j], q2);
      }
    __syncthreads();
  }
  if (tid < P * P) {
    double *o = Q + (int64_t)box * 3 * P * P;
    o[tid] = q0;
    o[P * P + tid] = q1;
    o[2 * P * P + tid] = q2;
  }
}

// Parent multipole from its (up to four) children, boxes [b0, b0 + grid);
// leaves of the level (no children) keep the multipole of their sources.
// m2[(q P + K) P + m] = S_K((t_m + 2q - 1) / 2): child node m of the lower
// (q = 0) or upper (q = 1) half in the parent's coordinate.
template <int P>
__global__ __launch_bounds__(kFmmThreads) void fmm_m2m(int b0, const int *__restrict__ child,
                                                       const double *__restrict__ m2, double *__restrict__ Q) {
  __shared__ double sm[2 * P * P];
  __shared__ double qc[3][P * P];
  __shared__ double tt[3][P * P];
  const int box = b0 + blockIdx.x, tid = threadIdx.x;
  if (child[4 * box] < 0 && child[4 * box + 1] < 0 && child[4 * box + 2] < 0 && child[4 * box + 3] < 0)
    return;   // a leaf (uniform over the workgroup)
  for (int e = tid; e < 2 * P * P; e += blockDim.x) sm[e] = m2[e];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int c = child[4 * box + q];
    if (c < 0) continue;   // uniform over the workgroup
    const int qx = q & 1, qy = q >> 1;
    __syncthreads();
    for (int e = tid; e < 3 * P * P; e += blockDim.x) qc[e / (P * P)][e % (P * P)] = Q[(int64_t)c * 3 * P * P + e];
    __syncthreads();
    if (tid < P * P) {
      // tt[.][Ax P + by] = sum_bx M[qx][Ax][bx] qc[.][by P + bx]
      const int Ax = tid / P, by = tid % P;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int bx = 0; bx < P; ++bx) {
        const double mm = sm[(qx * P + Ax) * P + bx];
        s0 = fma(mm, qc[0][by * P + bx], s0);
        s1 = fma(mm, qc[1][by * P + bx], s1);
        s2 = fma(mm, qc[2][by * P + bx], s2);
      }
      tt[0][tid] = s0;
      tt[1][tid] = s1;
      tt[2][tid] = s2;
    }
    __syncthreads();
    if (tid < P * P) {
      const int Ax = tid % P, Ay = tid / P;
#pragma unroll
      for (int by = 0; by < P; ++by) {
        const double mm = sm[(qy * P + Ay) * P + by];
        acc[0] = fma(mm, tt[0][Ax * P + by], acc[0]);
        acc[1] = fma(mm, tt[1][Ax * P + by], acc[1]);
        acc[2] = fma(mm, tt[2][Ax * P + by], acc[2]);
      }
    }
  }
  if (tid < P * P) {
    double *o = Q + (int64_t)box * 3 * P * P;
    o[tid] = acc[0];
    o[P * P + tid] = acc[1];
    o[2 * P * P + tid] = acc[2];
  }
}

// Local expansions of the boxes [b0, b0 + grid) from their interaction
// lists (written, not added: the parent's share is added by fmm_l2l).
template <int P>
__global__ __launch_bounds__(kFmmThreads) void fmm_m2l(int b0, const int *__restrict__ vl_off,
                                                       const int *__restrict__ vl, const double *__restrict__ ctr,
                                                       const double *__restrict__ hb, const double *__restrict__ tn,
                                                       const double *__restrict__ Q, double *__restrict__ Lc) {
  __shared__ double ys[2][P * P];
  __shared__ double yq[3][P * P];
  const int box = b0 + blockIdx.x, tid = threadIdx.x;
  const double h = hb[box];
  double xi = 0.0, yi = 0.0;
  if (tid < P * P) {
    xi = fma(h, tn[tid % P], ctr[2 * box]);
    yi = fma(h, tn[tid / P], ctr[2 * box + 1]);
  }
  double ax = 0.0, ay = 0.0;
  for (int v = vl_off[box]; v < vl_off[box + 1]; ++v) {
    const int y = vl[v];
    __syncthreads();
    if (tid < P * P) {
      const double hy = hb[y];
      ys[0][tid] = fma(hy, tn[tid % P], ctr[2 * y]);
      ys[1][tid] = fma(hy, tn[tid / P], ctr[2 * y + 1]);
      const double *q = Q + (int64_t)y * 3 * P * P;
      yq[0][tid] = q[tid];
      yq[1][tid] = q[P * P + tid];
      yq[2][tid] = q[2 * P * P + tid];
    }
    __syncthreads();
    if (tid < P * P)
      for (int b = 0; b < P * P; ++b) dl_pair(xi, yi, ys[0][b], ys[1][b], yq[0][b], yq[1][b], yq[2][b], ax, ay);
  }
  if (tid < P * P) {
    double *o = Lc + (int64_t)box * 2 * P * P;
    o[tid] = ax;
    o[P * P + tid] = ay;
  }
}

// Local expansions of the boxes xbox[0..grid) += the direct sum of the
// sources of their X lists (leaves larger than the box, adjacent to its
// parent but well separated from the box itself).
template <int P>
__global__ __launch_bounds__(kFmmThreads) void fmm_p2l(int64_t nn, const int *__restrict__ xbox,
                                                       const int *__restrict__ xl_off, const int *__restrict__ xl,
                                                       const int *__restrict__ leaf_start,
                                                       const double *__restrict__ ctr, const double *__restrict__ hb,
                                                       const double *__restrict__ tn, const double *__restrict__ srt,
                                                       double *__restrict__ Lc) {
  __shared__ double ss[5][kFmmThreads];
  const int box = xbox[blockIdx.x], tid = threadIdx.x;
  const double h = hb[box];
  double xi = 0.0, yi = 0.0;
  if (tid < P * P) {
    xi = fma(h, tn[tid % P], ctr[2 * box]);
    yi = fma(h, tn[tid / P], ctr[2 * box + 1]);
  }
  double ax = 0.0, ay = 0.0;
  for (int v = xl_off[blockIdx.x]; v < xl_off[blockIdx.x + 1]; ++v) {
    const int c = xl[v];
    const int s0 = leaf_start[c], s1 = leaf_start[c + 1];
    for (int j0 = s0; j0 < s1; j0 += kFmmThreads) {
      const int n = min(kFmmThreads, s1 - j0);
      __syncthreads();
      if (tid < n)
#pragma unroll
        for (int q = 0; q < 5; ++q) ss[q][tid] = srt[q * nn + j0 + tid];
      __syncthreads();
      if (tid < P * P)
        for (int j = 0; j < n; ++j) dl_pair(xi, yi, ss[0][j], ss[1][j], ss[2][j], ss[3][j], ss[4][j], ax, ay);
    }
  }
  if (tid < P * P) {
    double *o = Lc + (int64_t)box * 2 * P * P;
    o[tid] += ax;
    o[P * P + tid] += ay;
  }
}

// Children's locals += the parent's local interpolated to their grids,
// boxes [b0, b0 + grid) of one level.
template <int P>
__global__ __launch_bounds__(kFmmThreads) void fmm_l2l(int b0, const int *__restrict__ par,
                                                       const int *__restrict__ quad, const double *__restrict__ m2,
                                                       double *__restrict__ Lc) {
  __shared__ double sm[2 * P * P];
  __shared__ double lp[2][P * P];
  __shared__ double tt[2][P * P];
  const int box = b0 + blockIdx.x, tid = threadIdx.x;
  const int pb = par[box], q = quad[box], qx = q & 1, qy = q >> 1;
  for (int e = tid; e < 2 * P * P; e += blockDim.x) {
    sm[e] = m2[e];
    lp[e / (P * P)][e % (P * P)] = Lc[(int64_t)pb * 2 * P * P + e];
  }
  __syncthreads();
  if (tid < P * P) {
    // tt[.][ax P + Ay] = sum_Ax M[qx][Ax][ax] lp[.][Ay P + Ax]
    const int ax = tid / P, Ay = tid % P;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int Ax = 0; Ax < P; ++Ax) {
      const double mm = sm[(qx * P + Ax) * P + ax];
      s0 = fma(mm, lp[0][Ay * P + Ax], s0);
      s1 = fma(mm, lp[1][Ay * P + Ax], s1);
    }
    tt[0][tid] = s0;
    tt[1][tid] = s1;
  }
  __syncthreads();
  if (tid < P * P) {
    const int ax = tid % P, ay = tid / P;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int Ay = 0; Ay < P; ++Ay) {
      const double mm = sm[(qy * P + Ay) * P + ay];
      s0 = fma(mm, tt[0][ax * P + Ay], s0);
      s1 = fma(mm, tt[1][ax * P + Ay], s1);
    }
    double *o = Lc + (int64_t)box * 2 * P * P;
    o[tid] += s0;
    o[P * P + tid] += s1;
  }
}

// One workgroup (one wave) per leaf: for each target of the leaf the local
// expansion (leaves at level 2 or below), the direct sum over the touching
// leaves (U list) and the multipoles of the W list (boxes smaller than the
// leaf, well separated from it, whose parents touch it), written to part in
// node order.  Boxes >= far0 carry local expansions.
template <int P>
__global__ __launch_bounds__(kLeafThreads) void fmm_leaf(int64_t nn, const int *__restrict__ leaf_box, int far0,
                                                         const int *__restrict__ leaf_start,
                                                         const int *__restrict__ ul_off, const int *__restrict__ ul,
                                                         const int *__restrict__ wl_off, const int *__restrict__ wl,
                                                         const int *__restrict__ perm, const double *__restrict__ ctr,
                                                         const double *__restrict__ hb, const double *__restrict__ tm,
                                                         const double *__restrict__ tn, const double *__restrict__ srt,
                                                         const double *__restrict__ Q, const double *__restrict__ Lc,
                                                         double *__restrict__ part) {
  __shared__ double stm[P * P];
  __shared__ double sl[2][P * P];
  __shared__ double ss[5][kLeafThreads];
  const int leaf = blockIdx.x, box = leaf_box[leaf], tid = threadIdx.x;
  const bool far = box >= far0;
  if (far)
    for (int e = tid; e < P * P; e += blockDim.x) {
      stm[e] = tm[e];
      sl[0][e] = Lc[(int64_t)box * 2 * P * P + e];
      sl[1][e] = Lc[(int64_t)box * 2 * P * P + P * P + e];
    }
  const double cx = ctr[2 * box], cy = ctr[2 * box + 1], ih = 1.0 / hb[box];
  const int t0 = leaf_start[leaf], t1 = leaf_start[leaf + 1];
  __syncthreads();
  for (int k0 = t0; k0 < t1; k0 += kLeafThreads) {
    const int k = k0 + tid;
    const bool active = k < t1;
    const double xi = active ? srt[k] : 0.0, yi = active ? srt[nn + k] : 0.0;
    double ax = 0.0, ay = 0.0;
    if (far && active) {
      double sxv[P], syv[P];
      cheb_interp<P>(stm, (xi - cx) * ih, sxv);
      cheb_interp<P>(stm, (yi - cy) * ih, syv);
#pragma unroll
      for (int a2 = 0; a2 < P; ++a2) {
        double rx = 0.0, ry = 0.0;
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) {
          rx = fma(sxv[a1], sl[0][a2 * P + a1], rx);
          ry = fma(sxv[a1], sl[1][a2 * P + a1], ry);
        }
        ax = fma(syv[a2], rx, ax);
        ay = fma(syv[a2], ry, ay);
      }
    }
    for (int u = ul_off[leaf]; u < ul_off[leaf + 1]; ++u) {
      const int nb = ul[u];
      const int s0 = leaf_start[nb], s1 = leaf_start[nb + 1];
      for (int j0 = s0; j0 < s1; j0 += kLeafThreads) {
        const int n = min(kLeafThreads, s1 - j0);
        __syncthreads();
        if (tid < n)
#pragma unroll
          for (int c = 0; c < 5; ++c) ss[c][tid] = srt[c * nn + j0 + tid];
        __syncthreads();
        if (active)
          for (int j = 0; j < n; ++j) dl_pair(xi, yi, ss[0][j], ss[1][j], ss[2][j], ss[3][j], ss[4][j], ax, ay);
      }
    }
    for (int u = wl_off[leaf]; u < wl_off[leaf + 1]; ++u) {
      const int wb = wl[u];
      const double wx = ctr[2 * wb], wy = ctr[2 * wb + 1], wh = hb[wb];
      const double *q = Q + (int64_t)wb * 3 * P * P;
      for (int b0 = 0; b0 < P * P; b0 += kLeafThreads) {
        const int n = min(kLeafThreads, P * P - b0);
        __syncthreads();
        if (tid < n) {
          const int b = b0 + tid;
          ss[0][tid] = fma(wh, tn[b % P], wx);
          ss[1][tid] = fma(wh, tn[b / P], wy);
          ss[2][tid] = q[b];
          ss[3][tid] = q[P * P + b];
          ss[4][tid] = q[2 * P * P + b];
        }
        __syncthreads();
        if (active)
          for (int j = 0; j < n; ++j) dl_pair(xi, yi, ss[0][j], ss[1][j], ss[2][j], ss[3][j], ss[4][j], ax, ay);
      }
    }
    if (active) {
      const int i = perm[k];
      part[i] = ax;
      part[nn + i] = ay;
    }
  }
}

template <class T>
DevBuf<T> upload(const std::vector<T> &h, hipStream_t s) {
  DevBuf<T> d(std::max<size_t>(h.size(), 1));
  if (!h.empty()) SBIE_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

}  // namespace

struct FmmPlan : PairSum {
  sbie_geom g{};
  int p = 0, depth = 0, nleaf = 0, nbox = 0, min_leaf_level = 0;
  bool adaptive = false;
  int64_t nn = 0;
  std::vector<int> lev_off;   // boxes of level l: [lev_off[l], lev_off[l + 1])
  int nxbox = 0;              // boxes with a non-empty X list
  DevBuf<int> perm, leaf_box, leaf_start, par, quad, child, vl_off, vl, ul_off, ul, wl_off, wl, xbox, xl_off, xl;
  DevBuf<double> ctr, hb, tm, tn, m2, Q, Lc, srt;
  int64_t m2l_pairs = 0;      // box pairs in the interaction (V) lists
  int64_t m2p_pairs = 0;      // (leaf, box) pairs in the W lists
  int64_t p2l_pairs = 0;      // (box, leaf) pairs in the X lists
  int64_t p2p_pairs = 0;      // node pairs in the near field (U lists)

  template <int P>
  void run_p(const double *src, double *part, hipStream_t s) const {
    fmm_gather<<<ceil_div(nn, 256), 256, 0, s>>>(nn, perm.p, src, srt.p);
    SBIE_LAUNCH_CHECK();
    const bool far = depth >= 2;
    if (far) {
      fmm_p2m<P><<<nleaf, kFmmThreads, 0, s>>>(nn, leaf_box.p, leaf_start.p, ctr.p, hb.p, tm.p, srt.p, Q.p);
      SBIE_LAUNCH_CHECK();
      for (int l = depth - 1; l >= 2; --l) {
        const int nb = lev_off[l + 1] - lev_off[l];
        if (nb == 0) continue;
        fmm_m2m<P><<<nb, kFmmThreads, 0, s>>>(lev_off[l], child.p, m2.p, Q.p);
        SBIE_LAUNCH_CHECK();
      }
      const int nfar = lev_off[depth + 1] - lev_off[2];
      fmm_m2l<P><<<nfar, kFmmThreads, 0, s>>>(lev_off[2], vl_off.p, vl.p, ctr.p, hb.p, tn.p, Q.p, Lc.p);
      SBIE_LAUNCH_CHECK();
      if (nxbox > 0) {
        fmm_p2l<P><<<nxbox, kFmmThreads, 0, s>>>(nn, xbox.p, xl_off.p, xl.p, leaf_start.p, ctr.p, hb.p, tn.p, srt.p,
                                                 Lc.p);
        SBIE_LAUNCH_CHECK();
      }
      for (int l = 3; l <= depth; ++l) {
        const int nb = lev_off[l + 1] - lev_off[l];
        if (nb == 0) continue;
        fmm_l2l<P><<<nb, kFmmThreads, 0, s>>>(lev_off[l], par.p, quad.p, m2.p, Lc.p);
        SBIE_LAUNCH_CHECK();
      }
    }
    fmm_leaf<P><<<nleaf, kLeafThreads, 0, s>>>(nn, leaf_box.p, far ? lev_off[2] : nbox, leaf_start.p, ul_off.p, ul.p,
                                               wl_off.p, wl.p, perm.p, ctr.p, hb.p, tm.p, tn.p, srt.p, Q.p, Lc.p,
                                               part);
    SBIE_LAUNCH_CHECK();
  }

  void run(const double *src, double *part, hipStream_t s) const override {
    switch (p) {
      case 4: run_p<4>(src, part, s); break;
      case 6: run_p<6>(src, part, s); break;
      case 8: run_p<8>(src, part, s); break;
      case 10: run_p<10>(src, part, s); break;
      case 12: run_p<12>(src, part, s); break;
      case 14: run_p<14>(src, part, s); break;
      case 16: run_p<16>(src, part, s); break;
      default: fail(SBIE_INVALID_ARGUMENT, "cheb_n must be 4, 6, ..., 16");
    }
  }

  void build(const sbie_geom *geom, const fmm_params *prm, hipStream_t s);
};

void FmmPlan::build(const sbie_geom *geom, const fmm_params *prm, hipStream_t s) {
  g = *geom;
  nn = g.n_nodes;
  p = prm->cheb_n;
  adaptive = prm->adaptive != 0;
  const int target = prm->leaf_target > 0 ? prm->leaf_target : 64;
  // host copy of the node positions
  std::vector<double> hx(nn), hy(nn);
  SBIE_HIP(hipMemcpyAsync(hx.data(), g.x, nn * sizeof(double), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipMemcpyAsync(hy.data(), g.y, nn * sizeof(double), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  FmmTree t = build_fmm_tree(hx.data(), hy.data(), nn, target, prm->max_depth, adaptive);
  depth = t.depth;
  nleaf = t.nleaf;
  nbox = t.nbox;
  nxbox = t.nxbox;
  min_leaf_level = t.min_leaf_level;
  lev_off = t.lev_off;
  m2l_pairs = t.m2l_pairs;
  p2p_pairs = t.p2p_pairs;
  m2p_pairs = t.m2p_pairs;
  p2l_pairs = t.p2l_pairs;
  // Chebyshev tables
  std::vector<double> htn(p), htm((size_t)p * p), hm2(2 * (size_t)p * p);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < p; ++k) {
    htn[k] = (double)std::cos((2.0L * k + 1.0L) * pi / (2.0L * p));
    for (int m = 0; m < p; ++m) htm[(size_t)k * p + m] = (double)std::cos((long double)m * (2.0L * k + 1.0L) * pi / (2.0L * p));
  }
  for (int q = 0; q < 2; ++q)
    for (int K = 0; K < p; ++K)
      for (int m = 0; m < p; ++m) {
        const long double tk = std::cos((2.0L * K + 1.0L) * pi / (2.0L * p));
        const long double tmv = std::cos((2.0L * m + 1.0L) * pi / (2.0L * p));
        const long double sv = 0.5L * (tmv + 2.0L * q - 1.0L);
        // S_K(sv) with T_j(x) = cos(j acos x), |x| <= 1
        long double acc = 0.0L;
        for (int j = 1; j < p; ++j) acc += std::cos(j * std::acos(tk)) * std::cos(j * std::acos(sv));
        hm2[((size_t)q * p + K) * p + m] = (double)((1.0L + 2.0L * acc) / p);
      }
  perm = upload(t.order, s);
  leaf_box = upload(t.leaf_box, s);
  leaf_start = upload(t.leaf_start, s);
  par = upload(t.par, s);
  quad = upload(t.quad, s);
  child = upload(t.child, s);
  vl_off = upload(t.vl_off, s);
  vl = upload(t.vl, s);
  ul_off = upload(t.ul_off, s);
  ul = upload(t.ul, s);
  wl_off = upload(t.wl_off, s);
  wl = upload(t.wl, s);
  xbox = upload(t.xbox, s);
  xl_off = upload(t.xl_off, s);
  xl = upload(t.xl, s);
  ctr = upload(t.ctr, s);
  hb = upload(t.hb, s);
  tn = upload(htn, s);
  tm = upload(htm, s);
  m2 = upload(hm2, s);
  Q.alloc(std::max<size_t>(1, (size_t)nbox * 3 * p * p));
  Lc.alloc(std::max<size_t>(1, (size_t)nbox * 2 * p * p));
  srt.alloc(5 * (size_t)nn);
  SBIE_HIP(hipStreamSynchronize(s));
}

}  // namespace sbie

struct sbie_fmm {
  sbie::FmmPlan plan;
};

namespace sbie {
const PairSum *fmm_pair_sum(const sbie_fmm *f) { return &f->plan; }
bool fmm_same_geometry(const sbie_fmm *f, const sbie_geom *g) {
  const sbie_geom &a = f->plan.g;
  return a.n_nodes == g->n_nodes && a.n_pores == g->n_pores && a.x == g->x && a.y == g->y && a.nx == g->nx &&
         a.ny == g->ny && a.w == g->w;
}
}  // namespace sbie

extern "C" int fmm_plan(const sbie_geom *g, const fmm_params *p, sbie_fmm **out, void *stream) {
  return sbie::guarded([&]() {
    if (!out || !p) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    *out = nullptr;
    sbie::validate_geom(g);
    if (p->adaptive != 0 && p->adaptive != 1) sbie::fail(SBIE_INVALID_ARGUMENT, "fmm_params.adaptive must be 0 or 1");
    if (p->cheb_n < 4 || p->cheb_n > 16 || (p->cheb_n & 1))
      sbie::fail(SBIE_INVALID_ARGUMENT, "cheb_n must be 4, 6, ..., 16 (got %d)", p->cheb_n);
    if (p->max_depth < 0 || p->max_depth > sbie::kFmmMaxDepth)
      sbie::fail(SBIE_INVALID_ARGUMENT, "max_depth must be in [0, %d]", sbie::kFmmMaxDepth);
    if (p->leaf_target < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "leaf_target must be >= 0");
    if (g->n_nodes >= ((int64_t)1 << 31)) sbie::fail(SBIE_UNSUPPORTED, "too many nodes");
    auto h = std::make_unique<sbie_fmm>();
    h->plan.build(g, p, (hipStream_t)stream);
    *out = h.release();
    return SBIE_OK;
  });
}

extern "C" int stokes_dlp_matvec_fmm(const sbie_fmm *f, const double *x, double *y, int mode, void *stream) {
  return sbie::guarded([&]() {
    if (!f) sbie::fail(SBIE_INVALID_ARGUMENT, "null plan");
    if (!x || !y) sbie::fail(SBIE_INVALID_ARGUMENT, "null vector");
    if (mode != SBIE_MV_FULL && mode != SBIE_MV_DLP_ONLY)
      sbie::fail(mode == SBIE_MV_FULL_ACCURATE ? SBIE_UNSUPPORTED : SBIE_INVALID_ARGUMENT,
                 "fast multipole matvec modes: SBIE_MV_FULL or SBIE_MV_DLP_ONLY (got %d)", mode);
    const sbie_geom *g = &f->plan.g;
    const int64_t n = sbie::n_unknowns(g);
    if (x < y + n && y < x + n) sbie::fail(SBIE_INVALID_ARGUMENT, "x and y overlap");
    hipStream_t s = (hipStream_t)stream;
    sbie::MatvecWork w = sbie::plan_matvec(g, false);
    w.chunks = 1;
    sbie::StreamBuf<double> scratch(sbie::matvec_scratch_doubles(w, g), s);
    sbie::bind_matvec_scratch(w, g, scratch.p);
    sbie::matvec_run(g, x, y, mode, w, s, &f->plan);
    return SBIE_OK;
  });
}

extern "C" int fmm_get_stats(const sbie_fmm *f, fmm_stats *st) {
  return sbie::guarded([&]() {
    if (!f || !st) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    st->depth = f->plan.depth;
    st->leaves = f->plan.nleaf;
    st->boxes = f->plan.nbox;
    st->min_leaf_level = f->plan.min_leaf_level;
    st->m2l_box_pairs = f->plan.m2l_pairs;
    st->near_node_pairs = f->plan.p2p_pairs;
    st->m2p_box_pairs = f->plan.m2p_pairs;
    st->p2l_box_pairs = f->plan.p2l_pairs;
    return SBIE_OK;
  });
}

extern "C" int fmm_destroy(sbie_fmm *f) {
  return sbie::guarded([&]() {
    delete f;
    return SBIE_OK;
  });
}

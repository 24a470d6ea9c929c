// Device-side checks that a geometry describes what the operator assumes
// (Section 2: a closed outer wall enclosing disjoint circular pores, each
// curve discretised by distinct trapezoid nodes, Section 2.2).
//
// Four small kernels set bits of one status word:
//   node_checks   every node: finite data, positive weight, unit normal;
//                 pore nodes on their circle
//   dup_checks    no node repeated on its own curve (distinct curves cannot
//                 share a node once the pores are disjoint circles strictly
//                 inside the wall); node i against one 256-node slice of the
//                 later nodes of its curve per thread
//   pore_pairs    every pair of pores: the discs do not touch
//   pore_in_wall  every pore: its centre inside the wall polygon (crossing
//                 count of a ray in +x) and every wall node outside its disc
// The word is read back once; a non-zero word becomes SBIE_INVALID_GEOMETRY
// with the reasons in the message.
#include <algorithm>
#include <cmath>
#include <string>

#include "common.hpp"

namespace sbie {

namespace {

enum : unsigned {
  kBadNodeData = 1u << 0,     // non-finite node data
  kBadNormal = 1u << 1,       // weight <= 0 or |n| != 1
  kOffCircle = 1u << 2,       // pore node not at distance r_k from c_k
  kDuplicate = 1u << 3,       // two nodes of a curve coincide
  kOverlap = 1u << 4,         // two pores touch or overlap
  kOutsideWall = 1u << 5,     // pore centre outside the wall or disc reaches a wall node
  kBadPoreData = 1u << 6,     // non-finite centre or non-positive radius
};

__device__ __forceinline__ int curve_of(const int64_t *__restrict__ off, int ncurves, int64_t i) {
  int lo = 0, hi = ncurves - 1;   // largest k with off[k] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void node_checks(int64_t nn, int m, const int64_t *__restrict__ off,
                            const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ nx, const double *__restrict__ ny,
                            const double *__restrict__ w, const double *__restrict__ kappa,
                            const double *__restrict__ cx, const double *__restrict__ cy,
                            const double *__restrict__ rad, unsigned *flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  unsigned f = 0;
  const double xi = x[i], yi = y[i];
  if (!isfinite(xi) || !isfinite(yi) || !isfinite(nx[i]) || !isfinite(ny[i]) || !isfinite(w[i]) ||
      !isfinite(kappa[i]))
    f |= kBadNodeData;
  const double n2 = nx[i] * nx[i] + ny[i] * ny[i];
  if (!(w[i] > 0.0) || !(fabs(n2 - 1.0) <= 1e-8)) f |= kBadNormal;
  const int k = curve_of(off, m + 1, i);
  if (k < m) {
    const double dx = xi - cx[k], dy = yi - cy[k], r = rad[k];
    if (!(fabs(dx * dx + dy * dy - r * r) <= 1e-8 * r * r)) f |= kOffCircle;
  }
  if (f) atomicOr(flags, f);
}

constexpr int kDupSlice = 256;

__global__ void dup_checks(int64_t nn, int m, const int64_t *__restrict__ off, const double *__restrict__ x,
                           const double *__restrict__ y, unsigned *flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int k = curve_of(off, m + 1, i);
  const int64_t lo = off[k] + (int64_t)blockIdx.y * kDupSlice, hi = min(off[k + 1], lo + kDupSlice);
  const double xi = x[i], yi = y[i];
  for (int64_t j = max(i + 1, lo); j < hi; ++j)
    if (x[j] == xi && y[j] == yi) {
      atomicOr(flags, kDuplicate);
      return;
    }
}

__global__ void pore_pairs(int m, const double *__restrict__ cx, const double *__restrict__ cy,
                           const double *__restrict__ rad, unsigned *flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)m * m) return;
  const int k = (int)(t / m), l = (int)(t % m);
  unsigned f = 0;
  if (k == l) {
    if (!isfinite(cx[k]) || !isfinite(cy[k]) || !(rad[k] > 0.0) || !isfinite(rad[k])) f |= kBadPoreData;
  } else if (l > k) {
    const double dx = cx[k] - cx[l], dy = cy[k] - cy[l], s = rad[k] + rad[l];
    if (!(dx * dx + dy * dy > s * s)) f |= kOverlap;
  }
  if (f) atomicOr(flags, f);
}

// One workgroup per pore.
__global__ void pore_in_wall(int m, int64_t w0, int64_t w1, const double *__restrict__ x,
                             const double *__restrict__ y, const double *__restrict__ cx,
                             const double *__restrict__ cy, const double *__restrict__ rad,
                             unsigned *flags) {
  __shared__ int cross[256];
  __shared__ int near[256];
  const int k = blockIdx.x;
  const double px = cx[k], py = cy[k], r2 = rad[k] * rad[k];
  int c = 0, nr = 0;
  const int64_t nw = w1 - w0;
  for (int64_t s = threadIdx.x; s < nw; s += blockDim.x) {
    const int64_t a = w0 + s, b = w0 + (s + 1 == nw ? 0 : s + 1);
    const double dx = x[a] - px, dy = y[a] - py;
    if (!(dx * dx + dy * dy > r2)) nr = 1;
    // does segment a-b cross the ray {(px + t, py), t > 0}?
    if ((y[a] > py) != (y[b] > py)) {
      const double xc = x[a] + (py - y[a]) * (x[b] - x[a]) / (y[b] - y[a]);
      if (xc > px) ++c;
    }
  }
  cross[threadIdx.x] = c;
  near[threadIdx.x] = nr;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      cross[threadIdx.x] += cross[threadIdx.x + h];
      near[threadIdx.x] |= near[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && (near[0] || (nw > 0 && (cross[0] & 1) == 0))) atomicOr(flags, kOutsideWall);
}

}  // namespace

void validate_geom_device(const sbie_geom *g, hipStream_t s) {
  validate_geom(g);
  const int64_t nn = g->n_nodes;
  const int m = g->n_pores;
  StreamBuf<unsigned> flags(1, s);
  SBIE_HIP(hipMemsetAsync(flags.p, 0, sizeof(unsigned), s));
  node_checks<<<ceil_div(nn, 256), 256, 0, s>>>(nn, m, g->curve_off_dev, g->x, g->y, g->nx, g->ny, g->w,
                                                g->kappa, g->cx, g->cy, g->radius, flags.p);
  SBIE_LAUNCH_CHECK();
  int64_t longest = 0;
  for (int k = 0; k <= m; ++k) longest = std::max<int64_t>(longest, g->curve_off[k + 1] - g->curve_off[k]);
  dup_checks<<<dim3(ceil_div(nn, 256), ceil_div(longest, kDupSlice)), 256, 0, s>>>(nn, m, g->curve_off_dev, g->x,
                                                                                 g->y, flags.p);
  SBIE_LAUNCH_CHECK();
  if (m > 0) {
    pore_pairs<<<ceil_div((int64_t)m * m, 256), 256, 0, s>>>(m, g->cx, g->cy, g->radius, flags.p);
    SBIE_LAUNCH_CHECK();
    pore_in_wall<<<m, 256, 0, s>>>(m, g->curve_off[m], g->curve_off[m + 1], g->x, g->y, g->cx, g->cy,
                                   g->radius, flags.p);
    SBIE_LAUNCH_CHECK();
  }
  unsigned h = 0;
  SBIE_HIP(hipMemcpyAsync(&h, flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  if (!h) return;
  std::string why;
  auto add = [&](unsigned bit, const char *msg) {
    if (h & bit) {
      if (!why.empty()) why += "; ";
      why += msg;
    }
  };
  add(kBadNodeData, "non-finite node data");
  add(kBadNormal, "non-positive weight or non-unit normal");
  add(kOffCircle, "a pore node is not on its circle");
  add(kDuplicate, "two nodes of a curve coincide");
  add(kOverlap, "two pores touch or overlap");
  add(kOutsideWall, "a pore is not strictly inside the wall");
  add(kBadPoreData, "non-finite pore centre or non-positive radius");
  fail(SBIE_INVALID_GEOMETRY, "invalid geometry: %s", why.c_str());
}

}  // namespace sbie

extern "C" int sbie_validate_geometry(const sbie_geom *g, void *stream) {
  return sbie::guarded([&] {
    sbie::validate_geom_device(g, reinterpret_cast<hipStream_t>(stream));
    return (int)SBIE_OK;
  });
}

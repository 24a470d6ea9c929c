// Inverse fast multipole method (Section 3) on the device.
//
// Factorisation, level by level from the leaves (Section 3.3), with every
// dense operation a batched device kernel and the host only scheduling:
//   * quadtree, neighbour and interaction lists: host bookkeeping (integers);
//   * near-field blocks S (Section 3.1): batched entry assembly;
//   * far field: Chebyshev interpolation (n x n nodes per box) of the
//     7-component kernel, reduced by a randomized range finder of the
//     interpolated kernel between interaction-list grids (the SVD reduction
//     of the black-box construction), one orthonormal basis W per box used on
//     both sides, reduced M2L couplings U_K^T K V_K;
//   * elimination of (x_i, z_i) for all boxes of one colour at once (boxes of
//     one colour are three boxes apart, so their neighbourhoods are
//     disjoint): batched Gauss-Jordan pivots, batched GEMMs for the Schur
//     complement, fill-ins between well-separated boxes and between x rows
//     and multipole / local variables compressed to tolerance eps by a
//     sketched truncated pivoted Gram-Schmidt and redirected through
//     augmented bases (Section 3.3, recompression);
//   * the remaining multipole system is the next level's H^2 matrix
//     (equation "A_H" applied recursively); the top level is inverted densely.
// Applying the preconditioner replays the eliminations on a right-hand side
// with device-resident GEMV descriptor lists prepared once per factorisation.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <string>
#include <cmath>
#include <map>
#include <memory>
#include <ctime>
#include <unordered_map>

#include "assemble.hpp"
#include "batched.hpp"
#include "precond.hpp"

namespace sbie {
namespace {

constexpr int kSketch = 48;   // Gaussian sketch width per far fill-in block
constexpr int kKernelSketch = 128;
constexpr int kPgsSketch = 192;   // sketch width of wide recompression candidates

// ---------------------------------------------------------------------------
// Device chunks recycled between the temporary arenas of one factorisation:
// hipMalloc and hipFree of hundreds of megabytes per level would stall the
// host (hipFree synchronises the device).  All work runs on one stream, so a
// chunk handed back can be reused by later launches without a wait.
// ---------------------------------------------------------------------------
struct ChunkCache {
  std::multimap<size_t, void *> idle;
  std::vector<void *> owned;
  std::map<void *, size_t> size_of;
  ChunkCache() = default;
  ChunkCache(const ChunkCache &) = delete;
  ChunkCache &operator=(const ChunkCache &) = delete;
  ~ChunkCache() {
    for (void *p : owned) (void)hipFree(p);
  }
  void *take(size_t bytes) {
    auto it = idle.lower_bound(bytes);
    if (it != idle.end()) {
      void *p = it->second;
      idle.erase(it);
      return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      fail(SBIE_OUT_OF_MEMORY, "device arena: hipMalloc of %zu bytes failed", bytes);
    }
    owned.push_back(p);
    size_of[p] = bytes;
    return p;
  }
  void give(void *p) { idle.insert({size_of[p], p}); }
};

// ---------------------------------------------------------------------------
// Device arena: bump allocation from large chunks, freed together (to the
// chunk cache when it has one)
// ---------------------------------------------------------------------------
struct Arena {
  std::vector<void *> chunks;
  std::vector<size_t> sizes;   // bytes of each chunk
  size_t chunk_bytes;
  ChunkCache *cache = nullptr;
  char *cur = nullptr;
  size_t left = 0;
  size_t total = 0;
  explicit Arena(size_t cb = (size_t)256 << 20, ChunkCache *c = nullptr) : chunk_bytes(cb), cache(c) {}
  Arena(const Arena &) = delete;
  Arena &operator=(const Arena &) = delete;
  ~Arena() { release(); }
  template <class T>
  T *get(size_t n) {
    const size_t b = ((n ? n : 1) * sizeof(T) + 255) & ~size_t(255);
    if (b > left) {
      const size_t cb = std::max(chunk_bytes, b);
      void *p = nullptr;
      if (cache) {
        p = cache->take(cb);
      } else if (hipMalloc(&p, cb) != hipSuccess) {
        (void)hipGetLastError();
        fail(SBIE_OUT_OF_MEMORY, "device arena: hipMalloc of %zu bytes failed", cb);
      }
      chunks.push_back(p);
      sizes.push_back(cb);
      cur = (char *)p;
      left = cb;
    }
    T *p = (T *)cur;
    cur += b;
    left -= b;
    total += b;
    return p;
  }
  void release() {
    for (void *c : chunks) {
      if (cache) cache->give(c);
      else (void)hipFree(c);
    }
    chunks.clear();
    sizes.clear();
    cur = nullptr;
    left = 0;
    total = 0;
  }
};

// ---------------------------------------------------------------------------
// Host quadtree
// ---------------------------------------------------------------------------
inline int64_t key_of(int64_t ix, int64_t iy) { return (ix << 32) ^ (iy & 0xffffffffLL); }

inline uint64_t morton(uint32_t ix, uint32_t iy) {
  uint64_t c = 0;
  for (int b = 0; b < 32; ++b)
    c |= (uint64_t)((ix >> b) & 1) << (2 * b) | (uint64_t)((iy >> b) & 1) << (2 * b + 1);
  return c;
}

struct HLevel {
  double h = 0.0;
  std::vector<int64_t> ix, iy;
  std::unordered_map<int64_t, int> index;
  std::vector<int> parent;
  std::vector<std::vector<int>> children, nbrs, ilist;
  std::vector<double> cx, cy;
  int size() const { return (int)ix.size(); }
};

struct HTree {
  double x0 = 0, y0 = 0, size = 0;
  int depth = 0, root = 0;
  std::vector<HLevel> lv;
  std::vector<std::vector<int64_t>> leaf_dofs;
};

// LSD radix sort of the low `bits` bits (8 per pass) of 64-bit keys.
void radix_sort(std::vector<uint64_t> &a, int bits) {
  std::vector<uint64_t> b(a.size());
  for (int sh = 0; sh < bits; sh += 8) {
    size_t cnt[257] = {0};
    for (uint64_t x : a) ++cnt[((x >> sh) & 255) + 1];
    for (int i = 0; i < 256; ++i) cnt[i + 1] += cnt[i];
    for (uint64_t x : a) b[cnt[(x >> sh) & 255]++] = x;
    a.swap(b);
  }
}

HTree build_tree(const std::vector<double> &px, const std::vector<double> &py, int64_t nn,
                 int64_t wall_start, int leaf_target, int max_depth) {
  HTree t;
  const int64_t np = (int64_t)px.size();
  double lx = 1e300, ly = 1e300, hx = -1e300, hy = -1e300;
  for (int64_t i = 0; i < np; ++i) {
    lx = std::min(lx, px[i]); hx = std::max(hx, px[i]);
    ly = std::min(ly, py[i]); hy = std::max(hy, py[i]);
  }
  (void)wall_start;
  const double ext = std::max(hx - lx, hy - ly);
  t.size = ext * (1.0 + 1e-9) + 1e-12;
  t.x0 = lx - 1e-12 * t.size;
  t.y0 = ly - 1e-12 * t.size;
  // Integer box coordinates at the finest admissible depth kTreeMax: the box
  // of a point at depth d is (ax >> (kTreeMax - d), ay >> (kTreeMax - d)),
  // exactly the floor of its coordinate over that level's side (the sides
  // are the root side over powers of two, so the quotients scale exactly).
  // Points are sorted once by the Morton code of that finest box; every
  // level's boxes are then the distinct code prefixes, already in Morton
  // order, with no hashing of points.
  constexpr int kTreeMax = 20;
  const double hmin = t.size / std::ldexp(1.0, kTreeMax);
  if (np >= ((int64_t)1 << 24)) fail(SBIE_UNSUPPORTED, "too many points for the quadtree");
  std::vector<uint32_t> ax(np), ay(np);
  std::vector<uint64_t> code(np), node_code(nn);
  for (int64_t i = 0; i < np; ++i) {
    ax[i] = (uint32_t)std::floor((px[i] - t.x0) / hmin);
    ay[i] = (uint32_t)std::floor((py[i] - t.y0) / hmin);
    code[i] = (morton(ax[i], ay[i]) << 24) | (uint64_t)i;   // 40-bit code, 24-bit index
    if (i < nn) node_code[i] = morton(ax[i], ay[i]);
  }
  radix_sort(code, 64);
  radix_sort(node_code, 40);
  int depth = 1;
  while (true) {
    const int sh = 2 * (kTreeMax - depth);
    size_t distinct = 0;
    uint64_t prev = ~0ull;
    for (uint64_t c : node_code)
      if ((c >> sh) != prev) {
        ++distinct;
        prev = c >> sh;
      }
    if ((double)nn / (double)distinct <= leaf_target || (max_depth > 0 && depth >= max_depth) ||
        depth >= kTreeMax)
      break;
    ++depth;
  }
  t.depth = depth;
  t.lv.resize(depth + 1);
  std::vector<int> leaf_box(np);
  for (int l = 0; l <= depth; ++l) {
    HLevel &L = t.lv[l];
    L.h = t.size / std::ldexp(1.0, l);
    // the level's code prefix (level 0: a single box; a shift by 64 bits
    // would be undefined)
    const int sh = 2 * (kTreeMax - l) + 24, cs = kTreeMax - l;
    uint64_t prev = ~0ull;
    for (uint64_t c : code) {
      const int64_t i = (int64_t)(c & 0xffffff);
      const uint64_t pre = sh >= 64 ? 0 : c >> sh;
      if (pre != prev) {
        prev = pre;
        const int64_t bx = ax[i] >> cs, by = ay[i] >> cs;
        L.index[key_of(bx, by)] = (int)L.ix.size();
        L.ix.push_back(bx);
        L.iy.push_back(by);
        L.cx.push_back(t.x0 + (bx + 0.5) * L.h);
        L.cy.push_back(t.y0 + (by + 0.5) * L.h);
      }
      if (l == depth) leaf_box[i] = L.size() - 1;
    }
    const int nb = L.size();
    L.nbrs.resize(nb);
    for (int b = 0; b < nb; ++b) {
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy) {
          auto it = L.index.find(key_of(L.ix[b] + dx, L.iy[b] + dy));
          if (it != L.index.end()) L.nbrs[b].push_back(it->second);
        }
      std::sort(L.nbrs[b].begin(), L.nbrs[b].end());
    }
    L.parent.assign(nb, -1);
    L.children.assign(nb, {});
    L.ilist.assign(nb, {});
  }
  for (int l = 1; l <= depth; ++l) {
    HLevel &L = t.lv[l], &P = t.lv[l - 1];
    for (int b = 0; b < L.size(); ++b) {
      const int p = P.index.at(key_of(L.ix[b] >> 1, L.iy[b] >> 1));
      L.parent[b] = p;
      P.children[p].push_back(b);
    }
    for (int b = 0; b < L.size(); ++b) {
      std::vector<int> il;
      for (int q : P.nbrs[L.parent[b]])
        for (int c : P.children[q]) {
          const int64_t dx = L.ix[c] - L.ix[b], dy = L.iy[c] - L.iy[b];
          if (std::max(std::llabs(dx), std::llabs(dy)) >= 2) il.push_back(c);
        }
      std::sort(il.begin(), il.end());
      L.ilist[b] = il;
    }
  }
  t.root = 0;
  for (int l = 0; l <= depth; ++l) {
    const HLevel &L = t.lv[l];
    bool all = true;
    for (int b = 0; b < L.size() && all; ++b) all = (int)L.nbrs[b].size() == L.size();
    if (all) t.root = l;
  }
  const HLevel &leaf = t.lv[depth];
  std::vector<std::vector<int64_t>> members(leaf.size());
  for (int64_t i = 0; i < np; ++i) members[leaf_box[i]].push_back(i);
  t.leaf_dofs.resize(leaf.size());
  for (int b = 0; b < leaf.size(); ++b) {
    auto &d = t.leaf_dofs[b];
    for (int64_t p : members[b]) if (p < nn) d.push_back(p);
    for (int64_t p : members[b]) if (p < nn) d.push_back(nn + p);
    for (int64_t p : members[b])
      if (p >= nn) {
        const int64_t k = p - nn;
        for (int c = 0; c < 3; ++c) d.push_back(2 * nn + 3 * k + c);
      }
  }
  return t;
}

// ---------------------------------------------------------------------------
// Chebyshev kernels
// ---------------------------------------------------------------------------
__device__ inline void cheb_1d(int n, double t, double *out) {
  // S_n(t, t_a) = 1/n + 2/n sum_{k=1}^{n-1} T_k(t) T_k(t_a)
  for (int a = 0; a < n; ++a) {
    const double ta = cos((2.0 * a + 1.0) * kPi / (2.0 * n));
    double s = 1.0 / n;
    double tp = 1.0, tk = t, ap = 1.0, ak = ta;
    for (int k = 1; k < n; ++k) {
      s += (2.0 / n) * tk * ak;
      const double tn = 2.0 * t * tk - tp;
      tp = tk;
      tk = tn;
      const double an = 2.0 * ta * ak - ap;
      ap = ak;
      ak = an;
    }
    out[a] = s;
  }
}

struct ChebBox {
  const int64_t *dofs;
  int m;
  double cx, cy, h;
  void *phi, *psi, *gv, *hv;  // T arrays: m x 2n^2, m x 7n^2, m, m
};

// Interpolation (target) and anterpolation (source) rows of every leaf dof.
template <class T>
__global__ __launch_bounds__(64) void cheb_leaf_kernel(const ChebBox *__restrict__ boxes,
                                                       GeomView g, int n) {
  const ChebBox bx = boxes[blockIdx.x];
  const int n2 = n * n;
  T *phi = (T *)bx.phi;
  T *psi = (T *)bx.psi;
  T *gv = (T *)bx.gv;
  T *hv = (T *)bx.hv;
  double sx[24], sy[24];
  for (int r = threadIdx.x; r < bx.m; r += blockDim.x) {
    const int64_t dof = bx.dofs[r];
    const int64_t nn = g.nn;
    double px, py;
    if (dof < 2 * nn) {
      const int64_t i = dof < nn ? dof : dof - nn;
      px = g.x[i];
      py = g.y[i];
    } else {
      const int64_t k = (dof - 2 * nn) / 3;
      px = g.cx[k];
      py = g.cy[k];
    }
    cheb_1d(n, (px - bx.cx) * (2.0 / bx.h), sx);
    cheb_1d(n, (py - bx.cy) * (2.0 / bx.h), sy);
    if (dof < 2 * nn) {
      const int64_t i = dof < nn ? dof : dof - nn;
      const int comp = dof < nn ? 0 : 1;
      const double nk[2] = {g.nx[i], g.ny[i]};
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const double s = sx[a] * sy[b];
          const int pt = a * n + b;
          phi[r + (size_t)(comp * n2 + pt) * bx.m] = (T)s;
          for (int kk = 0; kk < 2; ++kk)
            psi[r + (size_t)((2 * kk + comp) * n2 + pt) * bx.m] = (T)(s * g.w[i] * nk[kk]);
        }
      const bool wall = i >= g.wall_start;
      gv[r] = wall ? (T)nk[comp] : T(0);
      hv[r] = wall ? (T)(g.w[i] * nk[comp]) : T(0);
    } else {
      const int64_t q = dof - 2 * nn;
      const int64_t k = q / 3;
      const int comp = (int)(q - 3 * k);
      const double sc = comp < 2 ? 1.0 : g.rad[k];
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
          psi[r + (size_t)((4 + comp) * n2 + a * n + b) * bx.m] = (T)(sx[a] * sy[b] * sc);
      gv[r] = T(0);
      hv[r] = T(0);
    }
  }
}

// Parent Lagrange basis at the child's nodes, for the four child positions:
// out[q] is n^2 x n^2 (rows: child node, cols: parent node).
template <class T>
__global__ void cheb_transfer_kernel(int n, T *out) {
  const int n2 = n * n;
  const int q = blockIdx.x;  // child position: qx = q & 1, qy = q >> 1
  double sx[24], sy[24];
  for (int e = threadIdx.x; e < n2; e += blockDim.x) {
    const int a = e / n, b = e % n;
    const double ta = cos((2.0 * a + 1.0) * kPi / (2.0 * n));
    const double tb = cos((2.0 * b + 1.0) * kPi / (2.0 * n));
    const double cxp = -0.5 + (q & 1), cyp = -0.5 + (q >> 1);
    cheb_1d(n, cxp + 0.5 * ta, sx);
    cheb_1d(n, cyp + 0.5 * tb, sy);
    for (int a2 = 0; a2 < n; ++a2)
      for (int b2 = 0; b2 < n; ++b2)
        out[(size_t)q * n2 * n2 + e + (size_t)(a2 * n + b2) * n2] = (T)(sx[a2] * sy[b2]);
  }
}

// Far-field kernel between Chebyshev grids for the 40 interaction offsets:
// kfat  (2n^2) x (40 * 7n^2): block o is K_o (targets x sources)
// kthin (40 * 2n^2) x (7n^2): K_o stacked vertically
template <class T>
__global__ void far_kernel_tables(int n, double h, T *kfat, T *kthin) {
  const int n2 = n * n;
  const int o = blockIdx.y;
  int dx = 0, dy = 0, cnt = 0;
  for (int ddx = -3; ddx <= 3; ++ddx)
    for (int ddy = -3; ddy <= 3; ++ddy) {
      if (std::max(abs(ddx), abs(ddy)) < 2) continue;
      if (cnt == o) { dx = ddx; dy = ddy; }
      ++cnt;
    }
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (target pt, source pt)
  if (e >= n2 * n2) return;
  const int tp = e % n2, sp = e / n2;
  const double tx = 0.5 * h * cos((2.0 * (tp / n) + 1.0) * kPi / (2.0 * n));
  const double ty = 0.5 * h * cos((2.0 * (tp % n) + 1.0) * kPi / (2.0 * n));
  const double sx = dx * h + 0.5 * h * cos((2.0 * (sp / n) + 1.0) * kPi / (2.0 * n));
  const double sy = dy * h + 0.5 * h * cos((2.0 * (sp % n) + 1.0) * kPi / (2.0 * n));
  const double r[2] = {tx - sx, ty - sy};
  const double r2 = r[0] * r[0] + r[1] * r[1];
  const double inv4 = 1.0 / (r2 * r2);
  const double lg = 0.5 * log(r2);
  const size_t rows = 2 * n2, ld_thin = (size_t)40 * 2 * n2;
  for (int a = 0; a < 2; ++a) {
    double v[7];
    for (int kk = 0; kk < 2; ++kk)
      for (int ll = 0; ll < 2; ++ll) v[2 * kk + ll] = r[a] * r[kk] * r[ll] * inv4 / kPi;
    for (int b = 0; b < 2; ++b) v[4 + b] = (0.25 / kPi) * ((a == b ? -lg : 0.0) + r[a] * r[b] / r2);
    v[6] = (0.25 / kPi) * (a == 0 ? r[1] : -r[0]) / r2;
    const size_t row = (size_t)a * n2 + tp;
    for (int c = 0; c < 7; ++c) {
      const size_t col = (size_t)c * n2 + sp;
      kfat[row + ((size_t)o * 7 * n2 + col) * rows] = (T)v[c];
      kthin[(size_t)o * rows + row + col * ld_thin] = (T)v[c];
    }
  }
}

struct AsmDesc {
  const int64_t *rows;
  const int64_t *cols;
  int nr, nc;
  void *out;
};

template <class T>
__global__ __launch_bounds__(256) void assemble_desc_kernel(GeomView g,
                                                            const AsmDesc *__restrict__ d) {
  const AsmDesc a = d[blockIdx.x];
  const int c0 = blockIdx.y * 8;
  T *out = (T *)a.out;
  for (int c = c0; c < c0 + 8 && c < a.nc; ++c) {
    const int64_t col = a.cols[c];
    for (int r = threadIdx.x; r < a.nr; r += 256)
      out[r + (size_t)c * a.nr] = (T)op_entry(g, a.rows[r], col);
  }
}

template <class T>
__global__ void gather_rhs(const int64_t *__restrict__ dofs, int64_t n, const double *__restrict__ b,
                           T *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)b[dofs[i]];
}

template <class T>
__global__ void scatter_sol(const int64_t *__restrict__ dofs, int64_t n, const T *__restrict__ x,
                            double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[dofs[i]] = (double)x[i];
}

// ---------------------------------------------------------------------------
// Factorisation state
// ---------------------------------------------------------------------------
// Hash map from a pair of box indices to V: open addressing with linear
// probing in one flat array (power-of-two capacity, at most half full), so
// that the tens of thousands of blocks of a level cost no allocation each.
// find() returns a pointer to the (key, value) pair or end() (null);
// entries are never erased; emplace keeps an existing entry.  References
// stay valid only until the next emplace.
template <class V>
class PairMap {
 public:
  using value_type = std::pair<std::pair<int, int>, V>;
  void reserve(size_t n) {
    if (2 * n > cap_) rehash(pow2(2 * n));
  }
  value_type *find(const std::pair<int, int> &k) {
    if (cap_ == 0) return nullptr;
    for (size_t i = slot(k);; i = (i + 1) & (cap_ - 1)) {
      if (!used_[i]) return nullptr;
      if (tab_[i].first == k) return &tab_[i];
    }
  }
  value_type *end() const { return nullptr; }
  void emplace(const std::pair<int, int> &k, const V &v) {
    if (2 * (n_ + 1) > cap_) rehash(pow2(std::max<size_t>(16, 2 * cap_)));
    for (size_t i = slot(k);; i = (i + 1) & (cap_ - 1)) {
      if (!used_[i]) {
        used_[i] = 1;
        tab_[i] = value_type(k, v);
        ++n_;
        return;
      }
      if (tab_[i].first == k) return;
    }
  }

 private:
  std::vector<value_type> tab_;
  std::vector<unsigned char> used_;
  size_t cap_ = 0, n_ = 0;
  static size_t pow2(size_t n) {
    size_t c = 16;
    while (c < n) c <<= 1;
    return c;
  }
  // the 64-bit finaliser of MurmurHash3 on the packed pair
  size_t slot(const std::pair<int, int> &k) const {
    uint64_t x = ((uint64_t)(uint32_t)k.first << 32) | (uint32_t)k.second;
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (size_t)x & (cap_ - 1);
  }
  void rehash(size_t c) {
    std::vector<value_type> old;
    std::vector<unsigned char> oldu;
    old.swap(tab_);
    oldu.swap(used_);
    tab_.assign(c, value_type());
    used_.assign(c, 0);
    cap_ = c;
    n_ = 0;
    for (size_t i = 0; i < old.size(); ++i)
      if (oldu[i]) emplace(old[i].first, old[i].second);
  }
};

// Map from a box index to V for the handful of neighbours of one box:
// linear search in a small vector (operator[] inserts a value-initialised
// entry when the key is missing, like std::map).
template <class V>
class SmallMap {
 public:
  V &operator[](int k) {
    for (auto &e : v_)
      if (e.first == k) return e.second;
    v_.emplace_back(k, V{});
    return v_.back().second;
  }

 private:
  std::vector<std::pair<int, V>> v_;
};

template <class T>
struct Blk {
  T *p = nullptr;
  int ld = 0;
};

template <class M>
auto &blk(M &map, int a, int b) {
  auto it = map.find(std::make_pair(a, b));
  if (it == map.end()) fail(SBIE_HIP_ERROR, "internal: missing block (%d, %d)", a, b);
  return it->second;
}

// One colour phase of the application: a forward and a backward launch.
//   forward:  t_i = A_xx g_i;  (z-rhs of the parent) = A_zx g_i;
//             rhs_j -= N_ji g_i with N_ji = S_ji A_xx   (j active neighbour)
//   backward: x_i = t_i - sum_k M_ik x_k + A_xy y_i with M_ik = A_xx S_ik
template <class T, class TA = T>
struct SolvePhase {
  GemvDesc<T> *f = nullptr;
  GemvTerm<T, TA> *ft = nullptr;
  int nf = 0;
  GemvDesc<T> *b = nullptr;
  GemvTerm<T, TA> *bt = nullptr;
  int nb = 0;
};

}  // namespace

// Stage timers of the factorisation, printed when SBIE_VERBOSE is set (each
// stage boundary then synchronises the stream, so timings are exclusive).
struct StageClock {
  bool on = false;
  hipStream_t s = nullptr;
  std::chrono::steady_clock::time_point last;
  std::map<std::string, double> acc, host;   // wall time; time until the stage's last enqueue
  // host time blocked in the stage's own synchronisations; a read-back into
  // pageable memory already blocks inside the copy, so this is a lower bound
  // of the time the host waited for the device
  std::map<std::string, double> waits;
  std::map<std::string, double> cpu;         // CPU time of the calling thread
  double wait_now = 0.0, cpu_last = 0.0;
  static double thread_cpu() {
    timespec ts;
    clock_gettime(CLOCK_THREAD_CPUTIME_ID, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
  }
  // a read-back inside a stage: synchronise, counting the time blocked
  void sync(hipStream_t st) {
    if (!on) {
      SBIE_HIP(hipStreamSynchronize(st));
      return;
    }
    const auto t0 = std::chrono::steady_clock::now();
    SBIE_HIP(hipStreamSynchronize(st));
    wait_now += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  explicit StageClock(hipStream_t st) : on(std::getenv("SBIE_VERBOSE") != nullptr), s(st) {
    last = std::chrono::steady_clock::now();
    cpu_last = thread_cpu();
  }
  void tick(const char *name, int level = -1) {
    if (!on) return;
    if (level >= 0) {
      char buf[64];
      std::snprintf(buf, sizeof(buf), "%s_L%d", name, level);
      tick_s(buf);
      return;
    }
    tick_s(name);
  }
  void tick_s(const std::string &name) {
    const auto enq = std::chrono::steady_clock::now();
    const double c = thread_cpu();
    cpu[name] += c - cpu_last;
    (void)hipStreamSynchronize(s);
    const auto now = std::chrono::steady_clock::now();
    acc[name] += std::chrono::duration<double>(now - last).count();
    host[name] += std::chrono::duration<double>(enq - last).count();
    waits[name] += wait_now;
    wait_now = 0.0;
    last = now;
    cpu_last = thread_cpu();
  }
  ~StageClock() {
    if (!on) return;
    double tot = 0.0;
    for (auto &kv : acc) tot += kv.second;
    std::fprintf(stderr, "[ifmm] factor stages (s):");
    for (auto &kv : acc) std::fprintf(stderr, " %s=%.4f", kv.first.c_str(), kv.second);
    std::fprintf(stderr, " total=%.4f\n", tot);
    // the host part runs until the stage's last enqueue (read-backs included)
    std::fprintf(stderr, "[ifmm] host part of each stage (s):");
    for (auto &kv : host) std::fprintf(stderr, " %s=%.4f", kv.first.c_str(), kv.second);
    std::fprintf(stderr, "\n[ifmm] read-back waits inside each stage (s):");
    for (auto &kv : waits) std::fprintf(stderr, " %s=%.4f", kv.first.c_str(), kv.second);
    std::fprintf(stderr, "\n[ifmm] CPU time of the host thread until each stage's last enqueue (s):");
    for (auto &kv : cpu) std::fprintf(stderr, " %s=%.4f", kv.first.c_str(), kv.second);
    std::fprintf(stderr, "\n");
    {
      const HostProf &h = host_prof();
      const char *nm[HostProf::kSlots] = {"gemm_batched", "staging", "gemm_launch", "copy_batched",
                                          "inverse_prep", "inverse_launches", "gram_schmidt", "alloc"};
      std::fprintf(stderr, "[ifmm] host time in batched operations since process start (s, calls):");
      for (int k = 0; k < HostProf::kSlots; ++k) std::fprintf(stderr, " %s=%.4f/%lld", nm[k], h.t[k], (long long)h.n[k]);
      std::fprintf(stderr, "\n");
    }
  }
};

struct IfmmImplBase {
  virtual ~IfmmImplBase() = default;
  virtual void apply(const double *b, double *x, hipStream_t s) const = 0;
  // capture the application into a HIP graph (done by factor unless
  // defer_graph is set, in which case the caller captures later, from a
  // thread while no other thread works on the device)
  virtual void capture_graph() = 0;
  bool defer_graph = false;
  ifmm_stats stats{};
  int64_t n = 0;
};

namespace {

// The application's launch sequence: forward sweeps level by level, colour
// by colour, the root, then the backward sweeps in reverse order.
template <class T, class TA = T>
struct SolvePlan {
  std::vector<std::vector<SolvePhase<T, TA>>> phases;   // per eliminated level
  GemvDesc<T> *root_d = nullptr;
  GemvTerm<T, TA> *root_t = nullptr;
  int root_nd = 0;
  T *rhs0 = nullptr, *x0 = nullptr;                  // leaf-level rhs and solution
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  SolvePlan() = default;
  SolvePlan(const SolvePlan &) = delete;
  SolvePlan &operator=(const SolvePlan &) = delete;
  ~SolvePlan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  void run(hipStream_t s) const {
    const int nl = (int)phases.size();
    for (int l = 0; l < nl; ++l)
      for (const auto &ph : phases[l]) gemv_launch<T, TA>(ph.f, ph.ft, ph.nf, 64, s);
    gemv_launch<T, TA>(root_d, root_t, root_nd, 64, s);
    for (int l = nl - 1; l >= 0; --l)
      for (auto it = phases[l].rbegin(); it != phases[l].rend(); ++it)
        gemv_launch<T, TA>(it->b, it->bt, it->nb, 64, s);
  }
  // Capture the fixed launch sequence of one application (everything between
  // the gather of b and the scatter of x) into a HIP graph.
  void capture() {
    if (std::getenv("SBIE_NO_GRAPH")) return;
    SBIE_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    SBIE_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    run(cap_stream);
    SBIE_HIP(hipStreamEndCapture(cap_stream, &graph));
    SBIE_HIP(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
  }
  void apply(const int64_t *dofs, int64_t nd, const double *b, double *x, hipStream_t s) const {
    gather_rhs<T><<<ceil_div(nd, 256), 256, 0, s>>>(dofs, nd, b, rhs0);
    SBIE_LAUNCH_CHECK();
    if (graph_exec)
      SBIE_HIP(hipGraphLaunch(graph_exec, s));
    else
      run(s);
    scatter_sol<T><<<ceil_div(nd, 256), 256, 0, s>>>(dofs, nd, x0, x);
    SBIE_LAUNCH_CHECK();
  }
};

// Host copies of one phase's descriptors (kept when an FP32 copy of the
// application is built from an FP64 factorisation).
template <class T>
struct HostPhase {
  std::vector<GemvDesc<T>> fd, bd;
  std::vector<GemvTerm<T>> ft, bt;
};

template <class T>
struct IfmmImpl : IfmmImplBase {
  Arena persist{(size_t)512 << 20};
  DevBuf<int64_t> leaf_dofs_all;
  int64_t n_leaf_dofs = 0;
  SolvePlan<T> plan;
  std::vector<std::vector<SolvePhase<T>>> &phases = plan.phases;
  std::vector<T *> rhs, gsave, tbuf, vbuf, xbuf;     // per level index (0 = leaf)
  T *root_inv = nullptr;
  int root_dim = 0;
  // FP32 storage of an FP64 factorisation (precision 2): the matrices the
  // application reads are mirrored in FP32 at the same offsets and widened
  // to FP64 as they are read; vectors and arithmetic stay FP64.
  bool apply32 = false;
  std::vector<std::vector<HostPhase<T>>> host_phases;
  HostPhase<T> host_root;
  Arena mirror{(size_t)256 << 20};
  Arena mirror_desc{(size_t)16 << 20};
  std::vector<float *> mirror_base;
  SolvePlan<T, float> plan32;

  void build_graph() {
    if (apply32) plan32.capture();
    else plan.capture();
  }

  void capture_graph() override { build_graph(); }

  void apply(const double *b, double *x, hipStream_t s) const override {
    if (apply32) plan32.apply(leaf_dofs_all.p, n_leaf_dofs, b, x, s);
    else plan.apply(leaf_dofs_all.p, n_leaf_dofs, b, x, s);
  }

  // the FP32 address of an FP64 array held in the persistent arena
  float *to32(const T *p) const {
    const char *c = reinterpret_cast<const char *>(p);
    for (size_t i = 0; i < persist.chunks.size(); ++i) {
      const char *base = reinterpret_cast<const char *>(persist.chunks[i]);
      if (c >= base && c < base + persist.sizes[i])
        return reinterpret_cast<float *>(reinterpret_cast<char *>(mirror_base[i]) + (c - base) / 2);
    }
    fail(SBIE_INVALID_ARGUMENT, "array outside the factorisation's storage");
  }

  // Mirror the persistent arena in FP32 and translate the solve plan.
  void build_plan32(hipStream_t s) {
    for (size_t i = 0; i < persist.chunks.size(); ++i) {
      const size_t nel = persist.sizes[i] / sizeof(T);
      float *f = mirror.get<float>(nel);
      convert<T, float>(reinterpret_cast<const T *>(persist.chunks[i]), f, nel, s);
      mirror_base.push_back(f);
    }
    auto desc32 = [&](const std::vector<GemvDesc<T>> &d) { return d; };
    auto term32 = [&](const std::vector<GemvTerm<T>> &t) {
      std::vector<GemvTerm<T, float>> o;
      for (const auto &q : t) o.push_back({to32(q.A), q.x, q.lda, q.cols, q.trans, q.alpha});
      return o;
    };
    Packed pk;
    struct Offs { size_t f, ft, b, bt; int nf, nb; };
    std::vector<std::vector<Offs>> offs(host_phases.size());
    for (size_t l = 0; l < host_phases.size(); ++l)
      for (const auto &hp : host_phases[l])
        offs[l].push_back({pk.add(desc32(hp.fd)), pk.add(term32(hp.ft)), pk.add(desc32(hp.bd)),
                           pk.add(term32(hp.bt)), (int)hp.fd.size(), (int)hp.bd.size()});
    const size_t root_d = pk.add(desc32(host_root.fd)), root_t = pk.add(term32(host_root.ft));
    char *base = send(pk, mirror_desc, s);
    plan32.phases.resize(host_phases.size());
    for (size_t l = 0; l < host_phases.size(); ++l)
      for (const Offs &o : offs[l]) {
        SolvePhase<T, float> ph;
        ph.f = at<GemvDesc<T>>(base, o.f);
        ph.ft = at<GemvTerm<T, float>>(base, o.ft);
        ph.nf = o.nf;
        ph.b = at<GemvDesc<T>>(base, o.b);
        ph.bt = at<GemvTerm<T, float>>(base, o.bt);
        ph.nb = o.nb;
        plan32.phases[l].push_back(ph);
      }
    plan32.root_d = at<GemvDesc<T>>(base, root_d);
    plan32.root_t = at<GemvTerm<T, float>>(base, root_t);
    plan32.root_nd = (int)host_root.fd.size();
    plan32.rhs0 = rhs[0];
    plan32.x0 = xbuf[0];
    host_phases.clear();
    host_root = HostPhase<T>{};
    SBIE_HIP(hipStreamSynchronize(s));
  }

  template <class D>
  D *upload(const std::vector<D> &v) {
    if (v.empty()) return nullptr;
    D *p = persist.get<D>(v.size());
    SBIE_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(D), hipMemcpyHostToDevice));
    return p;
  }

  // Descriptor arrays of many solve phases packed into one host block and
  // sent with one stream-ordered copy (instead of one blocking copy each).
  // The host blocks stay alive until the factorisation's final wait.
  struct Packed {
    std::vector<char> bytes;
    template <class D>
    size_t add(const std::vector<D> &v) {
      if (v.empty()) return SIZE_MAX;
      const size_t o = (bytes.size() + 255) & ~size_t(255);
      bytes.resize(o + v.size() * sizeof(D));
      std::memcpy(bytes.data() + o, v.data(), v.size() * sizeof(D));
      return o;
    }
  };
  std::vector<std::vector<char>> sent_blocks;
  char *send(Packed &pk, Arena &a, hipStream_t s) {
    if (pk.bytes.empty()) return nullptr;
    char *p = a.get<char>(pk.bytes.size());
    sent_blocks.push_back(std::move(pk.bytes));
    const std::vector<char> &b = sent_blocks.back();
    SBIE_HIP(hipMemcpyAsync(p, b.data(), b.size(), hipMemcpyHostToDevice, s));
    return p;
  }
  template <class D>
  static D *at(char *base, size_t o) {
    return o == SIZE_MAX ? nullptr : reinterpret_cast<D *>(base + o);
  }

  // split a y-block of `rows` rows into <= 64-row GEMV descriptors
  static void add_gemv(std::vector<GemvDesc<T>> &ds, std::vector<GemvTerm<T>> &ts, T *y, int rows,
                       T beta, const std::vector<GemvTerm<T>> &terms, const T *y0 = nullptr) {
    for (int r0 = 0; r0 < rows; r0 += 64) {
      GemvDesc<T> d;
      d.y = y + r0;
      d.y0 = y0 ? y0 + r0 : nullptr;
      d.rows = std::min(64, rows - r0);
      d.t0 = (int)ts.size();
      d.beta = beta;
      for (auto t : terms) {
        if (!t.trans) t.A = t.A + r0;
        else t.A = t.A + (size_t)r0 * t.lda;
        ts.push_back(t);
      }
      d.nt = (int)ts.size() - d.t0;
      ds.push_back(d);
    }
  }

  void factor(const sbie_geom *g, const ifmm_params *prm, hipStream_t s);
};

template <class T>
void IfmmImpl<T>::factor(const sbie_geom *g, const ifmm_params *prm, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t nn = g->n_nodes;
  const int m_p = g->n_pores;
  n = n_unknowns(g);
  const double eps = prm->eps;
  const int cn = prm->cheb_n;
  // inputs of the two sketch products of the recompression (the far
  // fill-ins times a Gaussian matrix, the wide candidate sets times a
  // Gaussian matrix): the factor's precision, or FP16 / BF16 on the matrix
  // cores with FP32 accumulation
  const GemmInputs sketch_in = (GemmInputs)prm->compress;
  const int n2 = cn * cn;
  if (cn < 2 || cn > 24) fail(SBIE_INVALID_ARGUMENT, "cheb_n must be in [2, 24]");
  if (!(eps > 0.0 && eps < 1.0)) fail(SBIE_INVALID_ARGUMENT, "eps must be in (0, 1)");
  const int leaf_target = prm->leaf_target > 0 ? prm->leaf_target : 64;

  // ---- host copies of the point data and the quadtree
  std::vector<double> px(nn + m_p), py(nn + m_p), rad(m_p);
  SBIE_HIP(hipMemcpy(px.data(), g->x, nn * 8, hipMemcpyDeviceToHost));
  SBIE_HIP(hipMemcpy(py.data(), g->y, nn * 8, hipMemcpyDeviceToHost));
  if (m_p) {
    SBIE_HIP(hipMemcpy(px.data() + nn, g->cx, m_p * 8, hipMemcpyDeviceToHost));
    SBIE_HIP(hipMemcpy(py.data() + nn, g->cy, m_p * 8, hipMemcpyDeviceToHost));
    SBIE_HIP(hipMemcpy(rad.data(), g->radius, m_p * 8, hipMemcpyDeviceToHost));
  }
  StageClock clk(s);
  op_flops() = OpFlops{};
  HTree tr = build_tree(px, py, nn, g->curve_off[m_p], leaf_target, prm->max_depth);
  clk.tick("tree");
  const double leaf_h = tr.lv[tr.depth].h;
  for (int k = 0; k < m_p; ++k)
    if (rad[k] >= leaf_h)
      fail(SBIE_UNSUPPORTED, "pore %d radius %.3g exceeds the leaf box side %.3g", k, rad[k], leaf_h);

  StagerLease lease((size_t)64 << 20, s);
  Stager &st = *lease;
  ChunkCache chunk_cache;   // declared before every temporary arena: outlives them
  DevBuf<double> wl(1);
  wall_length(g, wl.p, s);
  double wall_len = 1.0;
  SBIE_HIP(hipMemcpyAsync(&wall_len, wl.p, 8, hipMemcpyDeviceToHost, s));
  clk.sync(s);
  if (!(wall_len > 0.0)) wall_len = 1.0;
  const GeomView gv = make_view(g, wl.p);
  DevBuf<int32_t> info(2 * 65536);
  DevBuf<int> counts(65536);
  DevBuf<double> norms(65536);

  // ---- leaf dofs
  const HLevel &leaf = tr.lv[tr.depth];
  const int nleaf = leaf.size();
  std::vector<int64_t> all_dofs, dof_off(nleaf + 1, 0);
  for (int b = 0; b < nleaf; ++b) {
    dof_off[b] = (int64_t)all_dofs.size();
    all_dofs.insert(all_dofs.end(), tr.leaf_dofs[b].begin(), tr.leaf_dofs[b].end());
  }
  dof_off[nleaf] = (int64_t)all_dofs.size();
  n_leaf_dofs = (int64_t)all_dofs.size();
  if (n_leaf_dofs != n) fail(SBIE_INVALID_GEOMETRY, "tree lost unknowns");
  leaf_dofs_all.alloc(n_leaf_dofs);
  SBIE_HIP(hipMemcpy(leaf_dofs_all.p, all_dofs.data(), n_leaf_dofs * 8, hipMemcpyHostToDevice));

  // ---- level-independent tables: transfer matrices for the 4 child slots
  T *transfer = persist.get<T>((size_t)4 * n2 * n2);
  cheb_transfer_kernel<T><<<4, 256, 0, s>>>(cn, transfer);
  SBIE_LAUNCH_CHECK();

  // per-level state containers
  std::vector<int> m(nleaf);
  for (int b = 0; b < nleaf; ++b) m[b] = (int)tr.leaf_dofs[b].size();
  PairMap<Blk<T>> S;  // near field of the level
  auto level_arena = std::make_unique<Arena>((size_t)256 << 20, &chunk_cache);
  // leaf near field
  {
    std::vector<AsmDesc> ad;
    int maxc = 0;
    for (int b = 0; b < nleaf; ++b)
      for (int c : leaf.nbrs[b]) {
        Blk<T> bl;
        bl.p = level_arena->get<T>((size_t)m[b] * m[c]);
        bl.ld = m[b];
        S.emplace(std::make_pair(b, c), bl);
        AsmDesc a;
        a.rows = leaf_dofs_all.p + dof_off[b];
        a.cols = leaf_dofs_all.p + dof_off[c];
        a.nr = m[b];
        a.nc = m[c];
        a.out = bl.p;
        ad.push_back(a);
        maxc = std::max(maxc, m[c]);
      }
    for (size_t b0 = 0; b0 < ad.size(); b0 += 60000) {
      const size_t nb = std::min(ad.size() - b0, size_t(60000));
      auto *dd = (const AsmDesc *)st.put(ad.data() + b0, nb * sizeof(AsmDesc), s);
      dim3 grid((unsigned)nb, ceil_div(maxc, 8));
      assemble_desc_kernel<T><<<grid, 256, 0, s>>>(gv, dd);
      SBIE_LAUNCH_CHECK();
    }
  }
  clk.tick("leaf_assemble");
  // leaf Chebyshev rows
  std::vector<T *> phi(nleaf), psi(nleaf), gvec(nleaf), hvec(nleaf);
  {
    std::vector<ChebBox> cb(nleaf);
    std::vector<CopyDesc<T>> zero;   // alpha = 0 without accumulation: a fill
    for (int b = 0; b < nleaf; ++b) {
      phi[b] = level_arena->get<T>((size_t)m[b] * 2 * n2);
      psi[b] = level_arena->get<T>((size_t)m[b] * 7 * n2);
      gvec[b] = level_arena->get<T>(m[b]);
      hvec[b] = level_arena->get<T>(m[b]);
      zero.push_back({nullptr, 1, phi[b], m[b], m[b], 2 * n2, 0, 0, T(0)});
      zero.push_back({nullptr, 1, psi[b], m[b], m[b], 7 * n2, 0, 0, T(0)});
      cb[b] = ChebBox{leaf_dofs_all.p + dof_off[b], m[b], leaf.cx[b], leaf.cy[b], leaf.h,
                      phi[b], psi[b], gvec[b], hvec[b]};
    }
    copy_batched<T>(zero, st, s);
    auto *dd = (const ChebBox *)st.put(cb.data(), cb.size() * sizeof(ChebBox), s);
    cheb_leaf_kernel<T><<<nleaf, 64, 0, s>>>(dd, gv, cn);
    SBIE_LAUNCH_CHECK();
  }

  // per-level solve buffers: index 0 = leaf level
  const int nelim = tr.depth - tr.root;
  std::vector<std::vector<int64_t>> lvl_off(nelim + 1);
  auto alloc_level_vectors = [&](int li, const std::vector<int> &dims) {
    std::vector<int64_t> &off = lvl_off[li];
    off.assign(dims.size() + 1, 0);
    for (size_t b = 0; b < dims.size(); ++b) off[b + 1] = off[b] + dims[b];
    const int64_t tot = std::max<int64_t>(1, off.back());
    rhs.push_back(persist.get<T>(tot));
    gsave.push_back(persist.get<T>(tot));
    tbuf.push_back(persist.get<T>(tot));
    vbuf.push_back(persist.get<T>(tot));
    xbuf.push_back(persist.get<T>(tot));
  };
  alloc_level_vectors(0, m);
  phases.resize(nelim);
  if (apply32) host_phases.resize(nelim);
  int max_rank = 0;

  for (int li = 0; li < nelim; ++li) {
    const int lev = tr.depth - li;
    const HLevel &L = tr.lv[lev];
    const int nb = L.size();
    Arena phase_arena((size_t)256 << 20, &chunk_cache);
    // ---- kernel bases of this level (randomized range finder of the
    //      interpolated kernel between interaction-list grids)
    T *kfat = phase_arena.get<T>((size_t)2 * n2 * 40 * 7 * n2);
    T *kthin = phase_arena.get<T>((size_t)40 * 2 * n2 * 7 * n2);
    far_kernel_tables<T><<<dim3(ceil_div(n2 * n2, 256), 40), 256, 0, s>>>(cn, L.h, kfat, kthin);
    SBIE_LAUNCH_CHECK();
    const int ps = kKernelSketch;
    T *om1 = phase_arena.get<T>((size_t)40 * 7 * n2 * ps);
    T *om2 = phase_arena.get<T>((size_t)40 * 2 * n2 * ps);
    gaussian_fill<T>(om1, (size_t)40 * 7 * n2 * ps, 1000 + lev, s);
    gaussian_fill<T>(om2, (size_t)40 * 2 * n2 * ps, 2000 + lev, s);
    T *yu = phase_arena.get<T>((size_t)2 * n2 * ps);
    T *yv = phase_arena.get<T>((size_t)7 * n2 * ps);
    gemm_batched<T>({GemmDesc<T>{2 * n2, ps, 40 * 7 * n2, 0, 0, kfat, 2 * n2, om1, 40 * 7 * n2, yu,
                                 2 * n2, T(1), T(0)},
                     GemmDesc<T>{7 * n2, ps, 40 * 2 * n2, 1, 0, kthin, 40 * 2 * n2, om2,
                                 40 * 2 * n2, yv, 7 * n2, T(1), T(0)}},
                    st, s);
    norms_batched<T>({NormDesc<T>{yu, 2 * n2, 2 * n2, ps}, NormDesc<T>{yv, 7 * n2, 7 * n2, ps}},
                     norms.p, st, s);
    double hn[2];
    SBIE_HIP(hipMemcpyAsync(hn, norms.p, 16, hipMemcpyDeviceToHost, s));
    clk.sync(s);
    const int cap_u = std::min(2 * n2, ps), cap_v = std::min(7 * n2, ps);
    T *uk = phase_arena.get<T>((size_t)2 * n2 * cap_u);
    T *vk = phase_arena.get<T>((size_t)7 * n2 * cap_v);
    // the Frobenius norm over ps Gaussian columns estimates sqrt(ps) times
    // the Frobenius norm of the kernel; truncate relative to the largest
    // column scale
    pgs_batched<T>({PgsDesc<T>{yu, 2 * n2, 2 * n2, ps, uk, 2 * n2, 0, cap_u,
                               eps * hn[0] / std::sqrt((double)ps), counts.p},
                    PgsDesc<T>{yv, 7 * n2, 7 * n2, ps, vk, 7 * n2, 0, cap_v,
                               eps * hn[1] / std::sqrt((double)ps), counts.p + 1}},
                   st, s);
    int hc[2];
    SBIE_HIP(hipMemcpyAsync(hc, counts.p, 8, hipMemcpyDeviceToHost, s));
    clk.sync(s);
    st.reset();
    const int ru = hc[0], rv = hc[1];
    // reduced M2L per offset: U_K^T K_o V_K
    T *kvt = phase_arena.get<T>((size_t)40 * 2 * n2 * rv);
    T *m2l = phase_arena.get<T>((size_t)40 * ru * rv);
    {
      std::vector<GemmDesc<T>> gd;
      for (int o = 0; o < 40; ++o)
        gd.push_back({2 * n2, rv, 7 * n2, 0, 0, kfat + (size_t)o * 7 * n2 * 2 * n2, 2 * n2, vk,
                      7 * n2, kvt + (size_t)o * 2 * n2 * rv, 2 * n2, T(1), T(0)});
      gemm_batched<T>(gd, st, s);
      gd.clear();
      for (int o = 0; o < 40; ++o)
        gd.push_back({ru, rv, 2 * n2, 1, 0, uk, 2 * n2, kvt + (size_t)o * 2 * n2 * rv, 2 * n2,
                      m2l + (size_t)o * ru * rv, ru, T(1), T(0)});
      gemm_batched<T>(gd, st, s);
    }

    clk.tick("kernel_tables");
    // ---- initial bases W_b = orth([Phi U_K, Psi V_K, g, h])
    std::vector<T *> W(nb), phiU(nb), psiV(nb);
    std::vector<int> r(nb);
    {
      std::vector<GemmDesc<T>> gd;
      std::vector<CopyDesc<T>> cd;
      std::vector<T *> cand(nb);
      for (int b = 0; b < nb; ++b) {
        W[b] = level_arena->get<T>((size_t)m[b] * std::max(1, m[b]));
        phiU[b] = level_arena->get<T>((size_t)m[b] * ru);
        psiV[b] = level_arena->get<T>((size_t)m[b] * rv);
        cand[b] = phase_arena.get<T>((size_t)m[b] * (ru + rv + 2));
        gd.push_back({m[b], ru, 2 * n2, 0, 0, phi[b], m[b], uk, 2 * n2, phiU[b], m[b], T(1), T(0)});
        gd.push_back({m[b], rv, 7 * n2, 0, 0, psi[b], m[b], vk, 7 * n2, psiV[b], m[b], T(1), T(0)});
      }
      gemm_batched<T>(gd, st, s);
      for (int b = 0; b < nb; ++b) {
        cd.push_back({phiU[b], m[b], cand[b], m[b], m[b], ru, 0, 0, T(1)});
        cd.push_back({psiV[b], m[b], cand[b] + (size_t)m[b] * ru, m[b], m[b], rv, 0, 0, T(1)});
        cd.push_back({gvec[b], m[b], cand[b] + (size_t)m[b] * (ru + rv), m[b], m[b], 1, 0, 0, T(1)});
        cd.push_back({hvec[b], m[b], cand[b] + (size_t)m[b] * (ru + rv + 1), m[b], m[b], 1, 0, 0, T(1)});
      }
      copy_batched<T>(cd, st, s);
      {
        std::vector<NormDesc<T>> nd;
        for (int b = 0; b < nb; ++b) nd.push_back({cand[b], m[b], m[b], ru + rv + 2});
        normalize_batched<T>(nd, st, s);
      }
      std::vector<PgsDesc<T>> pd;
      for (int b = 0; b < nb; ++b)
        pd.push_back({cand[b], m[b], m[b], ru + rv + 2, W[b], m[b], 0, m[b], eps, counts.p + b});
      pgs_batched<T>(pd, st, s);
      std::vector<int> hr(nb);
      SBIE_HIP(hipMemcpyAsync(hr.data(), counts.p, nb * sizeof(int), hipMemcpyDeviceToHost, s));
      clk.sync(s);
      st.reset();
      r = hr;
    }
    clk.tick("initial_bases");
    // ---- projections and initial couplings
    std::vector<T *> Gh(nb), Hh(nb), g0(nb), h0(nb);
    PairMap<Blk<T>> Tc;
    {
      std::vector<GemmDesc<T>> gd;
      for (int b = 0; b < nb; ++b) {
        Gh[b] = phase_arena.get<T>((size_t)std::max(1, r[b]) * ru);
        Hh[b] = phase_arena.get<T>((size_t)std::max(1, r[b]) * rv);
        g0[b] = phase_arena.get<T>(std::max(1, r[b]));
        h0[b] = phase_arena.get<T>(std::max(1, r[b]));
        gd.push_back({r[b], ru, m[b], 1, 0, W[b], m[b], phiU[b], m[b], Gh[b], std::max(1, r[b]), T(1), T(0)});
        gd.push_back({r[b], rv, m[b], 1, 0, W[b], m[b], psiV[b], m[b], Hh[b], std::max(1, r[b]), T(1), T(0)});
        gd.push_back({r[b], 1, m[b], 1, 0, W[b], m[b], gvec[b], m[b], g0[b], std::max(1, r[b]), T(1), T(0)});
        gd.push_back({r[b], 1, m[b], 1, 0, W[b], m[b], hvec[b], m[b], h0[b], std::max(1, r[b]), T(1), T(0)});
      }
      gemm_batched<T>(gd, st, s);
      // coupling blocks z_b <- y_c for the interaction list and the
      // neighbours; capacity m_b x m_c, zero-initialised
      {
        size_t tot = 0;
        for (int b = 0; b < nb; ++b) {
          for (int c : L.ilist[b]) tot += (size_t)std::max(1, m[b]) * std::max(1, m[c]);
          for (int c : L.nbrs[b]) tot += (size_t)std::max(1, m[b]) * std::max(1, m[c]);
        }
        T *pool = level_arena->get<T>(tot);
        fill_value<T>(pool, tot, T(0), s);
        size_t used = 0;
        size_t nblk = 0;
        for (int b = 0; b < nb; ++b) nblk += L.ilist[b].size() + L.nbrs[b].size();
        Tc.reserve(2 * nblk);
        for (int b = 0; b < nb; ++b) {
          auto add = [&](int c) {
            Blk<T> bl;
            bl.ld = std::max(1, m[b]);
            bl.p = pool + used;
            used += (size_t)bl.ld * std::max(1, m[c]);
            Tc.emplace(std::make_pair(b, c), bl);
          };
          for (int c : L.ilist[b]) add(c);
          for (int c : L.nbrs[b]) add(c);
        }
      }
      gd.clear();
      std::vector<GemmDesc<T>> gd2;
      // index of each interaction-list offset (dx, dy) among the 40 tables
      int offset_index[7][7] = {};
      {
        int cnt = 0;
        for (int ddx = -3; ddx <= 3; ++ddx)
          for (int ddy = -3; ddy <= 3; ++ddy) {
            if (std::max(std::abs(ddx), std::abs(ddy)) < 2) continue;
            offset_index[ddx + 3][ddy + 3] = cnt++;
          }
      }
      for (int b = 0; b < nb; ++b)
        for (int c : L.ilist[b]) {
          const int dx = (int)(L.ix[c] - L.ix[b]), dy = (int)(L.iy[c] - L.iy[b]);
          const int o = offset_index[dx + 3][dy + 3];
          T *tmp = phase_arena.get<T>((size_t)std::max(1, r[b]) * rv);
          gd.push_back({r[b], rv, ru, 0, 0, Gh[b], std::max(1, r[b]), m2l + (size_t)o * ru * rv, ru, tmp,
                        std::max(1, r[b]), T(1), T(0)});
          Blk<T> &tb = blk(Tc, b, c);
          gd2.push_back({r[b], r[c], rv, 0, 1, tmp, std::max(1, r[b]), Hh[c], std::max(1, r[c]), tb.p, tb.ld,
                         T(1), T(1)});
          gd2.push_back({r[b], r[c], 1, 0, 1, g0[b], std::max(1, r[b]), h0[c], std::max(1, r[c]), tb.p, tb.ld,
                         T(1.0 / wall_len), T(1)});
        }
      gemm_batched<T>(gd, st, s);
      // the two accumulations into one block must not run concurrently:
      // split them into two launches
      std::vector<GemmDesc<T>> ga, gb2;
      for (size_t q = 0; q < gd2.size(); ++q) (q % 2 ? gb2 : ga).push_back(gd2[q]);
      gemm_batched<T>(ga, st, s);
      gemm_batched<T>(gb2, st, s);
      clk.sync(s);
      st.reset();
    }

    clk.tick("initial_couplings");
    // ---- elimination, colour by colour
    std::vector<char> gone(nb, 0);
    std::vector<std::vector<int>> colors(9);
    for (int b = 0; b < nb; ++b)
      colors[(int)((L.ix[b] % 3) * 3 + (L.iy[b] % 3))].push_back(b);
    T *lrhs = rhs[li], *lgs = gsave[li], *lt = tbuf[li], *lv = vbuf[li], *lx = xbuf[li];
    const std::vector<int64_t> &off = lvl_off[li];
    // parent offsets are known only after the level; record per-box data
    struct Rec {
      int i;
      std::vector<int> act;
      T *axx, *axy, *azx;
      int r;
      std::vector<T *> mik, nji;   // per active neighbour
    };
    std::vector<Rec> recs;
    std::vector<std::vector<int>> phase_boxes;
    T *omega = phase_arena.get<T>((size_t)std::max(1, *std::max_element(m.begin(), m.end())) * kSketch);
    gaussian_fill<T>(omega, (size_t)std::max(1, *std::max_element(m.begin(), m.end())) * kSketch,
                     3000 + lev, s);
    for (int col = 0; col < 9; ++col) {
      const std::vector<int> &E = colors[col];
      if (E.empty()) continue;
      phase_boxes.push_back(E);
      Arena pa((size_t)128 << 20, &chunk_cache);
      const int ne = (int)E.size();
      std::vector<std::vector<int>> act(ne);
      for (int e = 0; e < ne; ++e)
        for (int k : L.nbrs[E[e]])
          if (k != E[e] && !gone[k]) act[e].push_back(k);
      // A: S_ii^{-1}
      std::vector<T *> sinv(ne), X(ne), Y(ne), piv(ne), axy(ne), azx(ne);
      if (ne > 65536) fail(SBIE_UNSUPPORTED, "too many boxes in one colour");
      std::vector<CopyDesc<T>> cd;
      std::vector<int> ns;
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        sinv[e] = persist.get<T>((size_t)m[i] * m[i]);
        cd.push_back({blk(S, i, i).p, m[i], sinv[e], m[i], m[i], m[i], 0, 0, T(1)});
        ns.push_back(m[i]);
      }
      copy_batched<T>(cd, st, s);
      inverse_batched_blocked<T>(sinv, ns, info.p, st, s);
      // B: X = S^{-1} W, Y = S^{-T} W ; C: Piv = W^T X
      std::vector<GemmDesc<T>> gd;
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        const int ri = std::max(1, r[i]);
        X[e] = pa.get<T>((size_t)m[i] * ri);
        Y[e] = pa.get<T>((size_t)m[i] * ri);
        piv[e] = persist.get<T>((size_t)ri * ri);
        gd.push_back({m[i], r[i], m[i], 0, 0, sinv[e], m[i], W[i], m[i], X[e], m[i], T(1), T(0)});
        gd.push_back({m[i], r[i], m[i], 1, 0, sinv[e], m[i], W[i], m[i], Y[e], m[i], T(1), T(0)});
      }
      gemm_batched<T>(gd, st, s);
      gd.clear();
      std::vector<T *> pivp;
      std::vector<int> pivn;
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        if (r[i] == 0) continue;
        gd.push_back({r[i], r[i], m[i], 1, 0, W[i], m[i], X[e], m[i], piv[e], r[i], T(1), T(0)});
        pivp.push_back(piv[e]);
        pivn.push_back(r[i]);
      }
      gemm_batched<T>(gd, st, s);
      inverse_batched_blocked<T>(pivp, pivn, info.p + ne, st, s);
      // D: A_xy = X Piv^{-1}, A_zx = Piv^{-1} Y^T, A_xx = S^{-1} - A_xy Y^T
      gd.clear();
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        const int ri = std::max(1, r[i]);
        axy[e] = persist.get<T>((size_t)m[i] * ri);
        azx[e] = persist.get<T>((size_t)ri * m[i]);
        gd.push_back({m[i], r[i], r[i], 0, 0, X[e], m[i], piv[e], ri, axy[e], m[i], T(1), T(0)});
        gd.push_back({r[i], m[i], r[i], 0, 1, piv[e], ri, Y[e], m[i], azx[e], ri, T(1), T(0)});
      }
      gemm_batched<T>(gd, st, s);
      gd.clear();
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        gd.push_back({m[i], m[i], r[i], 0, 1, axy[e], m[i], Y[e], m[i], sinv[e], m[i], T(-1), T(1)});
      }
      gemm_batched<T>(gd, st, s);
      // E: M_ik = A_xx S_ik, G_ik = A_zx S_ik, B_ij = S_ji A_xy
      std::vector<SmallMap<T *>> Mik(ne), Gik(ne), Bij(ne), Nji(ne);
      gd.clear();
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        const int ri = std::max(1, r[i]);
        for (int k : act[e]) {
          T *mm = persist.get<T>((size_t)m[i] * m[k]);
          T *nn_ = persist.get<T>((size_t)m[k] * m[i]);
          Nji[e][k] = nn_;
          T *gg = pa.get<T>((size_t)ri * m[k]);
          T *bb = pa.get<T>((size_t)m[k] * ri);
          Mik[e][k] = mm;
          Gik[e][k] = gg;
          Bij[e][k] = bb;
          const Blk<T> &sik = blk(S, i, k), &ski = blk(S, k, i);
          gd.push_back({m[i], m[k], m[i], 0, 0, sinv[e], m[i], sik.p, sik.ld, mm, m[i], T(1), T(0)});
          gd.push_back({r[i], m[k], m[i], 0, 0, azx[e], ri, sik.p, sik.ld, gg, ri, T(1), T(0)});
          gd.push_back({m[k], r[i], m[i], 0, 0, ski.p, ski.ld, axy[e], m[i], bb, m[k], T(1), T(0)});
          gd.push_back({m[k], m[i], m[i], 0, 0, ski.p, ski.ld, sinv[e], m[i], nn_, m[k], T(1), T(0)});
        }
      }
      gemm_batched<T>(gd, st, s);
      clk.tick("elim_pivots", lev);
      // F: fill-ins
      struct Far {
        int e, j, k;
        T *f;
      };
      std::vector<Far> far;
      gd.clear();
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        for (int j : act[e])
          for (int k : act[e]) {
            const Blk<T> &sji = blk(S, j, i);
            const bool nbr = std::find(L.nbrs[j].begin(), L.nbrs[j].end(), k) != L.nbrs[j].end();
            if (nbr) {
              Blk<T> &sjk = blk(S, j, k);
              gd.push_back({m[j], m[k], m[i], 0, 0, sji.p, sji.ld, Mik[e][k], m[i], sjk.p, sjk.ld, T(-1), T(1)});
            } else {
              T *f = pa.get<T>((size_t)m[j] * m[k]);
              far.push_back({e, j, k, f});
              gd.push_back({m[j], m[k], m[i], 0, 0, sji.p, sji.ld, Mik[e][k], m[i], f, m[j], T(-1), T(0)});
            }
          }
      }
      gemm_batched<T>(gd, st, s);
      // G: augmentation of the neighbours' bases
      //   norms of the candidate blocks
      std::vector<NormDesc<T>> nd;
      for (int e = 0; e < ne; ++e) {
        const int ri = std::max(1, r[E[e]]);
        for (int k : act[e]) {
          nd.push_back({Bij[e][k], m[k], m[k], r[E[e]]});
          nd.push_back({Gik[e][k], ri, r[E[e]], m[k]});
        }
      }
      const size_t nfar0 = nd.size();
      for (auto &f : far) nd.push_back({f.f, m[f.j], m[f.j], m[f.k]});
      if (nd.size() > 65536) fail(SBIE_UNSUPPORTED, "too many fill-in blocks");
      norms_batched<T>(nd, norms.p, st, s);
      std::vector<double> hnorm(nd.size());
      if (!nd.empty())
        SBIE_HIP(hipMemcpyAsync(hnorm.data(), norms.p, nd.size() * 8, hipMemcpyDeviceToHost, s));
      std::vector<int32_t> hinfo(2 * ne);
      SBIE_HIP(hipMemcpyAsync(hinfo.data(), info.p, 2 * ne * 4, hipMemcpyDeviceToHost, s));
      clk.sync(s);
      st.reset();
      for (int e = 0; e < ne; ++e)
        if (hinfo[e] != 0) fail(SBIE_BREAKDOWN, "singular near-field pivot at level %d", lev);
      {
        int q = 0;
        for (int e = 0; e < ne; ++e) {
          if (r[E[e]] == 0) continue;
          if (hinfo[ne + q] != 0) fail(SBIE_BREAKDOWN, "singular multipole pivot at level %d", lev);
          ++q;
        }
      }
      //   candidate matrices per neighbour j (each j belongs to one e)
      struct Aug {
        int j, e;
        T *cand;
        int c;
      };
      std::vector<Aug> aug;
      std::vector<CopyDesc<T>> cc;
      gd.clear();
      {
        size_t q = 0;
        std::unordered_map<int, int> slot;
        // the fill-ins of each eliminated box are contiguous in `far`
        std::vector<size_t> far_end(ne + 1, 0);
        for (const Far &f : far) ++far_end[f.e + 1];
        for (int e = 0; e < ne; ++e) far_end[e + 1] += far_end[e];
        for (int e = 0; e < ne; ++e)
          for (int j : act[e]) {
            int cols = 2 * r[E[e]];
            for (size_t fi = far_end[e]; fi < far_end[e + 1]; ++fi)
              if (far[fi].j == j || far[fi].k == j) cols += kSketch;
            slot[j] = (int)aug.size();
            aug.push_back({j, e, pa.get<T>((size_t)m[j] * std::max(1, cols)), cols});
          }
        std::vector<int> fillc(aug.size(), 0);
        for (int e = 0; e < ne; ++e) {
          const int ri = r[E[e]];
          for (int k : act[e]) {
            Aug &a = aug[slot[k]];
            const double nb_ = hnorm[q++], ng_ = hnorm[q++];
            if (ri > 0) {
              cc.push_back({Bij[e][k], m[k], a.cand + (size_t)fillc[slot[k]] * m[k], m[k], m[k], ri, 0, 0,
                            T(nb_ > 0 ? 1.0 / nb_ : 0.0)});
              fillc[slot[k]] += ri;
              cc.push_back({Gik[e][k], std::max(1, ri), a.cand + (size_t)fillc[slot[k]] * m[k], m[k], m[k], ri, 1, 0,
                            T(ng_ > 0 ? 1.0 / ng_ : 0.0)});
              fillc[slot[k]] += ri;
            }
          }
        }
        for (size_t fi = 0; fi < far.size(); ++fi) {
          const Far &f = far[fi];
          const double nf = hnorm[nfar0 + fi];
          const T al = T(nf > 0 ? 1.0 / nf : 0.0);
          // column space of F_jk into W_j, row space (F_jk^T) into W_k
          Aug &aj = aug[slot[f.j]];
          gd.push_back({m[f.j], kSketch, m[f.k], 0, 0, f.f, m[f.j], omega, m[f.k],
                        aj.cand + (size_t)fillc[slot[f.j]] * m[f.j], m[f.j], al, T(0)});
          fillc[slot[f.j]] += kSketch;
          Aug &ak = aug[slot[f.k]];
          gd.push_back({m[f.k], kSketch, m[f.j], 1, 0, f.f, m[f.j], omega, m[f.j],
                        ak.cand + (size_t)fillc[slot[f.k]] * m[f.k], m[f.k], al, T(0)});
          fillc[slot[f.k]] += kSketch;
        }
        for (size_t a = 0; a < aug.size(); ++a) aug[a].c = fillc[a];
      }
      copy_batched<T>(cc, st, s);
      gemm_batched_sketch<T>(gd, sketch_in, st, s);
      clk.tick("elim_fillins");
      //   project out the current basis twice: P = W^T C, C -= W P
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<GemmDesc<T>> g1, g2;
        std::vector<T *> pp(aug.size());
        for (size_t a = 0; a < aug.size(); ++a) {
          const int j = aug[a].j;
          if (aug[a].c == 0 || r[j] == 0) continue;
          pp[a] = pa.get<T>((size_t)r[j] * aug[a].c);
          g1.push_back({r[j], aug[a].c, m[j], 1, 0, W[j], m[j], aug[a].cand, m[j], pp[a], r[j], T(1), T(0)});
          g2.push_back({m[j], aug[a].c, r[j], 0, 0, W[j], m[j], pp[a], r[j], aug[a].cand, m[j], T(-1), T(1)});
        }
        gemm_batched<T>(g1, st, s);
        gemm_batched<T>(g2, st, s);
      }
      //   wide candidate sets are sketched by a Gaussian matrix first: the
      //   range of C Omega is the range of C with high probability when the
      //   rank found stays well below the sketch width
      int cmax = 0;
      for (const auto &ag : aug) cmax = std::max(cmax, ag.c);
      std::vector<GemmDesc<T>> gsk;
      std::vector<T *> ysk(aug.size(), nullptr);
      if (cmax > kPgsSketch) {
        T *om = pa.get<T>((size_t)cmax * kPgsSketch);
        gaussian_fill<T>(om, (size_t)cmax * kPgsSketch, 5000 + 131 * lev + col, s);
        for (size_t a = 0; a < aug.size(); ++a) {
          if (aug[a].c <= kPgsSketch) continue;
          const int j = aug[a].j;
          ysk[a] = pa.get<T>((size_t)m[j] * kPgsSketch);
          gsk.push_back({m[j], kPgsSketch, aug[a].c, 0, 0, aug[a].cand, m[j], om, cmax, ysk[a], m[j],
                         T(1.0 / std::sqrt((double)kPgsSketch)), T(0)});
        }
        gemm_batched_sketch<T>(gsk, sketch_in, st, s);
        if (sketch_in != GemmInputs::kWorking) {
          // rounding the projected candidates to FP16 / BF16 brings back
          // components along the current basis of the size of the unit
          // roundoff; the pivoted Gram-Schmidt below assumes there are none,
          // so the sketch is projected once more in the factor's precision
          std::vector<GemmDesc<T>> g1, g2;
          for (size_t a = 0; a < aug.size(); ++a) {
            const int j = aug[a].j;
            if (!ysk[a] || r[j] == 0) continue;
            T *pp = pa.get<T>((size_t)r[j] * kPgsSketch);
            g1.push_back({r[j], kPgsSketch, m[j], 1, 0, W[j], m[j], ysk[a], m[j], pp, r[j], T(1), T(0)});
            g2.push_back({m[j], kPgsSketch, r[j], 0, 0, W[j], m[j], pp, r[j], ysk[a], m[j], T(-1), T(1)});
          }
          gemm_batched<T>(g1, st, s);
          gemm_batched<T>(g2, st, s);
        }
      }
      std::vector<PgsDesc<T>> pd;
      for (size_t a = 0; a < aug.size(); ++a) {
        const int j = aug[a].j;
        if (aug[a].c == 0) {
          continue;
        }
        // both candidate sets are orthogonal to W[j][:, :r[j]] (projected
        // twice above; the sketch only combines projected columns)
        if (ysk[a])
          pd.push_back({ysk[a], m[j], m[j], kPgsSketch, W[j], m[j], r[j], m[j], eps, counts.p + a, r[j]});
        else
          pd.push_back({aug[a].cand, m[j], m[j], aug[a].c, W[j], m[j], r[j], m[j], eps, counts.p + a,
                        r[j]});
      }
      fill_value<int>(counts.p, aug.size() + 1, 0, s);
      pgs_batched<T>(pd, st, s);
      std::vector<int> add(aug.size() + 1, 0);
      SBIE_HIP(hipMemcpyAsync(add.data(), counts.p, (aug.size() + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
      clk.sync(s);
      st.reset();
      std::vector<int> rold = r;
      for (size_t a = 0; a < aug.size(); ++a) r[aug[a].j] += add[a];
      clk.tick("elim_recompress", lev);
      // H: couplings with the new bases
      std::vector<CopyDesc<T>> tc;
      std::vector<GemmDesc<T>> g1, g2;
      for (int e = 0; e < ne; ++e) {
        const int i = E[e];
        const int ri = r[i];
        if (ri > 0) {
          Blk<T> &tii = blk(Tc, i, i);
          tc.push_back({piv[e], ri, tii.p, tii.ld, ri, ri, 0, 1, T(1)});
        }
        for (int j : act[e]) {
          Blk<T> &tji = blk(Tc, j, i), &tij = blk(Tc, i, j);
          g1.push_back({r[j], ri, m[j], 1, 0, W[j], m[j], Bij[e][j], m[j], tji.p, tji.ld, T(1), T(1)});
          g1.push_back({ri, r[j], m[j], 0, 0, Gik[e][j], std::max(1, ri), W[j], m[j], tij.p, tij.ld, T(1), T(1)});
        }
      }
      std::vector<T *> ftmp(far.size());
      for (size_t fi = 0; fi < far.size(); ++fi) {
        const Far &f = far[fi];
        ftmp[fi] = pa.get<T>((size_t)m[f.j] * std::max(1, r[f.k]));
        g1.push_back({m[f.j], r[f.k], m[f.k], 0, 0, f.f, m[f.j], W[f.k], m[f.k], ftmp[fi], m[f.j], T(1), T(0)});
        Blk<T> &tjk = blk(Tc, f.j, f.k);
        g2.push_back({r[f.j], r[f.k], m[f.j], 1, 0, W[f.j], m[f.j], ftmp[fi], m[f.j], tjk.p, tjk.ld, T(1), T(1)});
      }
      copy_batched<T>(tc, st, s);
      gemm_batched<T>(g1, st, s);
      gemm_batched<T>(g2, st, s);
      // record
      for (int e = 0; e < ne; ++e) {
        Rec rc{E[e], act[e], sinv[e], axy[e], azx[e], r[E[e]], {}, {}};
        for (int k : act[e]) {
          rc.mik.push_back(Mik[e][k]);
          rc.nji.push_back(Nji[e][k]);
        }
        recs.push_back(rc);
        gone[E[e]] = 1;
      }
      // no wait here: the next phase's host work overlaps these launches
      // (the staging ring waits by itself when it wraps, and the phase
      // arena's chunks are only reused by later launches on this stream)
      (void)rold;
      clk.tick("elim_couplings");
    }
    for (int b = 0; b < nb; ++b) max_rank = std::max(max_rank, r[b]);

    // ---- level change: the parent level's H^2 system
    const HLevel &P = tr.lv[lev - 1];
    const int np_ = P.size();
    std::vector<int> mp(np_, 0), in_par(nb, 0);
    for (int p = 0; p < np_; ++p)
      for (int c : P.children[p]) {
        in_par[c] = mp[p];
        mp[p] += r[c];
      }
    alloc_level_vectors(li + 1, mp);
    const std::vector<int64_t> &poff = lvl_off[li + 1];
    auto next_arena = std::make_unique<Arena>((size_t)256 << 20, &chunk_cache);
    std::vector<T *> nphi(np_), npsi(np_), ngv(np_), nhv(np_);
    decltype(S) Sp;
    {
      std::vector<CopyDesc<T>> cd;
      size_t tot = 0;
      for (int p = 0; p < np_; ++p)
        for (int q : P.nbrs[p]) tot += (size_t)std::max(1, mp[p]) * std::max(1, mp[q]);
      T *pool = next_arena->get<T>(tot);
      fill_value<T>(pool, tot, T(0), s);
      size_t used = 0;
      for (int p = 0; p < np_; ++p)
        for (int q : P.nbrs[p]) {
          Blk<T> bl;
          bl.ld = std::max(1, mp[p]);
          bl.p = pool + used;
          used += (size_t)bl.ld * std::max(1, mp[q]);
          Sp.emplace(std::make_pair(p, q), bl);
          for (int c : P.children[p])
            for (int d : P.children[q]) {
              auto it = Tc.find({c, d});
              if (it == Tc.end()) continue;
              cd.push_back({it->second.p, it->second.ld, bl.p + in_par[c] + (size_t)in_par[d] * bl.ld, bl.ld,
                            r[c], r[d], 0, 0, T(1)});
            }
        }
      copy_batched<T>(cd, st, s);
      std::vector<GemmDesc<T>> g1, g2;
      for (int p = 0; p < np_; ++p) {
        const int mpp = std::max(1, mp[p]);
        nphi[p] = next_arena->get<T>((size_t)mpp * 2 * n2);
        npsi[p] = next_arena->get<T>((size_t)mpp * 7 * n2);
        ngv[p] = next_arena->get<T>(mpp);
        nhv[p] = next_arena->get<T>(mpp);
        for (int c : P.children[p]) {
          if (r[c] == 0) continue;
          const int q = (int)((L.ix[c] & 1) + 2 * (L.iy[c] & 1));
          T *gfull = phase_arena.get<T>((size_t)r[c] * 2 * n2);
          T *hfull = phase_arena.get<T>((size_t)r[c] * 7 * n2);
          g1.push_back({r[c], 2 * n2, m[c], 1, 0, W[c], m[c], phi[c], m[c], gfull, r[c], T(1), T(0)});
          g1.push_back({r[c], 7 * n2, m[c], 1, 0, W[c], m[c], psi[c], m[c], hfull, r[c], T(1), T(0)});
          g1.push_back({r[c], 1, m[c], 1, 0, W[c], m[c], gvec[c], m[c], ngv[p] + in_par[c], mpp, T(1), T(0)});
          g1.push_back({r[c], 1, m[c], 1, 0, W[c], m[c], hvec[c], m[c], nhv[p] + in_par[c], mpp, T(1), T(0)});
          for (int comp = 0; comp < 7; ++comp) {
            if (comp < 2)
              g2.push_back({r[c], n2, n2, 0, 0, gfull + (size_t)comp * n2 * r[c], r[c], transfer + (size_t)q * n2 * n2,
                            n2, nphi[p] + in_par[c] + (size_t)comp * n2 * mpp, mpp, T(1), T(0)});
            g2.push_back({r[c], n2, n2, 0, 0, hfull + (size_t)comp * n2 * r[c], r[c], transfer + (size_t)q * n2 * n2,
                          n2, npsi[p] + in_par[c] + (size_t)comp * n2 * mpp, mpp, T(1), T(0)});
          }
        }
      }
      gemm_batched<T>(g1, st, s);
      gemm_batched<T>(g2, st, s);
    }
    clk.tick("level_change");
    // ---- solve plan of this level (parent offsets now known)
    {
      T *prhs = rhs[li + 1];
      T *px_ = xbuf[li + 1];
      std::unordered_map<int, const Rec *> byi;
      for (const Rec &rc : recs) byi[rc.i] = &rc;
      std::vector<SolvePhase<T>> &plist = phases[li];
      Packed pk;
      struct Offs { size_t f, ft, b, bt; int nf, nb; };
      std::vector<Offs> offs;
      for (const auto &E : phase_boxes) {
        std::vector<GemvDesc<T>> fd, bd;
        std::vector<GemvTerm<T>> ft, bt;
        for (int i : E) {
          const Rec &rc = *byi[i];
          const int mi = m[i], ri = rc.r;
          T *gi = lrhs + off[i];
          const int pp = L.parent[i];
          add_gemv(fd, ft, lt + off[i], mi, T(0), {GemvTerm<T>{rc.axx, gi, mi, mi, 0, T(1)}});
          if (ri > 0)
            add_gemv(fd, ft, prhs + poff[pp] + in_par[i], ri, T(0),
                     {GemvTerm<T>{rc.azx, gi, std::max(1, ri), mi, 0, T(1)}});
          for (size_t q = 0; q < rc.act.size(); ++q) {
            const int j = rc.act[q];
            add_gemv(fd, ft, lrhs + off[j], m[j], T(1), {GemvTerm<T>{rc.nji[q], gi, m[j], mi, 0, T(-1)}});
          }
          std::vector<GemvTerm<T>> terms;
          for (size_t q = 0; q < rc.act.size(); ++q) {
            const int k = rc.act[q];
            terms.push_back({rc.mik[q], lx + off[k], mi, m[k], 0, T(-1)});
          }
          if (ri > 0) terms.push_back({rc.axy, px_ + poff[pp] + in_par[i], mi, ri, 0, T(1)});
          add_gemv(bd, bt, lx + off[i], mi, T(1), terms, lt + off[i]);
        }
        offs.push_back({pk.add(fd), pk.add(ft), pk.add(bd), pk.add(bt), (int)fd.size(), (int)bd.size()});
        if (apply32) host_phases[li].push_back({fd, bd, ft, bt});
      }
      char *base = send(pk, persist, s);
      for (const Offs &o : offs) {
        SolvePhase<T> ph;
        ph.f = at<GemvDesc<T>>(base, o.f);
        ph.ft = at<GemvTerm<T>>(base, o.ft);
        ph.nf = o.nf;
        ph.b = at<GemvDesc<T>>(base, o.b);
        ph.bt = at<GemvTerm<T>>(base, o.bt);
        ph.nb = o.nb;
        plist.push_back(ph);
      }
    }
    clk.sync(s);
    st.reset();
    // advance
    clk.tick("solve_plan");
    S = std::move(Sp);
    phi = nphi;
    psi = npsi;
    gvec = ngv;
    hvec = nhv;
    m = mp;
    level_arena = std::move(next_arena);
  }

  // ---- root: dense inverse of the remaining system
  {
    const HLevel &R = tr.lv[tr.root];
    const int nb = R.size();
    if (tr.depth == tr.root) lvl_off[0] = lvl_off[0];
    const std::vector<int64_t> &off = lvl_off[nelim];
    root_dim = (int)off.back();
    const int rd = std::max(1, root_dim);
    root_inv = persist.get<T>((size_t)rd * rd);
    fill_value<T>(root_inv, (size_t)rd * rd, T(0), s);
    std::vector<CopyDesc<T>> cd;
    for (int b = 0; b < nb; ++b)
      for (int c : R.nbrs[b]) {
        const Blk<T> &bl = blk(S, b, c);
        cd.push_back({bl.p, bl.ld, root_inv + off[b] + (size_t)off[c] * rd, rd, m[b], m[c], 0, 0, T(1)});
      }
    copy_batched<T>(cd, st, s);
    if (root_dim > 0) {
      inverse_batched_blocked<T>({root_inv}, {root_dim}, info.p, st, s);
      int32_t hi = 0;
      SBIE_HIP(hipMemcpyAsync(&hi, info.p, 4, hipMemcpyDeviceToHost, s));
      clk.sync(s);
      if (hi != 0) fail(SBIE_BREAKDOWN, "singular root system");
      std::vector<GemvDesc<T>> rdsc;
      std::vector<GemvTerm<T>> rt;
      add_gemv(rdsc, rt, xbuf[nelim], root_dim, T(0), {GemvTerm<T>{root_inv, rhs[nelim], rd, root_dim, 0, T(1)}});
      plan.root_d = upload(rdsc);
      plan.root_t = upload(rt);
      plan.root_nd = (int)rdsc.size();
      if (apply32) host_root = {rdsc, {}, rt, {}};
    }
  }
  clk.sync(s);
  clk.tick("root");
  level_arena.reset();
  plan.rhs0 = rhs[0];
  plan.x0 = xbuf[0];
  if (apply32) build_plan32(s);
  if (!defer_graph) build_graph();
  clk.tick("graph");
  stats.levels = tr.depth + 1;
  stats.leaves = nleaf;
  stats.max_rank = max_rank;
  stats.factor_bytes = (int64_t)persist.total;
  stats.factor_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  stats.gemm_flops = op_flops().gemm;
  stats.gemm_low_flops = op_flops().gemm_low;
  stats.inverse_flops = op_flops().inverse;
}

}  // namespace
}  // namespace sbie

struct ifmm_handle {
  std::unique_ptr<sbie::IfmmImplBase> impl;
};

namespace sbie {
void ifmm_apply(const ifmm_handle *h, const double *b, double *x, hipStream_t s) {
  h->impl->apply(b, x, s);
}
}  // namespace sbie

namespace sbie {
ifmm_handle *ifmm_factor_internal(const sbie_geom *g, const ifmm_params *p, hipStream_t s,
                                  bool defer_graph) {
  validate_geom(g);
  if (!p) fail(SBIE_INVALID_ARGUMENT, "null pointer");
  if (p->reserved != 0) fail(SBIE_INVALID_ARGUMENT, "ifmm_params.reserved must be 0");
  if (p->compress < 0 || p->compress > 2)
    fail(SBIE_INVALID_ARGUMENT, "compress must be 0 (factor precision), 1 (FP16 inputs) or 2 (BF16 inputs)");
  validate_geom_device(g, s);
  auto h = std::make_unique<ifmm_handle>();
  if (p->precision == 0 || p->precision == 2) {
    auto impl = std::make_unique<IfmmImpl<double>>();
    impl->defer_graph = defer_graph;
    impl->apply32 = p->precision == 2;
    impl->factor(g, p, s);
    h->impl = std::move(impl);
  } else if (p->precision == 1) {
    auto impl = std::make_unique<IfmmImpl<float>>();
    impl->defer_graph = defer_graph;
    impl->factor(g, p, s);
    h->impl = std::move(impl);
  } else {
    fail(SBIE_INVALID_ARGUMENT, "precision must be 0 (FP64), 1 (FP32) or 2 (FP64 factor, FP32 apply)");
  }
  return h.release();
}

void ifmm_capture(ifmm_handle *h) {
  if (h->impl->defer_graph) {
    h->impl->capture_graph();
    h->impl->defer_graph = false;
  }
}
}  // namespace sbie

extern "C" int ifmm_factor(const sbie_geom *g, const ifmm_params *p, ifmm_handle **out,
                           void *stream) {
  return sbie::guarded([&]() {
    if (!out) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    *out = nullptr;
    *out = sbie::ifmm_factor_internal(g, p, (hipStream_t)stream, false);
    return SBIE_OK;
  });
}

extern "C" int ifmm_solve(const ifmm_handle *h, const double *b, double *x, void *stream) {
  return sbie::guarded([&]() {
    if (!h || !b || !x) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (b < x + h->impl->n && x < b + h->impl->n) sbie::fail(SBIE_INVALID_ARGUMENT, "b and x overlap");
    h->impl->apply(b, x, (hipStream_t)stream);
    return SBIE_OK;
  });
}

extern "C" int ifmm_destroy(ifmm_handle *h) {
  return sbie::guarded([&]() {
    delete h;
    return SBIE_OK;
  });
}

extern "C" int ifmm_get_stats(const ifmm_handle *h, ifmm_stats *s) {
  return sbie::guarded([&]() {
    if (!h || !s) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    *s = h->impl->stats;
    return SBIE_OK;
  });
}

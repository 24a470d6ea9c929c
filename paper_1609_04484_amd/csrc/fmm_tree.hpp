// Quadtree and interaction lists of the fast multipole method (host code,
// no device calls; used by fmm.hip and checked on the CPU by the tests).
//
// The tree covers the bounding square of the nodes; only non-empty boxes
// are kept, level by level in Morton order.  Uniform trees split every box
// down to one depth; adaptive trees split every box that holds more than
// `target` nodes.  Lists (for a box B):
//   V  children of the colleagues (touching same-level boxes) of B's parent
//      that do not touch B: multipole to local, same level
//   U  (leaf B) every leaf touching B, B included: direct sum
//   W  (leaf B) boxes smaller than B that do not touch B but whose parents
//      do: their multipoles are evaluated at B's nodes
//   X  the inverse of W: a larger leaf's sources into B's local expansion
// Together they cover every (target leaf, source leaf) pair exactly once.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace sbie {

constexpr int kFmmMaxDepth = 20;

inline uint64_t fmm_morton(uint32_t ix, uint32_t iy) {
  auto spread = [](uint64_t v) {
    v &= 0xffffffffull;
    v = (v | (v << 16)) & 0x0000ffff0000ffffull;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
  };
  return spread(ix) | (spread(iy) << 1);
}

inline void fmm_demorton(uint64_t c, uint32_t &ix, uint32_t &iy) {
  auto pack = [](uint64_t v) {
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v >> 4)) & 0x00ff00ff00ff00ffull;
    v = (v | (v >> 8)) & 0x0000ffff0000ffffull;
    v = (v | (v >> 16)) & 0x00000000ffffffffull;
    return (uint32_t)v;
  };
  ix = pack(c);
  iy = pack(c >> 1);
}

struct FmmTree {
  int depth = 0;             // deepest level
  int nleaf = 0, nbox = 0, nxbox = 0, min_leaf_level = 0;
  std::vector<int> lev_off;  // boxes of level l: [lev_off[l], lev_off[l + 1])
  std::vector<int> order;    // sorted position -> node
  std::vector<int> leaf_box, leaf_start;         // per leaf (node order)
  std::vector<int> par, quad, child, level;      // per box (child: 4 per box, -1 = none)
  std::vector<double> ctr, hb;                   // centre (2 per box), half width
  std::vector<int> vl_off, vl;                   // per box: V list (box indices)
  std::vector<int> ul_off, ul, wl_off, wl;       // per leaf: U (leaf indices), W (box indices)
  std::vector<int> xbox, xl_off, xl;             // boxes with X lists, their leaves
  int64_t m2l_pairs = 0, p2p_pairs = 0, m2p_pairs = 0, p2l_pairs = 0;
};

inline FmmTree build_fmm_tree(const double *hx, const double *hy, int64_t nn, int target, int max_depth,
                              bool adaptive) {
  FmmTree t;
  int depth = 0, nbox = 0, nleaf = 0, min_leaf_level = 0, nxbox = 0;
  int64_t m2l_pairs = 0, p2p_pairs = 0, m2p_pairs = 0, p2l_pairs = 0;
  std::vector<int> lev_off;
  double x0 = hx[0], x1 = hx[0], y0 = hy[0], y1 = hy[0];
  for (int64_t i = 0; i < nn; ++i) {
    x0 = std::min(x0, hx[i]);
    x1 = std::max(x1, hx[i]);
    y0 = std::min(y0, hy[i]);
    y1 = std::max(y1, hy[i]);
  }
  const double cx0 = 0.5 * (x0 + x1), cy0 = 0.5 * (y0 + y1);
  double h0 = 0.5 * std::max(x1 - x0, y1 - y0);
  h0 = h0 > 0.0 ? h0 * (1.0 + 1e-12) : 1.0;
  auto codes_at = [&](int L, std::vector<uint64_t> &c) {
    const double scale = (double)(1u << L) / (2.0 * h0);
    const uint32_t top = (1u << L) - 1;
    c.resize(nn);
    for (int64_t i = 0; i < nn; ++i) {
      const double fx = std::floor((hx[i] - (cx0 - h0)) * scale), fy = std::floor((hy[i] - (cy0 - h0)) * scale);
      const uint32_t ix = (uint32_t)std::min<double>(top, std::max(0.0, fx));
      const uint32_t iy = (uint32_t)std::min<double>(top, std::max(0.0, fy));
      c[i] = fmm_morton(ix, iy);
    }
  };
  // the finest level the tree may reach: uniform trees stop at one depth
  // (given, or the shallowest whose non-empty boxes hold at most `target`
  // nodes on average); adaptive trees split every box holding more than
  // `target` nodes, down to max_depth (default 20)
  int cut;
  std::vector<uint64_t> code;
  if (adaptive) {
    cut = max_depth > 0 ? max_depth : kFmmMaxDepth;
    codes_at(cut, code);
  } else if (max_depth > 0) {
    cut = max_depth;
    codes_at(cut, code);
  } else {
    for (cut = 0;; ++cut) {
      codes_at(cut, code);
      std::vector<uint64_t> u(code);
      std::sort(u.begin(), u.end());
      const int64_t nl = std::unique(u.begin(), u.end()) - u.begin();
      if (nn <= (int64_t)target * nl || cut == kFmmMaxDepth) break;
    }
  }
  // nodes in Morton order of the finest level (stable: a box keeps the node
  // order of its curves); every box is then a contiguous range of nodes
  std::vector<int> order(nn);
  for (int64_t i = 0; i < nn; ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return code[a] < code[b]; });
  std::vector<uint64_t> sc(nn);
  for (int64_t k = 0; k < nn; ++k) sc[k] = code[order[k]];
  struct Box {
    uint64_t code;
    int lo, hi;     // sorted nodes [lo, hi)
    int parent;     // index in the level above
    int kids[4];    // indices in the level below, -1 = none
  };
  std::vector<std::vector<Box>> lv(1);
  lv[0].push_back({0, 0, (int)nn, -1, {-1, -1, -1, -1}});
  for (int l = 0; l < cut; ++l) {
    std::vector<Box> next;
    const int sh = 2 * (cut - l - 1);
    for (size_t b = 0; b < lv[l].size(); ++b) {
      Box &bx = lv[l][b];
      if (adaptive && bx.hi - bx.lo <= target) continue;   // a leaf
      int a = bx.lo;
      while (a < bx.hi) {
        const uint64_t cc = sc[a] >> sh;
        int e = a + 1;
        while (e < bx.hi && (sc[e] >> sh) == cc) ++e;
        bx.kids[cc & 3] = (int)next.size();
        next.push_back({cc, a, e, (int)b, {-1, -1, -1, -1}});
        a = e;
      }
    }
    if (next.empty()) break;
    lv.push_back(std::move(next));
  }
  depth = (int)lv.size() - 1;
  lev_off.assign(depth + 2, 0);
  for (int l = 0; l <= depth; ++l) lev_off[l + 1] = lev_off[l] + (int)lv[l].size();
  nbox = lev_off[depth + 1];
  auto is_leaf = [&](int l, int b) {
    const Box &x = lv[l][b];
    return x.kids[0] < 0 && x.kids[1] < 0 && x.kids[2] < 0 && x.kids[3] < 0;
  };
  std::vector<double> hctr(2 * (size_t)nbox), hhb(nbox);
  std::vector<int> hpar(nbox, -1), hquad(nbox, 0), hchild(4 * (size_t)nbox, -1), hlevel(nbox);
  for (int l = 0; l <= depth; ++l) {
    const double h = h0 / (double)(1u << l);
    for (size_t b = 0; b < lv[l].size(); ++b) {
      const int gb = lev_off[l] + (int)b;
      uint32_t ix, iy;
      fmm_demorton(lv[l][b].code, ix, iy);
      hctr[2 * gb] = cx0 - h0 + (2.0 * ix + 1.0) * h;
      hctr[2 * gb + 1] = cy0 - h0 + (2.0 * iy + 1.0) * h;
      hhb[gb] = h;
      hlevel[gb] = l;
      if (l > 0) {
        hpar[gb] = lev_off[l - 1] + lv[l][b].parent;
        hquad[gb] = (int)(lv[l][b].code & 3);
      }
      for (int q = 0; q < 4; ++q)
        if (lv[l][b].kids[q] >= 0) hchild[4 * (size_t)gb + q] = lev_off[l + 1] + lv[l][b].kids[q];
    }
  }
  // leaves in node order
  std::vector<int> hleaf_box, leaf_of(nbox, -1);
  for (int l = 0; l <= depth; ++l)
    for (size_t b = 0; b < lv[l].size(); ++b)
      if (is_leaf(l, (int)b)) hleaf_box.push_back(lev_off[l] + (int)b);
  std::vector<int> lo_of(nbox), hi_of(nbox);
  for (int l = 0; l <= depth; ++l)
    for (size_t b = 0; b < lv[l].size(); ++b) {
      lo_of[lev_off[l] + b] = lv[l][b].lo;
      hi_of[lev_off[l] + b] = lv[l][b].hi;
    }
  std::sort(hleaf_box.begin(), hleaf_box.end(), [&](int a, int b) { return lo_of[a] < lo_of[b]; });
  nleaf = (int)hleaf_box.size();
  std::vector<int> ls(nleaf + 1);
  min_leaf_level = depth;
  for (int i = 0; i < nleaf; ++i) {
    leaf_of[hleaf_box[i]] = i;
    ls[i] = lo_of[hleaf_box[i]];
    min_leaf_level = std::min(min_leaf_level, hlevel[hleaf_box[i]]);
  }
  ls[nleaf] = (int)nn;
  // geometry in units of the finest cell: box gb spans [x0b, x1b] x [y0b, y1b]
  auto span = [&](int gb, int64_t &ax0, int64_t &ax1, int64_t &ay0, int64_t &ay1) {
    const int l = hlevel[gb];
    uint32_t ix, iy;
    fmm_demorton(lv[l][gb - lev_off[l]].code, ix, iy);
    const int64_t w = (int64_t)1 << (cut - l);
    ax0 = (int64_t)ix * w;
    ax1 = ax0 + w;
    ay0 = (int64_t)iy * w;
    ay1 = ay0 + w;
  };
  auto touch = [&](int a, int b) {   // closed boxes intersect
    int64_t a0, a1, a2, a3, b0, b1, b2, b3;
    span(a, a0, a1, a2, a3);
    span(b, b0, b1, b2, b3);
    return a0 <= b1 && b0 <= a1 && a2 <= b3 && b2 <= a3;
  };
  auto find = [&](int l, uint64_t c) -> int {
    const auto &v = lv[l];
    int lo = 0, hi = (int)v.size();
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (v[mid].code < c) lo = mid + 1; else hi = mid;
    }
    return (lo < (int)v.size() && v[lo].code == c) ? lev_off[l] + lo : -1;
  };
  // V lists: children of the parent's colleagues that do not touch the box
  std::vector<int> hvl_off(nbox + 1, 0), hvl;
  for (int l = 0; l <= depth; ++l)
    for (size_t b = 0; b < lv[l].size(); ++b) {
      const int gb = lev_off[l] + (int)b;
      if (l >= 2) {
        uint32_t px, py;
        fmm_demorton(lv[l][b].code >> 2, px, py);
        const int64_t top = ((int64_t)1 << (l - 1)) - 1;
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int64_t jx = (int64_t)px + dx, jy = (int64_t)py + dy;
            if (jx < 0 || jy < 0 || jx > top || jy > top) continue;
            const int pn = find(l - 1, fmm_morton((uint32_t)jx, (uint32_t)jy));
            if (pn < 0) continue;
            for (int q = 0; q < 4; ++q) {
              const int c = hchild[4 * (size_t)pn + q];
              if (c >= 0 && !touch(c, gb)) hvl.push_back(c);
            }
          }
      }
      hvl_off[gb + 1] = (int)hvl.size();
    }
  m2l_pairs = (int64_t)hvl.size();
  // U and W lists of every leaf by a descent from the root through the boxes
  // that touch it: touching leaves form U; a box that does not touch the
  // leaf but whose parent does, and that is smaller than the leaf, is in W
  std::vector<int> hul_off(nleaf + 1, 0), hul, hwl_off(nleaf + 1, 0), hwl;
  std::vector<std::vector<int>> xlist(nbox);
  p2p_pairs = 0;
  std::vector<int> stack;
  for (int i = 0; i < nleaf; ++i) {
    const int B = hleaf_box[i];
    stack.assign(1, 0);
    while (!stack.empty()) {
      const int c = stack.back();
      stack.pop_back();
      if (touch(c, B)) {
        if (leaf_of[c] >= 0) {
          hul.push_back(leaf_of[c]);
          p2p_pairs += (int64_t)(hi_of[B] - lo_of[B]) * (hi_of[c] - lo_of[c]);
        } else {
          for (int q = 3; q >= 0; --q)
            if (hchild[4 * (size_t)c + q] >= 0) stack.push_back(hchild[4 * (size_t)c + q]);
        }
      } else if (hlevel[c] > hlevel[B]) {
        hwl.push_back(c);
        xlist[c].push_back(i);
      }
    }
    hul_off[i + 1] = (int)hul.size();
    hwl_off[i + 1] = (int)hwl.size();
  }
  m2p_pairs = (int64_t)hwl.size();
  // X lists: the inverse of the W lists
  std::vector<int> hxbox, hxl_off(1, 0), hxl;
  for (int b = 0; b < nbox; ++b)
    if (!xlist[b].empty()) {
      hxbox.push_back(b);
      hxl.insert(hxl.end(), xlist[b].begin(), xlist[b].end());
      hxl_off.push_back((int)hxl.size());
    }
  nxbox = (int)hxbox.size();
  p2l_pairs = (int64_t)hxl.size();
  t.depth = depth;
  t.nleaf = nleaf;
  t.nbox = nbox;
  t.nxbox = nxbox;
  t.min_leaf_level = min_leaf_level;
  t.lev_off = std::move(lev_off);
  t.order = std::move(order);
  t.leaf_box = std::move(hleaf_box);
  t.leaf_start = std::move(ls);
  t.par = std::move(hpar);
  t.quad = std::move(hquad);
  t.child = std::move(hchild);
  t.level = std::move(hlevel);
  t.ctr = std::move(hctr);
  t.hb = std::move(hhb);
  t.vl_off = std::move(hvl_off);
  t.vl = std::move(hvl);
  t.ul_off = std::move(hul_off);
  t.ul = std::move(hul);
  t.wl_off = std::move(hwl_off);
  t.wl = std::move(hwl);
  t.xbox = std::move(hxbox);
  t.xl_off = std::move(hxl_off);
  t.xl = std::move(hxl);
  t.m2l_pairs = m2l_pairs;
  t.p2p_pairs = p2p_pairs;
  t.m2p_pairs = m2p_pairs;
  t.p2l_pairs = p2l_pairs;
  return t;
}

}  // namespace sbie

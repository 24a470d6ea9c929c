"""The fast multipole method's quadtree and interaction lists (host code of
the library, `csrc/fmm_tree.hpp`), checked on the CPU by a small C++ program
compiled against that header.

For uniform and adaptive trees on the pipes of the workloads, on random
and clustered points and on degenerate inputs it checks that the lists
cover every (target leaf, source leaf) pair exactly once (U direct; V at the
leaf or an ancestor; W; X at the leaf or an ancestor), that every far pair
is well separated (V: same level, not touching; W: smaller, not touching,
parent touching; X the inverse of W), that the leaves partition the nodes
in Morton order with every node inside its leaf's box, and the adaptive
split rule (a split box holds more than the target, a leaf at most the
target unless at the deepest level)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from stokes_inputs import make_geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_04484_amd", "csrc")

CHECKER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "fmm_tree.hpp"
using namespace sbie;
static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails < 20) { std::printf("FAIL %s: ", #c); std::printf(__VA_ARGS__); std::printf("\n"); } ++fails; } } while (0)
int main(int argc, char **argv) {
  FILE *f = std::fopen(argv[1], "rb");
  int64_t nn = 0;
  if (std::fread(&nn, 8, 1, f) != 1) return 2;
  std::vector<double> x(nn), y(nn);
  if (std::fread(x.data(), 8, nn, f) != (size_t)nn || std::fread(y.data(), 8, nn, f) != (size_t)nn) return 2;
  std::fclose(f);
  const int target = std::atoi(argv[2]), maxd = std::atoi(argv[3]), adaptive = std::atoi(argv[4]);
  FmmTree t = build_fmm_tree(x.data(), y.data(), nn, target, maxd, adaptive != 0);
  const int nb = t.nbox, nl = t.nleaf;
  // permutation and leaf partition
  std::vector<int> seen(nn, 0);
  for (int64_t k = 0; k < nn; ++k) seen[t.order[k]]++;
  for (int64_t i = 0; i < nn; ++i) CHECK(seen[i] == 1, "node %lld", (long long)i);
  CHECK(t.leaf_start[0] == 0 && t.leaf_start[nl] == nn, "leaf ranges");
  for (int l = 0; l < nl; ++l) CHECK(t.leaf_start[l] < t.leaf_start[l + 1], "empty leaf %d", l);
  // nodes inside their leaf box (closed, with a relative slack)
  for (int l = 0; l < nl; ++l) {
    const int b = t.leaf_box[l];
    const double h = t.hb[b] * (1.0 + 1e-9);
    for (int k = t.leaf_start[l]; k < t.leaf_start[l + 1]; ++k) {
      const int i = t.order[k];
      CHECK(std::fabs(x[i] - t.ctr[2 * b]) <= h && std::fabs(y[i] - t.ctr[2 * b + 1]) <= h, "node %d outside leaf %d", i, l);
    }
  }
  // box sizes and ancestry
  std::vector<int> leaf_of(nb, -1), cnt(nb, 0);
  for (int l = 0; l < nl; ++l) leaf_of[t.leaf_box[l]] = l;
  for (int l = 0; l < nl; ++l)
    for (int b = t.leaf_box[l]; b >= 0; b = t.par[b]) cnt[b] += t.leaf_start[l + 1] - t.leaf_start[l];
  for (int b = 0; b < nb; ++b) {
    const bool leaf = leaf_of[b] >= 0;
    bool kids = false;
    for (int q = 0; q < 4; ++q) kids |= t.child[4 * b + q] >= 0;
    CHECK(leaf != kids, "box %d leaf %d kids %d", b, (int)leaf, (int)kids);
    if (adaptive) {
      if (kids) CHECK(cnt[b] > target, "split box %d holds %d", b, cnt[b]);
      if (leaf && t.level[b] < t.depth) CHECK(cnt[b] <= target, "leaf %d holds %d", b, cnt[b]);
    } else if (leaf) {
      CHECK(t.level[b] == t.depth, "uniform leaf %d at level %d", b, t.level[b]);
    }
  }
  auto anc = [&](int b, int lev) { while (t.level[b] > lev) b = t.par[b]; return b; };
  auto touch = [&](int a, int b) {
    const double ha = t.hb[a], hb = t.hb[b];
    const double dx = std::fabs(t.ctr[2 * a] - t.ctr[2 * b]), dy = std::fabs(t.ctr[2 * a + 1] - t.ctr[2 * b + 1]);
    const double s = (ha + hb) * (1.0 + 1e-12);
    return dx <= s && dy <= s;
  };
  // separation
  for (int b = 0; b < nb; ++b)
    for (int v = t.vl_off[b]; v < t.vl_off[b + 1]; ++v) {
      const int c = t.vl[v];
      CHECK(t.level[c] == t.level[b] && t.level[b] >= 2 && !touch(b, c), "V %d-%d", b, c);
      CHECK(touch(t.par[b], t.par[c]), "V parents %d-%d", b, c);
    }
  std::vector<std::vector<int>> xinv(nb);
  for (int l = 0; l < nl; ++l) {
    const int B = t.leaf_box[l];
    for (int w = t.wl_off[l]; w < t.wl_off[l + 1]; ++w) {
      const int c = t.wl[w];
      CHECK(t.level[c] > t.level[B] && !touch(B, c) && touch(B, t.par[c]), "W %d-%d", B, c);
      xinv[c].push_back(l);
    }
  }
  {
    std::vector<std::vector<int>> xs(nb);
    for (size_t i = 0; i < t.xbox.size(); ++i)
      for (int v = t.xl_off[i]; v < t.xl_off[i + 1]; ++v) xs[t.xbox[i]].push_back(t.xl[v]);
    for (int b = 0; b < nb; ++b) CHECK(xs[b] == xinv[b], "X list of %d is not the inverse of W", b);
  }
  // coverage of every (target leaf, source leaf) pair
  std::vector<int> count(nl);
  int64_t covered = 0;
  for (int T = 0; T < nl; ++T) {
    std::fill(count.begin(), count.end(), 0);
    const int B = t.leaf_box[T];
    for (int u = t.ul_off[T]; u < t.ul_off[T + 1]; ++u) count[t.ul[u]]++;
    for (int S = 0; S < nl; ++S) {
      const int sb = t.leaf_box[S];
      for (int w = t.wl_off[T]; w < t.wl_off[T + 1]; ++w) {
        const int c = t.wl[w];
        if (t.level[sb] >= t.level[c] && anc(sb, t.level[c]) == c) count[S]++;
      }
      for (int A = B; A >= 0; A = t.par[A])
        for (int v = t.vl_off[A]; v < t.vl_off[A + 1]; ++v) {
          const int c = t.vl[v];
          if (t.level[sb] >= t.level[c] && anc(sb, t.level[c]) == c) count[S]++;
        }
    }
    for (int A = B; A >= 0; A = t.par[A])
      for (size_t i = 0; i < t.xbox.size(); ++i)
        if (t.xbox[i] == A)
          for (int v = t.xl_off[i]; v < t.xl_off[i + 1]; ++v) count[t.xl[v]]++;
    for (int S = 0; S < nl; ++S) {
      CHECK(count[S] == 1, "pair (%d, %d) covered %d times", T, S, count[S]);
      covered += count[S] == 1;
    }
  }
  std::printf("nodes %lld depth %d leaves %d boxes %d min_leaf_level %d V %lld W %lld X %lld U-pairs %lld covered %lld\n",
              (long long)nn, t.depth, nl, nb, t.min_leaf_level, (long long)t.m2l_pairs, (long long)t.m2p_pairs,
              (long long)t.p2l_pairs, (long long)t.p2p_pairs, (long long)covered);
  std::printf(fails ? "FAILED %d\n" : "OK\n", fails);
  return fails ? 1 : 0;
}
'''


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    d = tmp_path_factory.mktemp("fmmtree")
    src = d / "check.cpp"
    src.write_text(CHECKER)
    exe = d / "check"
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return d, exe


def run(checker, x, y, target, max_depth, adaptive):
    d, exe = checker
    f = d / "pts.bin"
    with open(f, "wb") as fh:
        fh.write(np.int64(len(x)).tobytes())
        fh.write(np.ascontiguousarray(x, dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(y, dtype=np.float64).tobytes())
    r = subprocess.run([str(exe), str(f), str(target), str(max_depth), str(adaptive)],
                       capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def clustered(n, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 1, size=(8, 2))
    k = rng.integers(0, 8, n)
    s = 10.0 ** rng.uniform(-4, -1, 8)
    p = c[k] + rng.standard_normal((n, 2)) * s[k][:, None]
    return p[:, 0], p[:, 1]


@pytest.mark.parametrize("adaptive", [0, 1])
@pytest.mark.parametrize("case", ["tiny", "medium", "uniform", "clustered"])
def test_lists_cover_every_pair_once(checker, case, adaptive):
    if case in ("tiny", "medium"):
        cfg = "tiny" if case == "tiny" else dict(length=10.0, n_ext=2048, n_pores=100, r_lo=0.02, r_hi=0.05,
                                                n_int=64, gap_pore=0.005, gap_wall=0.1)
        g = make_geometry(cfg, 3)
        x, y = g.x, g.y
    elif case == "uniform":
        p = np.random.default_rng(2).uniform(0, 1, size=(3000, 2))
        x, y = p[:, 0], p[:, 1]
    else:
        x, y = clustered(3000, 4)
    out = run(checker, x, y, 32 if adaptive else 48, 0, adaptive)
    if adaptive and case == "clustered":
        # strongly uneven density: leaves on several levels and W/X lists
        assert " W 0 " not in out and " X 0 " not in out


@pytest.mark.parametrize("adaptive", [0, 1])
def test_degenerate_inputs(checker, adaptive):
    # one node; two nodes; repeated positions; a straight line
    run(checker, np.array([0.3]), np.array([0.7]), 8, 0, adaptive)
    run(checker, np.array([0.0, 1.0]), np.array([0.0, 1.0]), 1, 0, adaptive)
    run(checker, np.full(50, 0.25), np.full(50, 0.5), 8, 6, adaptive)
    t = np.linspace(0, 1, 500)
    run(checker, t, 0.2 * t, 16, 0, adaptive)
    # a fixed shallow depth (no far field) and a fixed deep one
    p = np.random.default_rng(5).uniform(0, 1, size=(400, 2))
    run(checker, p[:, 0], p[:, 1], 16, 1, adaptive)
    run(checker, p[:, 0], p[:, 1], 4, 7, adaptive)

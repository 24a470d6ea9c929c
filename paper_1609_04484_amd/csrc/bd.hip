// Block-diagonal preconditioner (Section 4.1.1): the self-interaction block
// of every pore (its nodes plus its three constraint unknowns) and of the
// wall, each assembled on the device and inverted exactly.  Applying it is
// one batched block GEMV for the pores and one split-K GEMV for the wall.
#include <algorithm>

#include "assemble.hpp"
#include "batched.hpp"
#include "dense.hpp"
#include "slp.hpp"

struct sbie_bd {
  int64_t n = 0;
  int nsmall = 0;
  int max_small = 0;
  sbie::DevBuf<int64_t> idx, ioff, moff;
  sbie::DevBuf<int32_t> sz;
  sbie::DevBuf<double> mats;
  int64_t nwall = 0;
  sbie::DevBuf<int64_t> widx;
  sbie::DevBuf<double> wmat, wpart;
  int wch = 0;
  int64_t factor_bytes = 0;
};

namespace sbie {

namespace {

// In-place inverse of the wall block (n x n, column-major, ld n) by blocked
// Gauss-Jordan elimination over nb x nb pivot tiles: each tile is inverted
// with partial pivoting inside it (one workgroup), the rank-nb updates run
// on the FP64 matrix-core GEMM tiles.  There is no pivoting across tiles;
// the second-kind wall block is well conditioned and diagonally dominant in
// its tiles (the -1/2 jump).  A singular tile raises SBIE_BREAKDOWN.
void wall_inverse_tiles(double *M, int n, int nb, hipStream_t s) {
  const int npan = (n + nb - 1) / nb;
  StreamBuf<double> P((size_t)nb * nb, s), Z((size_t)nb * nb, s), C((size_t)n * nb, s), R((size_t)nb * n, s);
  StreamBuf<int32_t> info((size_t)npan, s);
  fill_value<double>(Z.p, (size_t)nb * nb, 0.0, s);
  fill_value<int>(reinterpret_cast<int *>(info.p), (size_t)npan, 0, s);
  StagerLease lease((size_t)4 << 20, s);
  Stager &st = *lease;
  for (int it = 0; it < npan; ++it) {
    const int p0 = it * nb, pb = std::min(nb, n - p0);
    double *Mpp = M + p0 + (size_t)p0 * n;
    copy_batched<double>({{Mpp, n, P.p, pb, pb, pb, 0, 0, 1.0}}, st, s);
    inverse_batched<double>({P.p}, {pb}, info.p + it, st, s);
    // C = M[:, p] with its pivot rows zeroed
    copy_batched<double>({{M + (size_t)p0 * n, n, C.p, n, n, pb, 0, 0, 1.0}}, st, s);
    copy_batched<double>({{Z.p, nb, C.p + p0, n, pb, pb, 0, 0, 1.0}}, st, s);
    // R = P M[p, :] with its pivot columns zeroed
    gemm_batched<double>({{pb, n, pb, 0, 0, P.p, pb, M + p0, n, R.p, pb, 1.0, 0.0}}, st, s);
    copy_batched<double>({{Z.p, nb, R.p + (size_t)p0 * pb, pb, pb, pb, 0, 0, 1.0}}, st, s);
    // every row outside p: M -= C R (pivot rows and columns untouched)
    gemm_batched<double>({{n, n, pb, 0, 0, C.p, n, R.p, pb, M, n, -1.0, 1.0}}, st, s);
    // pivot rows = R, pivot columns = -C P, pivot tile = P
    copy_batched<double>({{R.p, pb, M + p0, n, pb, n, 0, 0, 1.0}}, st, s);
    gemm_batched<double>({{n, pb, pb, 0, 0, C.p, n, P.p, pb, M + (size_t)p0 * n, n, -1.0, 0.0}}, st, s);
    copy_batched<double>({{P.p, pb, Mpp, n, pb, pb, 0, 0, 1.0}}, st, s);
  }
  std::vector<int32_t> h(npan);
  SBIE_HIP(hipMemcpyAsync(h.data(), info.p, npan * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  for (int it = 0; it < npan; ++it)
    if (h[it] != 0) fail(SBIE_BREAKDOWN, "wall block: singular pivot tile at row %d", it * nb);
}

}  // namespace

void bd_build(const sbie_geom *g, sbie_bd *bd, hipStream_t s) {
  const int64_t nn = g->n_nodes;
  const int m = g->n_pores;
  bd->n = n_unknowns(g);
  std::vector<int64_t> idx, ioff, moff;
  std::vector<int32_t> sz;
  int64_t mo = 0;
  for (int k = 0; k < m; ++k) {
    const int64_t a = g->curve_off[k], b = g->curve_off[k + 1];
    ioff.push_back((int64_t)idx.size());
    for (int64_t j = a; j < b; ++j) idx.push_back(j);
    for (int64_t j = a; j < b; ++j) idx.push_back(nn + j);
    for (int c = 0; c < 3; ++c) idx.push_back(2 * nn + 3 * (int64_t)k + c);
    const int32_t nb = (int32_t)(2 * (b - a) + 3);
    sz.push_back(nb);
    moff.push_back(mo);
    mo += (int64_t)nb * nb;
    if (nb > bd->max_small) bd->max_small = nb;
  }
  bd->nsmall = m;
  if (bd->max_small > 2560)
    fail(SBIE_UNSUPPORTED, "pore block of size %d exceeds 2560", bd->max_small);
  DevBuf<double> wl(1);
  wall_length(g, wl.p, s);
  const GeomView v = make_view(g, wl.p);
  if (m > 0) {
    bd->idx.alloc(idx.size());
    bd->ioff.alloc(m);
    bd->moff.alloc(m);
    bd->sz.alloc(m);
    bd->mats.alloc(mo);
    SBIE_HIP(hipMemcpyAsync(bd->idx.p, idx.data(), idx.size() * 8, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(bd->ioff.p, ioff.data(), m * 8, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(bd->moff.p, moff.data(), m * 8, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(bd->sz.p, sz.data(), m * 4, hipMemcpyHostToDevice, s));
    assemble_diag_batched(v, bd->idx.p, bd->ioff.p, bd->sz.p, bd->moff.p, m,
                          bd->max_small, bd->mats.p, s);
    DevBuf<int32_t> info(m);
    gj_inverse_batched(bd->mats.p, bd->moff.p, bd->sz.p, m, bd->max_small, info.p, s);
    std::vector<int32_t> hinfo(m);
    SBIE_HIP(hipMemcpyAsync(hinfo.data(), info.p, m * 4, hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < m; ++k)
      if (hinfo[k] != 0) fail(SBIE_BREAKDOWN, "pore block %d is singular", k);
  }
  const int64_t ws = g->curve_off[m], we = g->curve_off[m + 1];
  bd->nwall = 2 * (we - ws);
  if (bd->nwall > 0) {
    std::vector<int64_t> widx;
    for (int64_t j = ws; j < we; ++j) widx.push_back(j);
    for (int64_t j = ws; j < we; ++j) widx.push_back(nn + j);
    bd->widx.alloc(widx.size());
    SBIE_HIP(hipMemcpyAsync(bd->widx.p, widx.data(), widx.size() * 8, hipMemcpyHostToDevice, s));
    bd->wmat.alloc((size_t)bd->nwall * bd->nwall);
    assemble_block(v, bd->widx.p, bd->nwall, bd->widx.p, bd->nwall, bd->wmat.p, bd->nwall, s);
    if (bd->nwall > 8192)
      fail(SBIE_UNSUPPORTED, "wall block of order %lld exceeds 8192", (long long)bd->nwall);
    wall_inverse_tiles(bd->wmat.p, (int)bd->nwall, 128, s);
    bd->wch = (int)((bd->nwall + 255) / 256);
    if (bd->wch > 64) bd->wch = 64;
    bd->wpart.alloc((size_t)bd->wch * bd->nwall);
    SBIE_HIP(hipStreamSynchronize(s));
  }
  bd->factor_bytes = (mo + bd->nwall * bd->nwall) * 8;
}

// Block-diagonal preconditioner of the single-layer system (Section 4.1.1
// applied to the first-kind matrix): one block per curve, [sigma_x | sigma_y]
// of its nodes, assembled with the corrected rule and inverted exactly (the
// blocks are ill conditioned: on a closed curve the normal density is a near
// null vector of the single layer).
void bd_build_slp(const sbie_geom *g, sbie_bd *bd, hipStream_t s) {
  const int64_t nn = g->n_nodes;
  const int m = g->n_pores;
  bd->n = 2 * nn;
  std::vector<int64_t> idx, ioff, moff;
  std::vector<int32_t> sz;
  int64_t mo = 0;
  for (int k = 0; k < m; ++k) {
    const int64_t a = g->curve_off[k], b = g->curve_off[k + 1];
    ioff.push_back((int64_t)idx.size());
    for (int64_t j = a; j < b; ++j) idx.push_back(j);
    for (int64_t j = a; j < b; ++j) idx.push_back(nn + j);
    const int32_t nb = (int32_t)(2 * (b - a));
    sz.push_back(nb);
    moff.push_back(mo);
    mo += (int64_t)nb * nb;
    if (nb > bd->max_small) bd->max_small = nb;
  }
  bd->nsmall = m;
  if (bd->max_small > 2560)
    fail(SBIE_UNSUPPORTED, "pore block of size %d exceeds 2560", bd->max_small);
  if (m > 65535) fail(SBIE_UNSUPPORTED, "more than 65535 pores");
  if (m > 0) {
    bd->idx.alloc(idx.size());
    bd->ioff.alloc(m);
    bd->moff.alloc(m);
    bd->sz.alloc(m);
    bd->mats.alloc(mo);
    SBIE_HIP(hipMemcpyAsync(bd->idx.p, idx.data(), idx.size() * 8, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(bd->ioff.p, ioff.data(), m * 8, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(bd->moff.p, moff.data(), m * 8, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(bd->sz.p, sz.data(), m * 4, hipMemcpyHostToDevice, s));
    slp_assemble_diag_batched(g, bd->idx.p, bd->ioff.p, bd->sz.p, bd->moff.p, m, bd->max_small, bd->mats.p, s);
    DevBuf<int32_t> info(m);
    gj_inverse_batched(bd->mats.p, bd->moff.p, bd->sz.p, m, bd->max_small, info.p, s);
    std::vector<int32_t> hinfo(m);
    SBIE_HIP(hipMemcpyAsync(hinfo.data(), info.p, m * 4, hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < m; ++k)
      if (hinfo[k] != 0) fail(SBIE_BREAKDOWN, "pore block %d is singular", k);
  }
  const int64_t ws = g->curve_off[m], we = g->curve_off[m + 1];
  bd->nwall = 2 * (we - ws);
  if (bd->nwall > 0) {
    if (bd->nwall > 8192)
      fail(SBIE_UNSUPPORTED, "wall block of order %lld exceeds 8192", (long long)bd->nwall);
    std::vector<int64_t> widx;
    for (int64_t j = ws; j < we; ++j) widx.push_back(j);
    for (int64_t j = ws; j < we; ++j) widx.push_back(nn + j);
    bd->widx.alloc(widx.size());
    SBIE_HIP(hipMemcpyAsync(bd->widx.p, widx.data(), widx.size() * 8, hipMemcpyHostToDevice, s));
    bd->wmat.alloc((size_t)bd->nwall * bd->nwall);
    slp_assemble(g, bd->widx.p, bd->nwall, bd->widx.p, bd->nwall, bd->wmat.p, bd->nwall, s);
    {
      StagerLease lease((size_t)48 << 20, s);
      Stager &st = *lease;
      DevBuf<int32_t> winfo(1);
      inverse_batched_blocked<double>({bd->wmat.p}, {(int)bd->nwall}, winfo.p, st, s);
      int32_t hw = 0;
      SBIE_HIP(hipMemcpyAsync(&hw, winfo.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      SBIE_HIP(hipStreamSynchronize(s));
      if (hw != 0) fail(SBIE_BREAKDOWN, "wall block is singular (pivot %d)", (int)hw);
    }
    bd->wch = (int)((bd->nwall + 255) / 256);
    if (bd->wch > 64) bd->wch = 64;
    bd->wpart.alloc((size_t)bd->wch * bd->nwall);
    SBIE_HIP(hipStreamSynchronize(s));
  }
  bd->factor_bytes = (mo + bd->nwall * bd->nwall) * 8;
}

int64_t bd_size(const sbie_bd *bd) { return bd->n; }

void bd_apply(const sbie_bd *bd, const double *b, double *x, hipStream_t s) {
  block_gemv(bd->mats.p, bd->moff.p, bd->idx.p, bd->ioff.p, bd->sz.p, bd->nsmall,
             bd->max_small, b, x, s);
  if (bd->nwall > 0)
    big_gemv(bd->wmat.p, bd->nwall, bd->widx.p, b, x, bd->wpart.p, bd->wch, s);
}

}  // namespace sbie

extern "C" int bd_factor(const sbie_geom *g, sbie_bd **out, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!out) sbie::fail(SBIE_INVALID_ARGUMENT, "null output handle");
    *out = nullptr;
    sbie::validate_geom_device(g, (hipStream_t)stream);
    auto *bd = new sbie_bd();
    try {
      sbie::bd_build(g, bd, (hipStream_t)stream);
    } catch (...) {
      delete bd;
      throw;
    }
    *out = bd;
    return SBIE_OK;
  });
}

extern "C" int bd_factor_slp(const sbie_geom *g, sbie_bd **out, void *stream) {
  return sbie::guarded([&]() {
    sbie::validate_geom(g);
    if (!out) sbie::fail(SBIE_INVALID_ARGUMENT, "null output handle");
    *out = nullptr;
    sbie::slp_check_geom(g);
    sbie::validate_geom_device(g, (hipStream_t)stream);
    auto *bd = new sbie_bd();
    try {
      sbie::bd_build_slp(g, bd, (hipStream_t)stream);
    } catch (...) {
      delete bd;
      throw;
    }
    *out = bd;
    return SBIE_OK;
  });
}

extern "C" int bd_solve(const sbie_bd *bd, const double *b, double *x, void *stream) {
  return sbie::guarded([&]() {
    if (!bd || !b || !x) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (b < x + bd->n && x < b + bd->n) sbie::fail(SBIE_INVALID_ARGUMENT, "b and x overlap");
    sbie::bd_apply(bd, b, x, (hipStream_t)stream);
    return SBIE_OK;
  });
}

extern "C" int bd_destroy(sbie_bd *bd) {
  return sbie::guarded([&]() {
    delete bd;
    return SBIE_OK;
  });
}

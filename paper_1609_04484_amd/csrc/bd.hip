// Block-diagonal preconditioner (Section 4.1.1): the self-interaction block
// of every pore (its nodes plus its three constraint unknowns) and of the
// wall, each assembled on the device and inverted exactly.  Applying it is
// one batched block GEMV for the pores and one split-K GEMV for the wall.
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
    // blocked Gauss-Jordan with partial pivoting by columns; its rank-32
    // updates run on the FP64 matrix-core GEMM tiles (the descriptors of
    // all panel steps are staged in one transfer)
    {
      Stager st((size_t)48 << 20);
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
      Stager st((size_t)48 << 20);
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

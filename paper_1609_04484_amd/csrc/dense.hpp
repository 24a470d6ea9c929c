// Dense building blocks (batched inversion, blocked inversion, block GEMV).
#pragma once

#include "common.hpp"

namespace sbie {

struct DenseWork {
  DevBuf<double> C, R, P;
  DevBuf<int64_t> meta;
};

// In-place inverses of nmat column-major square matrices stored at
// base + off[b] with size sz[b] (device arrays); info[b] != 0 flags a
// singular pivot.
void gj_inverse_batched(double *base, const int64_t *off, const int32_t *sz,
                        int nmat, int max_n, int32_t *info, hipStream_t s);

void copy_submatrix(const double *src, int64_t ld_src, double *dst,
                    int64_t ld_dst, int64_t rows, int64_t cols, hipStream_t s,
                    int64_t zero_r0 = 0, int64_t zero_r1 = 0);

// In-place inverse of a large n x n matrix (column-major, ld n) by blocked
// Gauss-Jordan elimination without pivoting across tiles (each nb x nb
// pivot tile is inverted with pivoting).  Suitable for the well-conditioned
// second-kind wall block; a singular tile raises SBIE_BREAKDOWN.
void blocked_inverse_nopivot(double *M, int64_t n, int nb, hipStream_t s,
                             DenseWork &w);

// out[idx[r]] = sum_c M_b[r, c] v[idx[c]] for every small block b.
void block_gemv(const double *mats, const int64_t *moff_dev, const int64_t *idx,
                const int64_t *ioff_dev, const int32_t *sz_dev, int nsmall,
                int max_small, const double *v, double *out, hipStream_t s);

// Same for one large block (split over column chunks; part holds nch * n).
void big_gemv(const double *M, int64_t n, const int64_t *ix, const double *v,
              double *out, double *part, int nch, hipStream_t s);

}  // namespace sbie

// Dense building blocks of the block-diagonal preconditioner (batched
// inversion, block GEMV).
#pragma once

#include "common.hpp"

namespace sbie {

// In-place inverses of nmat column-major square matrices stored at
// base + off[b] with size sz[b] (device arrays); info[b] != 0 flags a
// singular pivot.
void gj_inverse_batched(double *base, const int64_t *off, const int32_t *sz,
                        int nmat, int max_n, int32_t *info, hipStream_t s);

// out[idx[r]] = sum_c M_b[r, c] v[idx[c]] for every small block b.
void block_gemv(const double *mats, const int64_t *moff_dev, const int64_t *idx,
                const int64_t *ioff_dev, const int32_t *sz_dev, int nsmall,
                int max_small, const double *v, double *out, hipStream_t s);

// Same for one large block (split over column chunks; part holds nch * n).
void big_gemv(const double *M, int64_t n, const int64_t *ix, const double *v,
              double *out, double *part, int nch, hipStream_t s);

}  // namespace sbie

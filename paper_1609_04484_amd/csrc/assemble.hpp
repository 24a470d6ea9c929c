// Block assembly of the operator (device), shared by the preconditioners.
#pragma once

#include "entry.hpp"

namespace sbie {

void assemble_block(const GeomView &v, const int64_t *rows, int64_t nr,
                    const int64_t *cols, int64_t nc, double *out, int64_t ld,
                    hipStream_t s);

void assemble_diag_batched(const GeomView &v, const int64_t *idx,
                           const int64_t *ioff, const int32_t *sz,
                           const int64_t *ooff, int nblocks, int max_n,
                           double *out, hipStream_t s);

}  // namespace sbie

// Single-layer (first-kind) formulation with the corrected trapezoid rule:
// matvec, block assembly and velocity (slp.hip), used by the block-diagonal
// preconditioner and the Krylov solver.
#pragma once

#include "common.hpp"

namespace sbie {

// Fails with SBIE_UNSUPPORTED when a curve has too few nodes for the
// corrected rule (at most 12).
void slp_check_geom(const sbie_geom *g);
// y = A x for the 2 Nn single-layer unknowns (accurate: compensated sums).
void slp_matvec_run(const sbie_geom *g, const double *x, double *y, bool accurate, hipStream_t s);
// A[rows, cols] (column-major, leading dimension ld); indices in [0, 2 Nn).
void slp_assemble(const sbie_geom *g, const int64_t *rows, int64_t nr, const int64_t *cols, int64_t nc,
                  double *out, int64_t ld, hipStream_t s);
// Square diagonal blocks in one launch (block b: indices idx[ioff[b] ..
// ioff[b] + sz[b]), column-major at out + ooff[b]); grid z limited to 65535.
void slp_assemble_diag_batched(const sbie_geom *g, const int64_t *idx, const int64_t *ioff, const int32_t *sz,
                               const int64_t *ooff, int nblocks, int max_n, double *out, hipStream_t s);
void slp_velocity_run(const sbie_geom *g, const double *sigma, const double *px, const double *py,
                      int64_t np, double *ux, double *uy, const double *rx, const double *ry, double *err,
                      hipStream_t s);

}  // namespace sbie

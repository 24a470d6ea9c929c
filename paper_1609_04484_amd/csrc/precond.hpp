// Preconditioner dispatch used by the Krylov solver.
#pragma once

#include "common.hpp"

namespace sbie {

void bd_apply(const sbie_bd *bd, const double *b, double *x, hipStream_t s);
int64_t bd_size(const sbie_bd *bd);
void ifmm_apply(const ifmm_handle *h, const double *b, double *x, hipStream_t s);
// Factorisation without the graph capture when defer_graph is set (see
// ifmm_capture); raises on error.
ifmm_handle *ifmm_factor_internal(const sbie_geom *g, const ifmm_params *p, hipStream_t s,
                                  bool defer_graph);
void ifmm_capture(ifmm_handle *h);

inline void precond_apply(const gmres_params *p, const double *in, double *out,
                          hipStream_t s) {
  if (p->pc == 1)
    bd_apply(p->bd, in, out, s);
  else
    ifmm_apply(p->ifmm, in, out, s);
}

}  // namespace sbie

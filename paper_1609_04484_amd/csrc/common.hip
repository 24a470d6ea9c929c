// Error plumbing and descriptor validation.
#include <cmath>
#include <mutex>

#include "common.hpp"

namespace sbie {

namespace {
thread_local std::string g_last_error;
}  // namespace

void set_last_error(const std::string &msg) { g_last_error = msg; }

void validate_geom(const sbie_geom *g) {
  if (!g) fail(SBIE_INVALID_ARGUMENT, "null geometry descriptor");
  if (g->n_nodes <= 0) fail(SBIE_INVALID_ARGUMENT, "n_nodes must be positive");
  if (g->n_pores < 0) fail(SBIE_INVALID_ARGUMENT, "n_pores must be >= 0");
  if (!g->curve_off || !g->curve_off_dev)
    fail(SBIE_INVALID_ARGUMENT, "curve offsets missing");
  if (!g->x || !g->y || !g->nx || !g->ny || !g->w || !g->kappa)
    fail(SBIE_INVALID_ARGUMENT, "node arrays missing");
  if (g->n_pores > 0 && (!g->cx || !g->cy || !g->radius))
    fail(SBIE_INVALID_ARGUMENT, "pore arrays missing");
  const int64_t *off = g->curve_off;
  if (off[0] != 0 || off[g->n_pores + 1] != g->n_nodes)
    fail(SBIE_INVALID_ARGUMENT, "curve offsets must run from 0 to n_nodes");
  for (int k = 0; k <= g->n_pores; ++k)
    if (off[k + 1] < off[k]) fail(SBIE_INVALID_ARGUMENT, "curve offsets decrease");
  for (int k = 0; k < g->n_pores; ++k)
    if (off[k + 1] - off[k] < 3)
      fail(SBIE_INVALID_GEOMETRY, "pore %d has fewer than 3 nodes", k);
}

}  // namespace sbie

extern "C" const char *sbie_last_error(void) {
  return sbie::g_last_error.c_str();
}

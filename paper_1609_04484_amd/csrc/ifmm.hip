// Inverse fast multipole method preconditioner (Section 3).
#include "precond.hpp"

struct ifmm_handle {
  int dummy;
};

namespace sbie {
void ifmm_apply(const ifmm_handle *, const double *, double *, hipStream_t) {
  fail(SBIE_UNSUPPORTED, "IFMM not available");
}
}  // namespace sbie

extern "C" int ifmm_factor(const sbie_geom *, const ifmm_params *, ifmm_handle **out, void *) {
  return sbie::guarded([&]() -> int {
    if (out) *out = nullptr;
    sbie::fail(SBIE_UNSUPPORTED, "IFMM not available");
  });
}
extern "C" int ifmm_solve(const ifmm_handle *, const double *, double *, void *) {
  return sbie::guarded([&]() -> int { sbie::fail(SBIE_UNSUPPORTED, "IFMM not available"); });
}
extern "C" int ifmm_destroy(ifmm_handle *h) { delete h; return 0; }
extern "C" int ifmm_get_stats(const ifmm_handle *, ifmm_stats *) {
  return sbie::guarded([&]() -> int { sbie::fail(SBIE_UNSUPPORTED, "IFMM not available"); });
}

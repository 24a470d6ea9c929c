// Device arithmetic shared by the pair kernels (direct double-layer and
// single-layer sums, the fast multipole method).
#pragma once

#include <hip/hip_runtime.h>

namespace sbie {

// s + c += x with the rounding error of the addition carried in c (Knuth's
// two-sum): used by the compensated modes, whose residuals must resolve
// 1e-10 of the data when the density is much larger than the data.
__device__ __forceinline__ void two_sum_acc(double &s, double &c, double x) {
#pragma clang fp contract(off)
  const double t = s + x;
  const double bp = t - s;
  c += (s - (t - bp)) + (x - bp);
  s = t;
}

// 1/d to full FP64 precision: hardware reciprocal estimate refined by one
// third-order Newton step, r' = r (1 + e + e^2) with e = 1 - d r.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

}  // namespace sbie

// olb_feq.hpp -- Hermite equilibrium factors on the device (shared by the
// stage and closure kernels).
#pragma once

#include <hip/hip_runtime.h>

#include "olb_consts.hpp"

namespace olbk {
using namespace olbc;

// Hermite equilibrium factor g_k(u, T) = W_k (1 + h_k(u, T)) (Eq. g_alpha,
// N = 4, m = 1): h = u He1 + (th + u^2)/2 He2 + (u^3 + 3 u th)/6 He3
//                 + (u^4 + 6 u^2 th + 3 th^2)/24 He4,  th = T - 1.
__device__ __forceinline__ void hfac(double u, double th, double h[5]) {
  const double u2 = u * u;
  const double c1 = u;
  const double c2 = 0.5 * (th + u2);
  const double c3 = (1.0 / 6.0) * u * (u2 + 3.0 * th);
  const double c4 = (1.0 / 24.0) * (u2 * u2 + 6.0 * u2 * th + 3.0 * th * th);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    h[k] = c1 * HE.v[1][k] + c2 * HE.v[2][k] + c3 * HE.v[3][k] + c4 * HE.v[4][k];
  }
}

}  // namespace olbk

// Transfer-function majorant of a value range: the largest TF opacity over the
// table entries [floor(x_min) - 1, ceil(x_max) + 1] of the range's table
// coordinates x = clamp((v - lo) / (hi - lo), 0, 1) (N - 1), taken in FP32.  A
// result of 0 means every value in the range has opacity exactly 0.
#pragma once

#include <hip/hip_runtime.h>

namespace dpr {

// alpha: the N table opacities (LDS or global).
__device__ __forceinline__ float tf_majorant(float2 r, const float* alpha, int ntf, float tf_lo, float tf_hi) {
  const float span = tf_hi - tf_lo;
  float ua = (r.x - tf_lo) / span;
  float ub = (r.y - tf_lo) / span;
  ua = fminf(fmaxf(ua, 0.f), 1.f);
  ub = fminf(fmaxf(ub, 0.f), 1.f);
  const float xa = ua * (float)(ntf - 1);
  const float xb = ub * (float)(ntf - 1);
  const int e0 = max((int)floorf(xa) - 1, 0);
  const int e1 = min((int)ceilf(xb) + 1, ntf - 1);
  float a = 0.f;
  for (int e = e0; e <= e1; ++e) a = fmaxf(a, alpha[e]);
  return a;
}

}  // namespace dpr

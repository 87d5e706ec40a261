// Regularization / interpolation kernels (Sec. 2.1, Fig. 1): M4' (Monaghan
// 1985) for point vortices and the smoothed three-point function (Yang et
// al. 2009) for surfaces.  Both have radius 2.
#pragma once

#include <hip/hip_runtime.h>

namespace gpf {

static __device__ __forceinline__ double m4p(double r) {
  r = fabs(r);
  if (r <= 1.0) return 1.0 - 2.5 * r * r + 1.5 * r * r * r;
  if (r <= 2.0) return 0.5 * (2.0 - r) * (2.0 - r) * (1.0 - r);
  return 0.0;
}

static __device__ __forceinline__ double yang3(double r) {
  r = fabs(r);
  const double s3 = 1.7320508075688772935;
  const double pi = 3.14159265358979323846;
  if (r <= 1.0) {
    return 17.0 / 48.0 + s3 * pi / 108.0 + r / 4.0 - r * r / 4.0 +
           (1.0 - 2.0 * r) / 16.0 * sqrt(fmax(-12.0 * r * r + 12.0 * r + 1.0, 0.0)) -
           s3 / 12.0 * asin(fmin(fmax(s3 / 2.0 * (2.0 * r - 1.0), -1.0), 1.0));
  }
  if (r <= 2.0) {
    return 55.0 / 48.0 - s3 * pi / 108.0 - 13.0 * r / 12.0 + r * r / 4.0 +
           (2.0 * r - 3.0) / 48.0 * sqrt(fmax(-12.0 * r * r + 36.0 * r - 23.0, 0.0)) +
           s3 / 36.0 * asin(fmin(fmax(s3 / 2.0 * (2.0 * r - 3.0), -1.0), 1.0));
  }
  return 0.0;
}

}  // namespace gpf

// Entries of the 1D FE matrices of eqs. (matrixK), (matrixM), evaluated on
// the fly (device and host).  Row i, column i + a with a in {-1, 0, 1};
// zero outside [0, n).  kLo/kHi are the corner entries of K times h:
// 1 - i w h on an absorbing face, 1 on a Neumann face.
#pragma once

#include <hip/hip_runtime.h>

namespace helm {

__host__ __device__ inline double m1d(int n, double h, int i, int a) {
  const int j = i + a;
  if (j < 0 || j >= n) return 0.0;
  if (a == 0) return (i == 0 || i == n - 1) ? 2.0 * h / 6.0 : 4.0 * h / 6.0;
  return h / 6.0;
}

__host__ __device__ inline double2 k1d(int n, double h, double2 kLo, double2 kHi, int i, int a) {
  const int j = i + a;
  if (j < 0 || j >= n) return make_double2(0.0, 0.0);
  if (a != 0) return make_double2(-1.0 / h, 0.0);
  if (i == 0) return make_double2(kLo.x / h, kLo.y / h);
  if (i == n - 1) return make_double2(kHi.x / h, kHi.y / h);
  return make_double2(2.0 / h, 0.0);
}

}  // namespace helm

// Workgroup-cooperative small tensor contractions (LDS or global operands).
#pragma once

#include <hip/hip_runtime.h>

namespace dgfv {

// ---------------------------------------------------------------------------
// generic workgroup contraction in LDS:
//   dst[f][..axis..] = sum_c Amat[r * C + c] * src[f][..c..]
// src dims (outer to inner) [nf][n2][n1][n0]; `axis` 0 = n0, 1 = n1, 2 = n2 has
// size C in src and R in dst.
// ---------------------------------------------------------------------------
__device__ inline void contract_axis(const double* src, double* dst, const double* Amat, int R, int C,
                              int nf, int n2, int n1, int n0, int axis) {
  int d2 = n2, d1 = n1, d0 = n0;
  if (axis == 0) d0 = R;
  else if (axis == 1) d1 = R;
  else d2 = R;
  const int total = nf * d2 * d1 * d0;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int x0 = t % d0, x1 = (t / d0) % d1, x2 = (t / (d0 * d1)) % d2, f = t / (d0 * d1 * d2);
    const double* s = src + (size_t)f * n2 * n1 * n0;
    double acc = 0.0;
    if (axis == 0) {
      const double* a = Amat + x0 * C;
      const double* sp = s + (x2 * n1 + x1) * n0;
      for (int c = 0; c < C; ++c) acc += a[c] * sp[c];
    } else if (axis == 1) {
      const double* a = Amat + x1 * C;
      const double* sp = s + x2 * n1 * n0 + x0;
      for (int c = 0; c < C; ++c) acc += a[c] * sp[c * n0];
    } else {
      const double* a = Amat + x2 * C;
      const double* sp = s + x1 * n0 + x0;
      for (int c = 0; c < C; ++c) acc += a[c] * sp[c * n1 * n0];
    }
    dst[t] = acc;
  }
}


}  // namespace dgfv

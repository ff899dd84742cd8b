// Per-node FP64 weighted least-squares solve of the local-linear fit
// (eqs. 2.3 / 2.4), shared by the smoother kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "fpca.h"

namespace fpca {

// Solve [[S0, S1^T], [S1, S2]] beta = [T0; T1] in FP64 for b0 = beta_0 by an
// L D L^T factorization (unit lower L, no square roots, one reciprocal per
// pivot). Status:
//   EMPTY    S0 <= 0: b0 = NaN;
//   FALLBACK a diagonal entry A_jj <= 0, or a pivot D_j < 1e-10 A_jj -- the
//            same test as a Cholesky pivot below 1e-10 of the Jacobi-scaled
//            (unit-diagonal) matrix, whose pivots are D_j / A_jj: b0 = T0/S0;
//   OK       otherwise.
// `m` holds the moments in the order S0, S1[D], S2 (upper triangle, row by
// row), T0, T1[D].
template <int D>
__device__ inline double wls_b0(const double *m, int8_t *st) {
  constexpr int n = D + 1;
  double A[n][n], r[n];
  const double S0 = m[0];
  const double T0 = m[1 + D + D * (D + 1) / 2];
  if (!(S0 > 0.0)) {
    *st = FPCA_STATUS_EMPTY;
    return __builtin_nan("");
  }
  A[0][0] = S0;
  r[0] = T0;
  int q = 1 + D;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    A[1 + k][0] = m[1 + k];
    r[1 + k] = m[2 + D + D * (D + 1) / 2 + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int l = k; l < D; ++l) A[1 + l][1 + k] = m[q++];  // lower triangle
  const double fb = T0 / S0;
  bool ok = true;
#pragma unroll
  for (int i = 1; i < n; ++i) ok = ok && (A[i][i] > 0.0);
  // In place: strictly lower A becomes L, the diagonal becomes D; W = L D.
  double invd[n];
#pragma unroll
  for (int j = 0; j < n; ++j) {
    double dj = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= A[j][k] * (A[j][k] * A[k][k]);
    ok = ok && (dj >= 1e-10 * A[j][j]);
    const double inv = 1.0 / dj;
    invd[j] = inv;
#pragma unroll
    for (int i = j + 1; i < n; ++i) {
      double v = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= A[i][k] * (A[j][k] * A[k][k]);
      A[i][j] = v * inv;
    }
    A[j][j] = dj;
  }
  if (!ok) {
    *st = FPCA_STATUS_FALLBACK;
    return fb;
  }
  // L z = r; y = D^-1 z; L^T x = y
#pragma unroll
  for (int i = 0; i < n; ++i) {
#pragma unroll
    for (int k = 0; k < i; ++k) r[i] -= A[i][k] * r[k];
  }
#pragma unroll
  for (int i = 0; i < n; ++i) r[i] *= invd[i];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) {
#pragma unroll
    for (int k = i + 1; k < n; ++k) r[i] -= A[k][i] * r[k];
  }
  *st = FPCA_STATUS_OK;
  return r[0];
}

}  // namespace fpca

// Per-node FP64 weighted least-squares solve of the local-linear fit
// (eqs. 2.3 / 2.4), shared by the smoother kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "fpca.h"

namespace fpca {

// Solve [[S0, S1^T], [S1, S2]] beta = [T0; T1] in FP64 for b0 = beta_0.
// Status: EMPTY if S0 <= 0 (b0 = NaN); FALLBACK (b0 = T0/S0) if a diagonal
// entry is not positive or the Cholesky factorization of the Jacobi-scaled
// (unit-diagonal) matrix meets a pivot that is not positive or below 1e-10;
// OK otherwise. `m` holds the moments in the order S0, S1[D], S2 (upper
// triangle, row by row), T0, T1[D].
template <int D>
__device__ inline double wls_b0(const double *m, int8_t *st) {
  constexpr int n = D + 1;
  double A[n][n], r[n], sc[n];
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
    A[0][1 + k] = A[1 + k][0] = m[1 + k];
    r[1 + k] = m[2 + D + D * (D + 1) / 2 + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int l = k; l < D; ++l) {
      A[1 + k][1 + l] = A[1 + l][1 + k] = m[q++];
    }
  const double fb = T0 / S0;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    if (!(A[i][i] > 0.0)) {
      *st = FPCA_STATUS_FALLBACK;
      return fb;
    }
    sc[i] = 1.0 / sqrt(A[i][i]);
  }
#pragma unroll
  for (int i = 0; i < n; ++i) {
    r[i] *= sc[i];
#pragma unroll
    for (int j = 0; j < n; ++j) A[i][j] *= sc[i] * sc[j];
  }
  // In-place Cholesky: lower triangle of A becomes L.
#pragma unroll
  for (int j = 0; j < n; ++j) {
    double dj = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= A[j][k] * A[j][k];
    if (!(dj >= 1e-10)) {
      *st = FPCA_STATUS_FALLBACK;
      return fb;
    }
    const double ljj = sqrt(dj);
    A[j][j] = ljj;
    const double inv = 1.0 / ljj;
#pragma unroll
    for (int i = j + 1; i < n; ++i) {
      double v = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
      A[i][j] = v * inv;
    }
  }
  double z[n];
#pragma unroll
  for (int i = 0; i < n; ++i) {
    double v = r[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= A[i][k] * z[k];
    z[i] = v / A[i][i];
  }
  double x0 = 0.0;
#pragma unroll
  for (int i = n - 1; i >= 0; --i) {
    double v = z[i];
#pragma unroll
    for (int k = i + 1; k < n; ++k) v -= A[k][i] * r[k];
    r[i] = v / A[i][i];  // reuse r as the solution
    if (i == 0) x0 = r[0];
  }
  *st = FPCA_STATUS_OK;
  return x0 * sc[0];
}

}  // namespace fpca

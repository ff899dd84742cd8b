// Internal view of the covariance operator (covop.hip); eig.hip drives it.
#pragma once

#include "common.hpp"

struct fpca_covop_s {
  fpca_context *ctx = nullptr;
  int d = 0;
  int M[3] = {1, 1, 1};
  int R[3] = {0, 0, 0};
  double H[3] = {1, 1, 1};
  int64_t P = 0;
  int64_t n = 0;
  int mode = 0;
  // device data, all FP64, owned by the operator
  double *Zn = nullptr;  // P x (d+1) x n: curves filtered by K, K u_0, .., K u_{d-1}
  double *Ln = nullptr;  // P x n: local-linear smooth of each curve
  double *Bn = nullptr;  // P x n: the boundary part of Ln (zero in the interior)
  double *Y2 = nullptr;  // P: sum over curves of Y^2
  double *mu = nullptr;  // P: the mean
  double *tab = nullptr;  // per coordinate: taps K, u; window sums W; shared-node sums E
  int64_t tab_K[3] = {0, 0, 0}, tab_U[3] = {0, 0, 0}, tab_W[3] = {0, 0, 0}, tab_E[3] = {0, 0, 0};
  double *band = nullptr;  // stored band blocks (mode FPCA_COVOP_STORE_BAND)
  double *lr_part = nullptr;  // partial products of the low-rank apply
  double *lr_tot = nullptr;
  int64_t lr_blocks = 0;
  int tb[3] = {1, 1, 1};    // tile extents
  int nt[3] = {1, 1, 1};    // tiles per coordinate
  int span[3] = {0, 0, 0};  // band reach in tiles
  int64_t n_stiles = 0;
  int nslot = 1;
  size_t band_lds = 0, apply_lds = 0;
};

namespace fpca {
// out = Gamma_hat X for X, out: P x r row-major (r <= 64), on the handle's stream.
int covop_apply_internal(fpca_covop_s *op, int r, const double *X, double *out);
}  // namespace fpca

// The linear-binning rule of Section 3.2 on the device: lower corner and
// fractions of an observation point, and its 2^d multilinear corner weights.
// Shared by the binning kernels and by interpolation from the grid.
#pragma once

#include <cmath>

#include "common.hpp"

namespace fpca {
namespace {

// Lower corner and fractions of one observation; false if any coordinate is
// outside [0,1] or NaN. u = x*(M-1) is one rounded FP64 multiply (exact for
// FP32 inputs), never fused with the subtraction that follows.
template <typename T>
__device__ inline bool locate(const T *x, const GridDims &g, int *k, double *rho) {
#pragma clang fp contract(off)
  for (int q = 0; q < g.d; ++q) {
    double xv = double(x[q]);
    if (!(xv >= 0.0 && xv <= 1.0)) return false;
    double u = xv * double(g.M[q] - 1);
    int kq = int(floor(u));
    if (kq > g.M[q] - 2) kq = g.M[q] - 2;
    k[q] = kq;
    rho[q] = u - double(kq);
  }
  return true;
}

__device__ inline void corner(const GridDims &g, const int *k, const double *rho, int c, int64_t *p,
                              double *W) {
  int64_t pp = 0;
  double w = 1.0;
  for (int q = 0; q < g.d; ++q) {
    int bit = (c >> (g.d - 1 - q)) & 1;
    pp += int64_t(k[q] + bit) * g.stride[q];
    w *= bit ? rho[q] : (1.0 - rho[q]);
  }
  *p = pp;
  *W = w;
}

}  // namespace
}  // namespace fpca

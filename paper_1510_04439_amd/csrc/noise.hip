// Noise variance (eq. 2.6) from the smoothed second moment of the responses
// (eq. 2.5). At each grid node t:
//   sigma2(t) = b0(t) - Gamma(t, t) - mu(t)^2,
// with b0 the local-linear smooth of the binned squares Y_ij^2 under the
// mean's curve weights 1/N_i (eq. 2.5), Gamma the assembled covariance and mu
// the smoothed mean. b0 estimates E Y^2 = mu^2 + Gamma(t, t) + sigma^2, so the
// square of the mean is subtracted (the paper prints the product with a plus
// sign). The constant sigma^2 is the integral over Omega divided by the volume
// of Omega, taken as the average of sigma2(t) over the grid nodes of Omega at
// which it is finite.
#include "common.hpp"

namespace fpca {

namespace {

constexpr int NV_THREADS = 1024;

// One workgroup: per-node values, then an FP64 sum and count in a fixed order
// (strided per thread, then the waves of the workgroup in index order).
template <typename T>
__global__ __launch_bounds__(NV_THREADS) void k_noise_variance(int64_t P, const T *__restrict__ b0,
                                                               const T *__restrict__ mu,
                                                               const T *__restrict__ gamma,
                                                               const uint8_t *__restrict__ mask, T *s2t,
                                                               double *out) {
  __shared__ double ps[NV_THREADS / 64], pc[NV_THREADS / 64];
  double sum = 0.0, cnt = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += NV_THREADS) {
    double v = 0.0;
    if (!mask || mask[p]) {
      const double m = double(mu[p]);
      v = (double(b0[p]) - double(gamma[p * P + p])) - m * m;
      if (isfinite(v)) {
        sum += v;
        cnt += 1.0;
      }
    }
    if (s2t) s2t[p] = T(v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o);
    cnt += __shfl_xor(cnt, o);
  }
  if ((threadIdx.x & 63) == 0) {
    ps[threadIdx.x >> 6] = sum;
    pc[threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, c = 0.0;
    for (int w = 0; w < NV_THREADS / 64; ++w) {
      s += ps[w];
      c += pc[w];
    }
    out[0] = c > 0.0 ? s / c : __builtin_nan("");
    out[1] = c;
  }
}

template <typename T>
int noise_variance_impl(fpca_context *ctx, const fpca_grid *grid, int64_t P, const T *b0, const T *mu,
                        const T *gamma, T *s2t, double *sigma2, int64_t *count) {
  if (int rc = ws_reserve(ctx, 256)) return rc;
  double *out = static_cast<double *>(ctx->ws);
  hipLaunchKernelGGL(k_noise_variance<T>, dim3(1), dim3(NV_THREADS), 0, ctx->stream, P, b0, mu, gamma, grid->mask,
                     s2t, out);
  FPCA_LAUNCH_CHECK("noise_variance");
  double *hb = ctx->h_stage;
  FPCA_HIP(hipMemcpyAsync(hb, out, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  *sigma2 = hb[0];
  if (count) *count = int64_t(hb[1]);
  return FPCA_OK;
}

}  // namespace

}  // namespace fpca

using namespace fpca;

extern "C" int fpca_noise_variance(fpca_handle ctx, const fpca_grid *grid, int dtype, const void *b0, const void *mu,
                                   const void *gamma, void *sigma2_t, double *sigma2, int64_t *count) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (!b0 || !mu || !gamma || !sigma2) return set_error(FPCA_ERR_INVALID_ARG, "b0, mu, gamma and sigma2 are required");
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return noise_variance_impl<double>(ctx, grid, P, static_cast<const double *>(b0), static_cast<const double *>(mu),
                                       static_cast<const double *>(gamma), static_cast<double *>(sigma2_t), sigma2,
                                       count);
  return noise_variance_impl<float>(ctx, grid, P, static_cast<const float *>(b0), static_cast<const float *>(mu),
                                    static_cast<const float *>(gamma), static_cast<float *>(sigma2_t), sigma2, count);
}

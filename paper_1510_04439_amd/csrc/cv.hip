// Batched cross-validation of the covariance bandwidth over bandwidths and
// leave-curves-out folds (a binned reading of the CV criterion of Section 3.3).
//
// For fold f the smoother sees the pairs of the other curves, C - C_f and
// G - G_f (slab 0 minus slab f+1 of fpca_bin with folds), giving Ghat_{-f,h};
// the held-out pairs of fold f are scored against it through their bins:
//   CV_f(h) = sum_{p,q} [ Q_f - 2 G_f Ghat + C_f Ghat^2 ],
// i.e. sum over held-out pairs of w (Y_ij Y_il - Ghat(bin))^2 spread over the
// pair's bins by the binning weights (Ghat = 0 where the window is empty).
#include <cmath>
#include <vector>

#include "common.hpp"

namespace fpca {
namespace {

constexpr int SCORE_BLOCKS = 512;

template <typename T>
__global__ void k_fold_diff(int64_t n, const T *__restrict__ C0, const T *__restrict__ Cf, const T *__restrict__ G0,
                            const T *__restrict__ Gf, T *__restrict__ W, T *__restrict__ S) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (; e < n; e += step) {
    W[e] = C0[e] - Cf[e];
    S[e] = G0[e] - Gf[e];
  }
}

// Per-block FP64 partial sums of Q - 2 G g + C g^2 (g = 0 where NaN), fixed
// grid for a deterministic order.
template <typename T>
__global__ __launch_bounds__(256) void k_cv_score(int64_t n, const T *__restrict__ Qf, const T *__restrict__ Gf,
                                                   const T *__restrict__ Cf, const T *__restrict__ Gh,
                                                   double *__restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    double g = double(Gh[e]);
    if (g != g) g = 0.0;
    s += double(Qf[e]) - 2.0 * double(Gf[e]) * g + double(Cf[e]) * g * g;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_cv_finish(int njobs, const double *__restrict__ part, double *__restrict__ scores) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  double s = 0.0;
  for (int b = 0; b < SCORE_BLOCKS; ++b) s += part[int64_t(j) * SCORE_BLOCKS + b];
  scores[j] = s;
}

template <typename T>
int cv_impl(fpca_context *ctx, const fpca_grid *grid, int dtype, int n_folds, const T *C, const T *G, const T *Q,
            int n_h, const double *bw, double *scores_h) {
  const GridDims gd = make_dims(grid);
  const int64_t P = gd.P, PP = P * P;
  const int njobs = n_h * n_folds;
  const int64_t nin = (int64_t(n_folds) + 1) * PP;
  const size_t need = 3 * carve_bytes(nin, sizeof(T)) + 3 * carve_bytes(PP, sizeof(T)) +
                      carve_bytes(size_t(njobs) * SCORE_BLOCKS, 8) + carve_bytes(njobs, 8);
  if (int rc = ws3_reserve(ctx, need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws3), 0, ctx->ws3_size};
  // inputs are staged into the handle's buffers, so a captured graph depends
  // only on the shape and not on the caller's pointers
  T *Cs = cv.take<T>(nin);
  T *Gs = cv.take<T>(nin);
  T *Qs = cv.take<T>(nin);
  T *W = cv.take<T>(PP);
  T *S = cv.take<T>(PP);
  T *Gh = cv.take<T>(PP);
  double *part = cv.take<double>(size_t(njobs) * SCORE_BLOCKS);
  double *sc = cv.take<double>(njobs);
  FPCA_HIP(hipMemcpyAsync(Cs, C, sizeof(T) * nin, hipMemcpyDeviceToDevice, ctx->stream));
  FPCA_HIP(hipMemcpyAsync(Gs, G, sizeof(T) * nin, hipMemcpyDeviceToDevice, ctx->stream));
  FPCA_HIP(hipMemcpyAsync(Qs, Q, sizeof(T) * nin, hipMemcpyDeviceToDevice, ctx->stream));
  int64_t blocks = (PP + 255) / 256;
  if (blocks > 65536) blocks = 65536;

  auto queue_jobs = [&]() -> int {
    for (int f = 0; f < n_folds; ++f) {
      const int64_t o = (int64_t(f) + 1) * PP;
      hipLaunchKernelGGL(k_fold_diff<T>, dim3(unsigned(blocks)), dim3(256), 0, ctx->stream, PP, Cs, Cs + o, Gs,
                         Gs + o, W, S);
      FPCA_LAUNCH_CHECK("fold_diff");
      for (int hi = 0; hi < n_h; ++hi) {
        if (int rc = smooth_cov_internal(ctx, grid, dtype, W, 0.0, S, nullptr, bw + int64_t(hi) * grid->d, Gh,
                                         nullptr))
          return rc;
        const int job = hi * n_folds + f;
        hipLaunchKernelGGL(k_cv_score<T>, dim3(SCORE_BLOCKS), dim3(256), 0, ctx->stream, PP, Qs + o, Gs + o, Cs + o,
                           Gh, part + int64_t(job) * SCORE_BLOCKS);
        FPCA_LAUNCH_CHECK("cv_score");
      }
    }
    return FPCA_OK;
  };
  // The job sequence is captured into a graph on its second call with the
  // same shape and scratch layout (the first, eager call sizes every scratch
  // buffer, so capture performs no allocation) and replayed afterwards.
  auto make_key = [&]() {
    std::vector<double> k = {double(dtype), double(grid->d), double(n_folds), double(n_h),
                             double(reinterpret_cast<uintptr_t>(grid->mask)),
                             double(reinterpret_cast<uintptr_t>(ctx->ws)), double(ctx->ws_size),
                             double(reinterpret_cast<uintptr_t>(ctx->ws3)), double(ctx->ws3_size)};
    for (int q = 0; q < grid->d; ++q) k.push_back(double(grid->M[q]));
    for (int i = 0; i < n_h * grid->d; ++i) k.push_back(bw[i]);
    return k;
  };
  const std::vector<double> key = make_key();
  const bool same = (key == ctx->cv_key);
  if (same && ctx->cv_exec) {
    FPCA_HIP(hipEventRecord(ctx->ev_a, ctx->stream));
    FPCA_HIP(hipStreamWaitEvent(ctx->cap_stream, ctx->ev_a, 0));
    FPCA_HIP(hipGraphLaunch(ctx->cv_exec, ctx->cap_stream));
    FPCA_HIP(hipEventRecord(ctx->ev_b, ctx->cap_stream));
    FPCA_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_b, 0));
  } else if (same && ctx->cv_key_seen >= 1) {
    if (!ctx->cap_stream) {
      FPCA_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      FPCA_HIP(hipEventCreateWithFlags(&ctx->ev_a, hipEventDisableTiming));
      FPCA_HIP(hipEventCreateWithFlags(&ctx->ev_b, hipEventDisableTiming));
    }
    FPCA_HIP(hipEventRecord(ctx->ev_a, ctx->stream));
    FPCA_HIP(hipStreamWaitEvent(ctx->cap_stream, ctx->ev_a, 0));
    hipStream_t user = ctx->stream;
    FPCA_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
    ctx->stream = ctx->cap_stream;
    const int rc = queue_jobs();
    ctx->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc != FPCA_OK || ec != hipSuccess || make_key() != key) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      ctx->cv_key.clear();
      ctx->cv_key_seen = 0;
      if (rc != FPCA_OK) return rc;
      return set_error(FPCA_ERR_DEVICE, "batched CV graph capture failed");
    }
    if (ctx->cv_exec) (void)hipGraphExecDestroy(ctx->cv_exec);
    ctx->cv_exec = nullptr;
    FPCA_HIP(hipGraphInstantiate(&ctx->cv_exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    FPCA_HIP(hipGraphLaunch(ctx->cv_exec, ctx->cap_stream));
    FPCA_HIP(hipEventRecord(ctx->ev_b, ctx->cap_stream));
    FPCA_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_b, 0));
  } else {
    if (int rc = queue_jobs()) return rc;
    if (ctx->cv_exec) (void)hipGraphExecDestroy(ctx->cv_exec);
    ctx->cv_exec = nullptr;
    ctx->cv_key = make_key();  // after the run: the scratch it sized
    ctx->cv_key_seen = 1;
  }
  hipLaunchKernelGGL(k_cv_finish, dim3((njobs + 63) / 64), dim3(64), 0, ctx->stream, njobs, part, sc);
  FPCA_LAUNCH_CHECK("cv_finish");
  FPCA_HIP(hipMemcpyAsync(scores_h, sc, sizeof(double) * njobs, hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  return FPCA_OK;
}

}  // namespace
}  // namespace fpca

using namespace fpca;

extern "C" int fpca_cv_batched(fpca_handle ctx, const fpca_grid *grid, int dtype, int n_folds, const void *C,
                               const void *G, const void *Q, int n_h, const double *bandwidths, double *scores) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (n_folds < 1 || n_h < 1) return set_error(FPCA_ERR_INVALID_ARG, "need n_folds >= 1 and n_h >= 1");
  if (!C || !G || !Q || !bandwidths || !scores)
    return set_error(FPCA_ERR_INVALID_ARG, "C, G, Q, bandwidths and scores are required");
  if (P > (int64_t(1) << 15)) return set_error(FPCA_ERR_UNSUPPORTED, "covariance grid too large (P=%lld)", (long long)P);
  for (int i = 0; i < n_h * grid->d; ++i)
    if (!(bandwidths[i] > 0.0) || !std::isfinite(bandwidths[i]))
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidths must be positive and finite");
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return cv_impl<double>(ctx, grid, dtype, n_folds, static_cast<const double *>(C), static_cast<const double *>(G),
                           static_cast<const double *>(Q), n_h, bandwidths, scores);
  return cv_impl<float>(ctx, grid, dtype, n_folds, static_cast<const float *>(C), static_cast<const float *>(G),
                        static_cast<const float *>(Q), n_h, bandwidths, scores);
}

// Batched cross-validation of the covariance bandwidth over datasets,
// bandwidths and leave-curves-out folds (a binned reading of the CV criterion
// of Section 3.3).
//
// For fold f the smoother sees the pairs of the other curves, C - C_f and
// G - G_f (slab 0 minus slab f+1 of fpca_bin with folds), giving Ghat_{-f,h};
// the held-out pairs of fold f are scored against it through their bins:
//   CV_f(h) = sum_{p,q} [ Q_f - 2 G_f Ghat + C_f Ghat^2 ],
// i.e. sum over held-out pairs of w (Y_ij Y_il - Ghat(bin))^2 spread over the
// pair's bins by the binning weights (Ghat = 0 where the window is empty).
//
// Every (dataset, bandwidth, fold) job of a call runs in one persistent launch
// of the task-queue smoother (smooth_tiled.hip). Its tile shape (t-columns per
// task) and the number of persistent workgroups per compute unit are chosen
// per shape by timing the candidates that fit in LDS on the first call (with
// the job-by-job general pass engine as one more candidate); the
// second call with the same shape captures the launch into a HIP graph, later
// calls replay it (the job table, which holds the callers' pointers, is
// uploaded before each launch, outside the graph). Grids the queue smoother
// does not take run job by job through the general pass engine.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "tiled.hpp"

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

int64_t grid_P(const fpca_grid &g) {
  int64_t P = 1;
  for (int k = 0; k < g.d; ++k) P *= g.M[k];
  return P;
}

// Job by job through the general pass engine (grids the queue smoother does
// not take); scores of dataset `a` land in scores_h[(hi * n_folds + f)].
template <typename T>
int cv_general(fpca_context *ctx, const fpca_cv_data &ds, int dtype, int n_folds, int n_h, const double *bw,
               double *scores_h) {
  const fpca_grid *grid = &ds.grid;
  const int64_t P = grid_P(*grid), PP = P * P;
  const int njobs = n_h * n_folds;
  const T *C = static_cast<const T *>(ds.C);
  const T *G = static_cast<const T *>(ds.G);
  const T *Q = static_cast<const T *>(ds.Q);
  const size_t need = 3 * carve_bytes(PP, sizeof(T)) + carve_bytes(size_t(njobs) * SCORE_BLOCKS, 8) +
                      carve_bytes(njobs, 8);
  if (int rc = ws3_reserve(ctx, need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws3), 0, ctx->ws3_size};
  T *W = cv.take<T>(PP);
  T *S = cv.take<T>(PP);
  T *Gh = cv.take<T>(PP);
  double *part = cv.take<double>(size_t(njobs) * SCORE_BLOCKS);
  double *sc = cv.take<double>(njobs);
  int64_t blocks = (PP + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  for (int f = 0; f < n_folds; ++f) {
    const int64_t o = (int64_t(f) + 1) * PP;
    hipLaunchKernelGGL(k_fold_diff<T>, dim3(unsigned(blocks)), dim3(256), 0, ctx->stream, PP, C, C + o, G, G + o, W,
                       S);
    FPCA_LAUNCH_CHECK("fold_diff");
    for (int hi = 0; hi < n_h; ++hi) {
      if (int rc = smooth_cov_internal(ctx, grid, dtype, W, 0.0, S, nullptr, bw + int64_t(hi) * grid->d, Gh, nullptr))
        return rc;
      const int job = hi * n_folds + f;
      hipLaunchKernelGGL(k_cv_score<T>, dim3(SCORE_BLOCKS), dim3(256), 0, ctx->stream, PP, Q + o, G + o, C + o, Gh,
                         part + int64_t(job) * SCORE_BLOCKS);
      FPCA_LAUNCH_CHECK("cv_score");
    }
  }
  hipLaunchKernelGGL(k_cv_finish, dim3((njobs + 63) / 64), dim3(64), 0, ctx->stream, njobs, part, sc);
  FPCA_LAUNCH_CHECK("cv_finish");
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  FPCA_HIP(hipMemcpy(scores_h, sc, sizeof(double) * njobs, hipMemcpyDeviceToHost));
  return FPCA_OK;
}

// Waits for the stream and turns a stalled queue wait into an error.
int finish_and_check(fpca_context *ctx) {
  FPCA_HIP(hipMemcpyAsync(ctx->h_flags, ctx->d_flags, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  if (*ctx->h_flags & 2) {
    const int keep = *ctx->h_flags & ~2;
    *ctx->h_flags = 0;
    FPCA_HIP(hipMemcpy(ctx->d_flags, &keep, sizeof(int), hipMemcpyHostToDevice));
    return set_error(FPCA_ERR_DEVICE, "batched CV: a task waited past its spin limit");
  }
  return FPCA_OK;
}

template <typename T>
int cv_impl(fpca_context *ctx, int dtype, int n_data, const fpca_cv_data *data, int n_folds, int n_h,
            const double *bw, double *scores_h) {
  const int d = data[0].grid.d;
  bool all_tiled = ctx->engine != FPCA_ENGINE_PASSES;
  for (int a = 0; a < n_data; ++a) all_tiled = all_tiled && tiled_supported(&data[a].grid);
  if (!all_tiled) {
    for (int a = 0; a < n_data; ++a)
      if (int rc = cv_general<T>(ctx, data[a], dtype, n_folds, n_h, bw, scores_h + int64_t(a) * n_h * n_folds))
        return rc;
    return FPCA_OK;
  }
  // jobs: dataset-major, then bandwidth, then fold (the order of `scores`)
  std::vector<TiledJob> jobs;
  jobs.reserve(size_t(n_data) * n_h * n_folds);
  for (int a = 0; a < n_data; ++a) {
    const int64_t PP = grid_P(data[a].grid) * grid_P(data[a].grid);
    const T *C = static_cast<const T *>(data[a].C);
    const T *G = static_cast<const T *>(data[a].G);
    const T *Q = static_cast<const T *>(data[a].Q);
    for (int hi = 0; hi < n_h; ++hi)
      for (int f = 0; f < n_folds; ++f) {
        const int64_t o = (int64_t(f) + 1) * PP;
        TiledJob j{};
        j.grid = &data[a].grid;
        j.Ca = C;
        j.Cb = C + o;
        j.Ga = G;
        j.Gb = G + o;
        j.Qf = Q + o;
        j.Gf = G + o;
        j.Cf = C + o;
        j.h = bw + int64_t(hi) * d;
        jobs.push_back(j);
      }
  }
  const int J = int(jobs.size());
  // shape key: everything a launch depends on except the callers' pointers
  std::vector<double> shape = {double(dtype), double(d), double(n_data), double(n_folds), double(n_h)};
  for (int a = 0; a < n_data; ++a) {
    for (int k = 0; k < d; ++k) shape.push_back(double(data[a].grid.M[k]));
    shape.push_back(data[a].grid.mask ? 1.0 : 0.0);
  }
  for (int i = 0; i < n_h * d; ++i) shape.push_back(bw[i]);
  // autotune once per shape: every (qb, workgroups per CU) whose LDS fits,
  // timed over the whole launch
  TiledConfig cfg;
  bool tuned = false;
  for (const auto &e : ctx->tune_cache)
    if (e.first == shape) {
      cfg.qb = e.second.first;
      cfg.wg_per_cu = e.second.second;
      tuned = true;
    }
  // qb = 0 stands for the job-by-job general pass engine (small grids whose
  // FP64 intermediates stay in the caches can run faster that way)
  auto run_general = [&]() -> int {
    for (int a = 0; a < n_data; ++a)
      if (int rc = cv_general<T>(ctx, data[a], dtype, n_folds, n_h, bw, scores_h + int64_t(a) * n_h * n_folds))
        return rc;
    return FPCA_OK;
  };
  if (!tuned) {
    hipEvent_t e0, e1;
    FPCA_HIP(hipEventCreate(&e0));
    FPCA_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    // the job-by-job engine is a candidate when one job's FP64 moment arrays
    // (1 + D + D(D+1)/2 + 1 + D of them) fit in the 256 MB Infinity Cache;
    // its first run sizes its scratch, the second is timed
    size_t foot = 0;
    for (int a = 0; a < n_data; ++a) {
      const int64_t PP = grid_P(data[a].grid) * grid_P(data[a].grid);
      const int D = 2 * d;
      foot = std::max(foot, size_t(PP) * 8 * size_t(2 + 2 * D + D * (D + 1) / 2));
    }
    if (ctx->engine == FPCA_ENGINE_AUTO && foot <= (size_t(256) << 20)) {
      int rc = run_general();
      if (rc == FPCA_OK) rc = hipEventRecord(e0, ctx->stream) == hipSuccess ? FPCA_OK : FPCA_ERR_DEVICE;
      if (rc == FPCA_OK) rc = run_general();
      if (rc == FPCA_OK) rc = hipEventRecord(e1, ctx->stream) == hipSuccess ? FPCA_OK : FPCA_ERR_DEVICE;
      if (rc == FPCA_OK) rc = hipEventSynchronize(e1) == hipSuccess ? FPCA_OK : FPCA_ERR_DEVICE;
      if (rc != FPCA_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc == FPCA_ERR_DEVICE ? set_error(rc, "batched CV: timing the job-by-job engine failed") : rc;
      }
      FPCA_HIP(hipEventElapsedTime(&best, e0, e1));
      cfg.qb = 0;
      cfg.wg_per_cu = 0;
    }
    for (int qb : {8, 16}) {
      const size_t lds = tiled_lds(jobs, qb);
      if (!lds) continue;
      for (int wg : {1, 2, 3, 4}) {
        if ((lds + 256) * wg > 160 * 1024) continue;
        TiledConfig c;
        c.qb = qb;
        c.wg_per_cu = wg;
        TiledLaunch L;
        int rc = tiled_plan<T>(ctx, jobs, true, c, &L);
        if (rc == FPCA_OK) FPCA_HIP(hipEventRecord(e0, ctx->stream));
        if (rc == FPCA_OK) rc = tiled_queue(ctx, L);
        if (rc == FPCA_OK) FPCA_HIP(hipEventRecord(e1, ctx->stream));
        if (rc == FPCA_OK) rc = finish_and_check(ctx);
        if (rc != FPCA_OK) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return rc;
        }
        float ms = 0.f;
        FPCA_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          cfg = c;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best >= 1e30f) return set_error(FPCA_ERR_UNSUPPORTED, "batched CV: no tile shape fits in LDS");
    ctx->tune_cache.push_back({shape, {cfg.qb, cfg.wg_per_cu}});
  }
  if (cfg.qb == 0) return run_general();
  TiledLaunch L;
  if (int rc = tiled_plan<T>(ctx, jobs, true, cfg, &L)) return rc;
  // graph key: the shape, the chosen configuration and the scratch layout
  std::vector<double> key = shape;
  key.push_back(double(cfg.qb));
  key.push_back(double(cfg.wg_per_cu));
  key.push_back(double(reinterpret_cast<uintptr_t>(ctx->ws)));
  key.push_back(double(ctx->ws_size));
  key.push_back(double(reinterpret_cast<uintptr_t>(ctx->ws3)));
  key.push_back(double(ctx->ws3_size));
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
    const int rc = tiled_queue(ctx, L);
    ctx->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc != FPCA_OK || ec != hipSuccess) {
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
    if (int rc = tiled_queue(ctx, L)) return rc;
    if (ctx->cv_exec) (void)hipGraphExecDestroy(ctx->cv_exec);
    ctx->cv_exec = nullptr;
    ctx->cv_key = key;
    ctx->cv_key_seen = 1;
  }
  if (int rc = finish_and_check(ctx)) return rc;
  FPCA_HIP(hipMemcpy(scores_h, L.args.scores, sizeof(double) * J, hipMemcpyDeviceToHost));
  return FPCA_OK;
}

}  // namespace
}  // namespace fpca

using namespace fpca;

extern "C" int fpca_cv_batched(fpca_handle ctx, int dtype, int n_data, const fpca_cv_data *data, int n_folds,
                               int n_h, const double *bandwidths, double *scores) {
  if (int rc = check_handle(ctx)) return rc;
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (n_data < 1 || n_folds < 1 || n_h < 1)
    return set_error(FPCA_ERR_INVALID_ARG, "need n_data >= 1, n_folds >= 1 and n_h >= 1");
  if (!data || !bandwidths || !scores) return set_error(FPCA_ERR_INVALID_ARG, "data, bandwidths and scores are required");
  const int d = data[0].grid.d;
  for (int a = 0; a < n_data; ++a) {
    int64_t P;
    if (int rc = check_grid(&data[a].grid, &P)) return rc;
    if (data[a].grid.d != d) return set_error(FPCA_ERR_INVALID_ARG, "dataset %d: every dataset needs the same d", a);
    if (!data[a].C || !data[a].G || !data[a].Q)
      return set_error(FPCA_ERR_INVALID_ARG, "dataset %d: C, G and Q are required", a);
    if (P > (int64_t(1) << 15))
      return set_error(FPCA_ERR_UNSUPPORTED, "dataset %d: covariance grid too large (P=%lld)", a, (long long)P);
  }
  for (int i = 0; i < n_h * d; ++i)
    if (!(bandwidths[i] > 0.0) || !std::isfinite(bandwidths[i]))
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidths must be positive and finite");
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64) return cv_impl<double>(ctx, dtype, n_data, data, n_folds, n_h, bandwidths, scores);
  return cv_impl<float>(ctx, dtype, n_data, data, n_folds, n_h, bandwidths, scores);
}

extern "C" int fpca_cv_select(int n_h, int d, const double *bandwidths, const double *cv, double *h_out) {
  if (n_h < 1 || d < 1 || d > 3 || !bandwidths || !cv || !h_out)
    return set_error(FPCA_ERR_INVALID_ARG, "need n_h >= 1, d in 1..3 and non-null arrays");
  for (int i = 0; i < n_h; ++i) {
    if (!(bandwidths[i * d] > 0.0) || !std::isfinite(bandwidths[i * d]))
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidths must be positive and finite");
    if (i > 0 && !(bandwidths[i * d] > bandwidths[(i - 1) * d]))
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidth rows must increase along their first coordinate");
    for (int k = 1; k < d; ++k) {
      const double r0 = bandwidths[k] / bandwidths[0], ri = bandwidths[i * d + k] / bandwidths[i * d];
      if (std::fabs(ri - r0) > 1e-12 * r0)
        return set_error(FPCA_ERR_INVALID_ARG, "bandwidth rows must be positive multiples of one vector");
    }
  }
  // grid argmin (first on ties; NaN scores never win)
  int b = -1;
  for (int i = 0; i < n_h; ++i)
    if (std::isfinite(cv[i]) && (b < 0 || cv[i] < cv[b])) b = i;
  if (b < 0) return set_error(FPCA_ERR_INVALID_ARG, "no finite CV score");
  double s = bandwidths[b * d];
  if (b > 0 && b < n_h - 1 && std::isfinite(cv[b - 1]) && std::isfinite(cv[b + 1])) {
    // vertex of the parabola through the three points in log h
    const double x0 = std::log(bandwidths[(b - 1) * d]), x1 = std::log(bandwidths[b * d]),
                 x2 = std::log(bandwidths[(b + 1) * d]);
    const double f0 = cv[b - 1], f1 = cv[b], f2 = cv[b + 1];
    const double den = (x0 - x1) * (x0 - x2) * (x1 - x2);
    const double A = (x2 * (f1 - f0) + x1 * (f0 - f2) + x0 * (f2 - f1)) / den;
    const double B = (x2 * x2 * (f0 - f1) + x1 * x1 * (f2 - f0) + x0 * x0 * (f1 - f2)) / den;
    if (A > 0.0) {
      const double xv = std::min(std::max(-B / (2.0 * A), x0), x2);
      s = std::exp(xv);
    }
  }
  for (int k = 0; k < d; ++k) h_out[k] = bandwidths[b * d + k] * (s / bandwidths[b * d]);
  return FPCA_OK;
}

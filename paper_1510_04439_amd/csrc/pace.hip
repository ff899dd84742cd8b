// Principal component scores by conditional expectation (PACE, eq. 2.7):
// for curve i,
//   xi_i = Lambda Phi_i^T Sigma_i^{-1} (Y_i - mu_i),
//   Sigma_i = Phi_i Lambda Phi_i^T + sigma^2 I,
// with Phi_i[j][l] = phi_l(t_ij) and mu_i[j] = mu(t_ij) interpolated from the
// grid by the multilinear corner weights of linear binning. The push-through
// identity Lambda Phi^T (Phi Lambda Phi^T + sigma^2 I)^{-1}
//   = (Phi^T Phi + sigma^2 Lambda^{-1})^{-1} Phi^T
// turns the N_i x N_i system into a k x k one:
//   (Phi_i^T Phi_i + sigma^2 Lambda^{-1}) xi_i = Phi_i^T (Y_i - mu_i).
// Components with lambda_l <= 0 are left out of Sigma_i and score 0.
#include "binrule.hpp"
#include "common.hpp"

namespace fpca {

namespace {

constexpr int PACE_KMAX = 32;
constexpr int PACE_CH = 64;  // observations staged in LDS per chunk
constexpr int PACE_THREADS = 256;
constexpr int PACE_TRI = PACE_KMAX * (PACE_KMAX + 1) / 2;
constexpr int PACE_ACC = (PACE_TRI + PACE_KMAX + PACE_THREADS - 1) / PACE_THREADS;

// sigma^2 / lambda_l for the kept components, -1 for the others
struct PaceDiag {
  double v[PACE_KMAX];
};

// One workgroup per curve (grid-stride). Chunks of observations: each thread
// of the first PACE_CH interpolates one observation (every component and the
// mean), then thread e accumulates entries e, e + 256, ... of the upper
// triangle of Phi^T Phi (row by row) followed by the k entries of
// Phi^T (Y - mu), in observation order.
// Thread 0 solves the k x k system by Cholesky in FP64.
template <typename T>
__global__ __launch_bounds__(PACE_THREADS) void k_pace(GridDims g, int64_t n, int design,
                                                       const int64_t *__restrict__ off, const T *__restrict__ t,
                                                       const T *__restrict__ y, const T *__restrict__ mu,
                                                       const T *__restrict__ efuns, int k, PaceDiag dg,
                                                       T *__restrict__ scores) {
  __shared__ double ph[PACE_CH][PACE_KMAX + 1];
  __shared__ double yc[PACE_CH];
  __shared__ double A[PACE_KMAX][PACE_KMAX + 1];
  __shared__ double rhs[PACE_KMAX];
  __shared__ unsigned char tri_r[PACE_TRI], tri_c[PACE_TRI];
  const int tid = threadIdx.x;
  const int64_t P = g.P;
  const int nmat = k * (k + 1) / 2, nacc = nmat + k;
  if (tid == 0)
    for (int r = 0, e = 0; r < k; ++r)
      for (int c = r; c < k; ++c, ++e) {
        tri_r[e] = (unsigned char)r;
        tri_c[e] = (unsigned char)c;
      }
  __syncthreads();
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    int64_t a, b;
    if (design == FPCA_IRREGULAR) {
      a = off[i];
      b = off[i + 1];
    } else {
      a = i * P;
      b = a + P;
    }
    double acc[PACE_ACC];
#pragma unroll
    for (int q = 0; q < PACE_ACC; ++q) acc[q] = 0.0;
    for (int64_t c0 = a; c0 < b; c0 += PACE_CH) {
      const int m = int(min(int64_t(PACE_CH), b - c0));
      __syncthreads();  // the previous chunk has been read
      if (tid < m) {
        const int64_t j = c0 + tid;
        int64_t node[8];
        double W[8];
        int nc = 0;
        bool ok = true;
        if (design == FPCA_IRREGULAR) {
          int kk[3];
          double rho[3];
          ok = locate(t + j * g.d, g, kk, rho);
          if (ok) {
            nc = 1 << g.d;
            for (int cc = 0; cc < nc; ++cc) corner(g, kk, rho, cc, &node[cc], &W[cc]);
          }
        } else {
          nc = 1;
          node[0] = j - a;
          W[0] = 1.0;
        }
        const double yv = double(y[j]);
        ok = ok && isfinite(yv);
        double mv = 0.0;
        if (ok)
          for (int cc = 0; cc < nc; ++cc) mv += W[cc] * double(mu[node[cc]]);
        yc[tid] = ok ? yv - mv : 0.0;
        for (int l = 0; l < k; ++l) {
          double v = 0.0;
          if (ok)
            for (int cc = 0; cc < nc; ++cc) v += W[cc] * double(efuns[int64_t(l) * P + node[cc]]);
          ph[tid][l] = v;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PACE_ACC; ++q) {
        const int e = tid + PACE_THREADS * q;
        if (e < nmat) {
          const int r = tri_r[e], c = tri_c[e];
          double s = 0.0;
          for (int o = 0; o < m; ++o) s += ph[o][r] * ph[o][c];
          acc[q] += s;
        } else if (e < nacc) {
          const int r = e - nmat;
          double s = 0.0;
          for (int o = 0; o < m; ++o) s += ph[o][r] * yc[o];
          acc[q] += s;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PACE_ACC; ++q) {
      const int e = tid + PACE_THREADS * q;
      if (e < nmat) {
        const int r = tri_r[e], c = tri_c[e];
        const bool kr = dg.v[r] >= 0.0, kc = dg.v[c] >= 0.0;
        // dropped components: identity rows and columns, zero right-hand side
        const double v = (kr && kc) ? acc[q] + (r == c ? dg.v[r] : 0.0) : (r == c ? 1.0 : 0.0);
        A[r][c] = v;
        A[c][r] = v;
      } else if (e < nacc) {
        const int r = e - nmat;
        rhs[r] = dg.v[r] >= 0.0 ? acc[q] : 0.0;
      }
    }
    __syncthreads();
    if (tid == 0) {
      bool good = true;
      for (int c = 0; c < k && good; ++c) {  // A = L L^T in place (lower triangle)
        double d = A[c][c];
        for (int p = 0; p < c; ++p) d -= A[c][p] * A[c][p];
        if (!(d > 0.0)) {
          good = false;
          break;
        }
        const double lc = sqrt(d);
        A[c][c] = lc;
        for (int r = c + 1; r < k; ++r) {
          double s = A[r][c];
          for (int p = 0; p < c; ++p) s -= A[r][p] * A[c][p];
          A[r][c] = s / lc;
        }
      }
      if (good) {
        for (int r = 0; r < k; ++r) {  // L z = rhs
          double s = rhs[r];
          for (int p = 0; p < r; ++p) s -= A[r][p] * rhs[p];
          rhs[r] = s / A[r][r];
        }
        for (int r = k - 1; r >= 0; --r) {  // L^T xi = z
          double s = rhs[r];
          for (int p = r + 1; p < k; ++p) s -= A[p][r] * rhs[p];
          rhs[r] = s / A[r][r];
        }
      }
      for (int l = 0; l < k; ++l) scores[i * k + l] = T(good ? rhs[l] : __builtin_nan(""));
    }
  }
}

template <typename T>
int pace_impl(fpca_context *ctx, const fpca_grid *grid, int design, int64_t n, const int64_t *offsets, const T *t,
              const T *y, const T *mu, const T *efuns, int k, const PaceDiag &dg, T *scores) {
  if (n == 0) return FPCA_OK;
  const GridDims g = make_dims(grid);
  const unsigned blocks = unsigned(n < 65536 ? n : 65536);
  hipLaunchKernelGGL(k_pace<T>, dim3(blocks), dim3(PACE_THREADS), 0, ctx->stream, g, n, design, offsets, t, y, mu,
                     efuns, k, dg, scores);
  FPCA_LAUNCH_CHECK("pace");
  return FPCA_OK;
}

// Reconstruction on the grid (the display after eq. 2.7):
//   xhat[i][p] = mu[p] + sum_l xi[i][l] phi_l[p].
// Thread per node p of a 256-node block with its k basis values in registers;
// the block's RC_CURVES score rows in LDS; writes are contiguous along p.
constexpr int RC_CURVES = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_reconstruct(int64_t P, int64_t n, int k, const T *__restrict__ mu,
                                                     const T *__restrict__ efuns, const T *__restrict__ xi,
                                                     T *__restrict__ xhat) {
  __shared__ double xs[RC_CURVES][PACE_KMAX];
  const int64_t i0 = int64_t(blockIdx.y) * RC_CURVES;
  const int nc = int(min(int64_t(RC_CURVES), n - i0));
  for (int e = threadIdx.x; e < nc * k; e += blockDim.x) xs[e / k][e % k] = double(xi[(i0 + e / k) * k + e % k]);
  __syncthreads();
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double ph[PACE_KMAX];
#pragma unroll
  for (int l = 0; l < PACE_KMAX; ++l) ph[l] = l < k ? double(efuns[int64_t(l) * P + p]) : 0.0;
  const double m = double(mu[p]);
  for (int c = 0; c < nc; ++c) {
    double v = m;
#pragma unroll
    for (int l = 0; l < PACE_KMAX; ++l)
      if (l < k) v += xs[c][l] * ph[l];
    xhat[(i0 + c) * P + p] = T(v);
  }
}

template <typename T>
int reconstruct_impl(fpca_context *ctx, int64_t P, int64_t n, int k, const T *mu, const T *efuns, const T *xi,
                     T *xhat) {
  if (n == 0 || P == 0) return FPCA_OK;
  const int64_t gy = (n + RC_CURVES - 1) / RC_CURVES;
  if (gy > 65535) return set_error(FPCA_ERR_UNSUPPORTED, "n = %lld curves exceeds %d", (long long)n, 65535 * RC_CURVES);
  hipLaunchKernelGGL(k_reconstruct<T>, dim3(unsigned((P + 255) / 256), unsigned(gy)), dim3(256), 0, ctx->stream, P,
                     n, k, mu, efuns, xi, xhat);
  FPCA_LAUNCH_CHECK("reconstruct");
  return FPCA_OK;
}

}  // namespace

}  // namespace fpca

using namespace fpca;

extern "C" int fpca_pace_scores(fpca_handle ctx, const fpca_grid *grid, int design, int dtype, int64_t n,
                                const int64_t *offsets, const void *t, const void *y, const void *mu,
                                const void *efuns, int k, const double *evals, double sigma2, void *scores) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (design != FPCA_IRREGULAR && design != FPCA_COMMON_GRID)
    return set_error(FPCA_ERR_INVALID_ARG, "bad design %d", design);
  if (n < 0) return set_error(FPCA_ERR_INVALID_ARG, "n < 0");
  if (k < 1 || k > PACE_KMAX) return set_error(FPCA_ERR_INVALID_ARG, "k = %d must be in 1..%d", k, PACE_KMAX);
  if (!(sigma2 > 0.0) || !std::isfinite(sigma2))
    return set_error(FPCA_ERR_INVALID_ARG, "sigma2 must be positive and finite");
  if (!y || !mu || !efuns || !evals || (!scores && n > 0))
    return set_error(FPCA_ERR_INVALID_ARG, "y, mu, efuns, evals and scores are required");
  if (design == FPCA_IRREGULAR && (!offsets || !t))
    return set_error(FPCA_ERR_INVALID_ARG, "the irregular design needs offsets and t");
  if (design == FPCA_COMMON_GRID && (offsets || t))
    return set_error(FPCA_ERR_INVALID_ARG, "the common-grid design takes offsets = t = NULL");
  PaceDiag dg{};
  for (int l = 0; l < PACE_KMAX; ++l) dg.v[l] = -1.0;
  for (int l = 0; l < k; ++l)
    if (evals[l] > 0.0 && std::isfinite(evals[l])) dg.v[l] = sigma2 / evals[l];
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return pace_impl<double>(ctx, grid, design, n, offsets, static_cast<const double *>(t),
                             static_cast<const double *>(y), static_cast<const double *>(mu),
                             static_cast<const double *>(efuns), k, dg, static_cast<double *>(scores));
  return pace_impl<float>(ctx, grid, design, n, offsets, static_cast<const float *>(t), static_cast<const float *>(y),
                          static_cast<const float *>(mu), static_cast<const float *>(efuns), k, dg,
                          static_cast<float *>(scores));
}

extern "C" int fpca_reconstruct(fpca_handle ctx, int dtype, int64_t P, int64_t n, int k, const void *mu,
                                const void *efuns, const void *scores, void *xhat) {
  if (int rc = check_handle(ctx)) return rc;
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (P < 0 || n < 0) return set_error(FPCA_ERR_INVALID_ARG, "P and n must be >= 0");
  if (k < 1 || k > PACE_KMAX) return set_error(FPCA_ERR_INVALID_ARG, "k = %d must be in 1..%d", k, PACE_KMAX);
  if ((n > 0 && P > 0) && (!mu || !efuns || !scores || !xhat))
    return set_error(FPCA_ERR_INVALID_ARG, "mu, efuns, scores and xhat are required");
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return reconstruct_impl<double>(ctx, P, n, k, static_cast<const double *>(mu), static_cast<const double *>(efuns),
                                    static_cast<const double *>(scores), static_cast<double *>(xhat));
  return reconstruct_impl<float>(ctx, P, n, k, static_cast<const float *>(mu), static_cast<const float *>(efuns),
                                 static_cast<const float *>(scores), static_cast<float *>(xhat));
}

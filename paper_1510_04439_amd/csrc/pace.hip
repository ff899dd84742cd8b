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
#include <mutex>

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

// A = L L^T in place (lower triangle of A, k x k, row stride PACE_KMAX + 1);
// false if a pivot is not positive.
__device__ inline bool chol_inplace(double (*A)[PACE_KMAX + 1], int k) {
  for (int c = 0; c < k; ++c) {
    double d = A[c][c];
    for (int p = 0; p < c; ++p) d -= A[c][p] * A[c][p];
    if (!(d > 0.0)) return false;
    const double lc = sqrt(d);
    A[c][c] = lc;
    for (int r = c + 1; r < k; ++r) {
      double s = A[r][c];
      for (int p = 0; p < c; ++p) s -= A[r][p] * A[c][p];
      A[r][c] = s / lc;
    }
  }
  return true;
}

// x = (L L^T)^{-1} x with L from chol_inplace.
__device__ inline void chol_solve(const double (*L)[PACE_KMAX + 1], double *x, int k) {
  for (int r = 0; r < k; ++r) {
    double s = x[r];
    for (int p = 0; p < r; ++p) s -= L[r][p] * x[p];
    x[r] = s / L[r][r];
  }
  for (int r = k - 1; r >= 0; --r) {
    double s = x[r];
    for (int p = r + 1; p < k; ++p) s -= L[p][r] * x[p];
    x[r] = s / L[r][r];
  }
}

// Common grid: the factor of Phi^T Phi + sigma^2 Lambda^{-1} over all P nodes,
// shared by every curve observed at all of them. One workgroup: the basis in
// chunks of 64 nodes through LDS, thread e accumulates upper-triangle entry e
// in node order; thread 0 factors. ok[0] = 1 on success.
template <typename T>
__global__ __launch_bounds__(PACE_THREADS) void k_pace_cg_prep(int64_t P, const T *__restrict__ efuns, int k,
                                                               PaceDiag dg, double *__restrict__ Lout,
                                                               int *__restrict__ ok) {
  __shared__ double ph[PACE_CH][PACE_KMAX + 1];
  __shared__ double A[PACE_KMAX][PACE_KMAX + 1];
  __shared__ unsigned char tri_r[PACE_TRI], tri_c[PACE_TRI];
  const int tid = threadIdx.x;
  const int nmat = k * (k + 1) / 2;
  if (tid == 0)
    for (int r = 0, e = 0; r < k; ++r)
      for (int c = r; c < k; ++c, ++e) {
        tri_r[e] = (unsigned char)r;
        tri_c[e] = (unsigned char)c;
      }
  double acc[PACE_ACC];
#pragma unroll
  for (int q = 0; q < PACE_ACC; ++q) acc[q] = 0.0;
  for (int64_t c0 = 0; c0 < P; c0 += PACE_CH) {
    const int m = int(min(int64_t(PACE_CH), P - c0));
    __syncthreads();
    if (tid < m)
      for (int l = 0; l < k; ++l) ph[tid][l] = double(efuns[int64_t(l) * P + c0 + tid]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PACE_ACC; ++q) {
      const int e = tid + PACE_THREADS * q;
      if (e < nmat) {
        const int r = tri_r[e], c = tri_c[e];
        double sum = 0.0;
        for (int o = 0; o < m; ++o) sum += ph[o][r] * ph[o][c];
        acc[q] += sum;
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
      const double v = (kr && kc) ? acc[q] + (r == c ? dg.v[r] : 0.0) : (r == c ? 1.0 : 0.0);
      A[r][c] = v;
      A[c][r] = v;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const bool good = chol_inplace(A, k);
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) Lout[r * k + c] = A[r][c];
    ok[0] = good ? 1 : 0;
  }
}

// One workgroup per curve (grid-stride). Chunks of observations: each thread
// of the first PACE_CH interpolates one observation (every component and the
// mean), then thread e accumulates entries e, e + 256, ... of the upper
// triangle of Phi^T Phi (row by row) followed by the k entries of
// Phi^T (Y - mu), in observation order.
// Thread 0 solves the k x k system by Cholesky in FP64. On the common grid a
// curve with no missing value takes the factor shared by all such curves.
template <typename T>
__global__ __launch_bounds__(PACE_THREADS) void k_pace(GridDims g, int64_t n, int design,
                                                       const int64_t *__restrict__ off, const T *__restrict__ t,
                                                       const T *__restrict__ y, const T *__restrict__ mu,
                                                       const T *__restrict__ efuns, int k, PaceDiag dg,
                                                       const double *__restrict__ Lcg, const int *__restrict__ cg_ok,
                                                       T *__restrict__ scores) {
  __shared__ double ph[PACE_CH][PACE_KMAX + 1];
  __shared__ double Lc[PACE_KMAX][PACE_KMAX + 1];
  __shared__ double red[PACE_THREADS / 64][PACE_KMAX];
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
  const bool fast = design == FPCA_COMMON_GRID && Lcg && cg_ok && cg_ok[0] == 1;
  if (fast)
    for (int e = tid; e < k * k; e += PACE_THREADS) Lc[e / k][e % k] = Lcg[e];
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
    if (fast) {
      // a curve observed at every node uses the shared factor: only
      // Phi^T (Y_i - mu) is formed (strided per thread, then the waves in order)
      bool missing = false;
      for (int64_t p = tid; p < P; p += PACE_THREADS) missing |= !isfinite(double(y[a + p]));
      if (!__syncthreads_or(missing)) {
        double part[PACE_KMAX];
#pragma unroll
        for (int l = 0; l < PACE_KMAX; ++l) part[l] = 0.0;
        for (int64_t p = tid; p < P; p += PACE_THREADS) {
          const double ycv = double(y[a + p]) - double(mu[p]);
#pragma unroll
          for (int l = 0; l < PACE_KMAX; ++l)
            if (l < k) part[l] += double(efuns[int64_t(l) * P + p]) * ycv;
        }
        // constant indices throughout, so part[] stays in registers
#pragma unroll
        for (int l = 0; l < PACE_KMAX; ++l) {
          double v = part[l];
          for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
          if ((tid & 63) == 0 && l < k) red[tid >> 6][l] = v;
        }
        __syncthreads();
        if (tid < k) {
          double v = 0.0;
          for (int w = 0; w < PACE_THREADS / 64; ++w) v += red[w][tid];
          rhs[tid] = dg.v[tid] >= 0.0 ? v : 0.0;
        }
        __syncthreads();
        if (tid == 0) {
          chol_solve(Lc, rhs, k);
          for (int l = 0; l < k; ++l) scores[i * k + l] = T(rhs[l]);
        }
        __syncthreads();  // rhs and red are reused by the next curve
        continue;
      }
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
#pragma unroll
            for (int cc = 0; cc < 8; ++cc)
              if (cc < nc) corner(g, kk, rho, cc, &node[cc], &W[cc]);
          }
        } else {
          nc = 1;
          node[0] = j - a;
          W[0] = 1.0;
        }
        const double yv = double(y[j]);
        ok = ok && isfinite(yv);
        double mv = 0.0;
        if (ok) {
#pragma unroll
          for (int cc = 0; cc < 8; ++cc)
            if (cc < nc) mv += W[cc] * double(mu[node[cc]]);
        }
        yc[tid] = ok ? yv - mv : 0.0;
        for (int l = 0; l < k; ++l) {
          double v = 0.0;
          if (ok) {
#pragma unroll
            for (int cc = 0; cc < 8; ++cc)
              if (cc < nc) v += W[cc] * double(efuns[int64_t(l) * P + node[cc]]);
          }
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
      const bool good = chol_inplace(A, k);
      if (good) chol_solve(A, rhs, k);
      for (int l = 0; l < k; ++l) scores[i * k + l] = T(good ? rhs[l] : __builtin_nan(""));
    }
  }
}

// Scratch of the common-grid design: the shared k x k factor and its flag.
constexpr size_t PACE_SCRATCH_BYTES = PACE_KMAX * PACE_KMAX * sizeof(double) + 256;

// `fixed`: caller-provided scratch of PACE_SCRATCH_BYTES (the allocation-free
// entry point), or NULL to carve it from the handle's arena.
template <typename T>
int pace_impl(fpca_context *ctx, const fpca_grid *grid, int design, int64_t n, const int64_t *offsets, const T *t,
              const T *y, const T *mu, const T *efuns, int k, const PaceDiag &dg, T *scores, void *fixed) {
  if (n == 0) return FPCA_OK;
  const GridDims g = make_dims(grid);
  const double *Lcg = nullptr;
  const int *cg_ok = nullptr;
  if (design == FPCA_COMMON_GRID) {
    if (!fixed)
      if (int rc = ws_reserve(ctx, PACE_SCRATCH_BYTES)) return rc;
    Carver cv{static_cast<char *>(fixed ? fixed : ctx->ws), 0, fixed ? PACE_SCRATCH_BYTES : ctx->ws_size};
    double *L = cv.take<double>(PACE_KMAX * PACE_KMAX);
    int *okf = cv.take<int>(1);
    hipLaunchKernelGGL(k_pace_cg_prep<T>, dim3(1), dim3(PACE_THREADS), 0, ctx->stream, g.P, efuns, k, dg, L, okf);
    FPCA_LAUNCH_CHECK("pace_cg_prep");
    Lcg = L;
    cg_ok = okf;
  }
  const unsigned blocks = unsigned(n < 65536 ? n : 65536);
  hipLaunchKernelGGL(k_pace<T>, dim3(blocks), dim3(PACE_THREADS), 0, ctx->stream, g, n, design, offsets, t, y, mu,
                     efuns, k, dg, Lcg, cg_ok, scores);
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

// One copy per GPU of the scratch used by fpca_pace_scores_noalloc. In host
// code `scratch` names a host-side stand-in: kernels get the device address
// looked up for each device by pace_scratch_init.
constexpr int PACE_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[PACE_MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[PACE_SCRATCH_BYTES];

// Looks up this device's address of `scratch` (the device must be current).
// Called by fpca_create, once per device.
int pace_scratch_init(int device) {
  if (device < 0 || device >= PACE_MAX_DEVICES)
    return set_error(FPCA_ERR_UNSUPPORTED, "device %d beyond the %d supported", device, PACE_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return FPCA_OK;
  void *ptr = nullptr;
  FPCA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return set_error(FPCA_ERR_DEVICE, "no device address for the PACE scratch");
  g_scratch_ptr[device] = ptr;
  return FPCA_OK;
}

}  // namespace fpca

using namespace fpca;

namespace {

int pace_entry(fpca_handle ctx, const fpca_grid *grid, int design, int dtype, int64_t n, const int64_t *offsets,
               const void *t, const void *y, const void *mu, const void *efuns, int k, const double *evals,
               double sigma2, void *scores, bool no_alloc) {
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
  void *fixed = nullptr;
  if (no_alloc) {
    // k <= PACE_KMAX was checked above, so the fixed scratch always suffices
    fixed = (ctx->device >= 0 && ctx->device < PACE_MAX_DEVICES) ? g_scratch_ptr[ctx->device] : nullptr;
    if (!fixed) return set_error(FPCA_ERR_DEVICE, "PACE scratch not set up on device %d", ctx->device);
  }
  if (dtype == FPCA_F64)
    return pace_impl<double>(ctx, grid, design, n, offsets, static_cast<const double *>(t),
                             static_cast<const double *>(y), static_cast<const double *>(mu),
                             static_cast<const double *>(efuns), k, dg, static_cast<double *>(scores), fixed);
  return pace_impl<float>(ctx, grid, design, n, offsets, static_cast<const float *>(t), static_cast<const float *>(y),
                          static_cast<const float *>(mu), static_cast<const float *>(efuns), k, dg,
                          static_cast<float *>(scores), fixed);
}

}  // namespace

extern "C" int fpca_pace_scores(fpca_handle ctx, const fpca_grid *grid, int design, int dtype, int64_t n,
                                const int64_t *offsets, const void *t, const void *y, const void *mu,
                                const void *efuns, int k, const double *evals, double sigma2, void *scores) {
  return pace_entry(ctx, grid, design, dtype, n, offsets, t, y, mu, efuns, k, evals, sigma2, scores, false);
}

extern "C" int fpca_pace_scores_noalloc(fpca_handle ctx, const fpca_grid *grid, int design, int dtype, int64_t n,
                                        const int64_t *offsets, const void *t, const void *y, const void *mu,
                                        const void *efuns, int k, const double *evals, double sigma2,
                                        void *scores) {
  return pace_entry(ctx, grid, design, dtype, n, offsets, t, y, mu, efuns, k, evals, sigma2, scores, true);
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

// Random-projection eigendecomposition of the matrixized covariance
// (Sections 3.1 and 3.4): A = W^1/2 Gamma W^1/2 is never formed; every product
// A X is computed as W^1/2 (Gamma (W^1/2 X)).
//
//   test matrix  : counter-based normals (splitmix64 + Box-Muller), P x r
//   products     : Gamma X on MFMA (FP32) with split K, FP64 reduction
//   orthonormal  : CholeskyQR2 in FP64 (columns that become numerically
//                  dependent are dropped: their basis vector is set to 0)
//   Rayleigh-Ritz: B = Q^T A Q in FP64, eigenpairs by a one-workgroup
//                  parallel-ordered cyclic Jacobi method in FP64
//   finalize     : psi = Q U, phi = psi / sqrt(w), sign rule, FVE.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace fpca {
namespace {

typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Standard normal number i of stream `seed`: Box-Muller cosine branch on
// u1 = ((a >> 11) + 1) 2^-53 in (0,1] and u2 = (b >> 11) 2^-53, a, b the
// splitmix64 outputs 2i and 2i+1.
__device__ inline double normal_at(uint64_t seed, uint64_t i) {
  const uint64_t a = splitmix64_at(seed, 2 * i), b = splitmix64_at(seed, 2 * i + 1);
  const double u1 = double((a >> 11) + 1) * 0x1.0p-53;
  const double u2 = double(b >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

__global__ void k_normals(uint64_t seed, int64_t count, double *out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (; i < count; i += step) out[i] = normal_at(seed, uint64_t(i));
}

// X[p, j] = sqrt(w_p) Omega[p, j] (row-major P x rp, zero for j >= r).
template <typename T>
__global__ void k_test_matrix(uint64_t seed, int64_t P, int r, int rp, const double *__restrict__ w, T *X) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P * rp) return;
  const int64_t p = e / rp;
  const int j = int(e % rp);
  double v = 0.0;
  if (j < r) v = sqrt(w[p]) * normal_at(seed, uint64_t(j) * uint64_t(P) + uint64_t(p));
  X[e] = T(v);
}

__global__ void k_default_w(int64_t P, double wv, const uint8_t *mask, double *w) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < P) w[p] = (mask && !mask[p]) ? 0.0 : wv;
}

// Partial products of Y^T = X^T Gamma over one K chunk (Gamma symmetric):
// workgroup (column block of 64 nodes, K chunk), 4 waves x 16 columns, MFMA
// 16x16x4 FP32 with the basis as the A operand and Gamma rows as B.
template <int RB>
__global__ __launch_bounds__(256) void k_panel_f32(int64_t P, const float *__restrict__ G,
                                                    const float *__restrict__ X, int64_t kchunk,
                                                    float *__restrict__ part) {
  constexpr int RP = RB * 16;
  __shared__ float As[16][64 + 4];
  __shared__ float Xs[16][RP + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = int64_t(blockIdx.x) * 64;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk;
  const int64_t k1 = min(P, k0 + kchunk);
  float4_t acc[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) acc[b] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int ar = tid >> 4, ac = (tid & 15) * 4;
  for (int64_t kb = k0; kb < k1; kb += 16) {
    {
      const int64_t q = kb + ar;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = (q < k1 && c0 + ac + e < P) ? G[q * P + c0 + ac + e] : 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[ar][ac + e] = v[e];
    }
    for (int e = tid; e < 16 * RP; e += 256) {
      const int rr = e / RP, cc = e % RP;
      const int64_t q = kb + rr;
      Xs[rr][cc] = (q < k1) ? X[q * RP + cc] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int krow = kk + (lane >> 4);
      const float b = As[krow][wave * 16 + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < RB; ++mb) {
        const float a = Xs[krow][mb * 16 + (lane & 15)];
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[mb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D[j][p]: row j = mb*16 + 4*(lane/16) + v, column p = c0 + wave*16 + lane%16.
  const int64_t p = c0 + wave * 16 + (lane & 15);
  if (p < P) {
    float *dst = part + (int64_t(blockIdx.y) * P + p) * RP;
#pragma unroll
    for (int mb = 0; mb < RB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[mb * 16 + 4 * (lane >> 4) + v] = acc[mb][v];
  }
}

// Y[p, j] = sqrt(w_p) sum over K chunks of the partials (FP64).
__global__ void k_panel_reduce(int64_t P, int rp, int nsplit, const float *__restrict__ part,
                               const double *__restrict__ w, double *__restrict__ Y) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P * rp) return;
  const int64_t p = e / rp;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += double(part[int64_t(k) * P * rp + e]);
  Y[e] = sqrt(w[p]) * s;
}

// FP64 product Y = W^1/2 Gamma X for FP64 storage (small grids).
__global__ void k_panel_f64(int64_t P, int rp, const double *__restrict__ G, const double *__restrict__ X,
                            const double *__restrict__ w, double *__restrict__ Y) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P * rp) return;
  const int64_t p = e / rp;
  const int j = int(e % rp);
  double s = 0.0;
  for (int64_t q = 0; q < P; ++q) s += G[p * P + q] * X[q * rp + j];
  Y[e] = sqrt(w[p]) * s;
}

// Partial Gram products of two P x rp FP64 matrices over row chunks:
// part[c][a][b] = sum_{p in chunk c} U[p][a] V[p][b].
__global__ __launch_bounds__(256) void k_gram_part(int64_t P, int rp, int64_t chunk, const double *__restrict__ U,
                                                    const double *__restrict__ V, double *__restrict__ part) {
  const int64_t p0 = int64_t(blockIdx.x) * chunk, p1 = min(P, p0 + chunk);
  for (int e = threadIdx.x; e < rp * rp; e += blockDim.x) {
    const int a = e / rp, b = e % rp;
    double s = 0.0;
    for (int64_t p = p0; p < p1; ++p) s += U[p * rp + a] * V[p * rp + b];
    part[int64_t(blockIdx.x) * rp * rp + e] = s;
  }
}

// One workgroup: G = sum of partials; Cholesky G = R^T R with numerically
// dependent columns dropped (pivot <= 1e-12 of the column's squared norm);
// Rinv = R^{-1} with the dropped columns zeroed; act[j] = 1 for kept columns.
__global__ __launch_bounds__(256) void k_chol(int rp, int nparts, const double *__restrict__ part,
                                               double *__restrict__ Rinv, int *__restrict__ act) {
  __shared__ double Gs[64][65];
  __shared__ double L[64][65];
  __shared__ double Ri[64][65];
  __shared__ int keep[64];
  const int tid = threadIdx.x;
  for (int e = tid; e < rp * rp; e += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nparts; ++c) s += part[int64_t(c) * rp * rp + e];
    Gs[e / rp][e % rp] = s;
    L[e / rp][e % rp] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < rp; ++j) {
    if (tid == 0) {
      double dj = Gs[j][j];
      for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k];
      const bool ok = Gs[j][j] > 0.0 && dj > 1e-12 * Gs[j][j];
      keep[j] = ok ? 1 : 0;
      L[j][j] = ok ? sqrt(dj) : 1.0;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < rp; i += blockDim.x) {
      double v = 0.0;
      if (keep[j]) {
        v = Gs[i][j];
        for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
        v /= L[j][j];
      }
      L[i][j] = v;
    }
    __syncthreads();
  }
  // R = L^T (upper). Column j of R^{-1}: solve R x = e_j by back substitution.
  for (int j = tid; j < rp; j += blockDim.x) {
    for (int i = rp - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) v -= L[k][i] * Ri[k][j];
      Ri[i][j] = (i <= j) ? v / L[i][i] : 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < rp * rp; e += blockDim.x) {
    const int i = e / rp, j = e % rp;
    Rinv[e] = keep[j] ? Ri[i][j] : 0.0;
  }
  for (int j = tid; j < rp; j += blockDim.x) act[j] = keep[j];
}

// Q = Y Rinv (FP64) and the next basis X = W^1/2 Q in storage type T.
template <typename T>
__global__ void k_apply_rinv(int64_t P, int rp, const double *__restrict__ Y, const double *__restrict__ Rinv,
                             const double *__restrict__ w, double *__restrict__ Q, T *__restrict__ X) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P * rp) return;
  const int64_t p = e / rp;
  const int j = int(e % rp);
  double s = 0.0;
  for (int i = 0; i <= j; ++i) s += Y[p * rp + i] * Rinv[i * rp + j];
  Q[e] = s;
  if (X) X[e] = T(sqrt(w[p]) * s);
}

// One workgroup: B = sum of partials restricted to the active columns,
// symmetrized; cyclic Jacobi with round-robin ordering (disjoint rotations
// applied together); eigenvalues sorted descending (stable); outputs the top k
// values, their eigenvectors mapped back to the rp basis columns, and FVE.
__global__ __launch_bounds__(1024) void k_jacobi(int rp, int nparts, const double *__restrict__ part,
                                                  const int *__restrict__ act, int k, double *__restrict__ evals,
                                                  double *__restrict__ fve, double *__restrict__ Uk) {
  __shared__ double B[64][65];
  __shared__ double V[64][65];
  __shared__ double cs[32], sn[32];
  __shared__ int pa[32], pb[32];
  __shared__ int idx[64];
  __shared__ int n_s, ne_s;
  __shared__ double red[1024];
  __shared__ int stop;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int n = 0;
    for (int j = 0; j < rp; ++j)
      if (act[j]) idx[n++] = j;
    n_s = n;
    ne_s = n + (n & 1);
  }
  __syncthreads();
  const int n = n_s, ne = ne_s;
  for (int e = tid; e < ne * ne; e += blockDim.x) {
    const int a = e / ne, b = e % ne;
    double v = 0.0;
    if (a < n && b < n) {
      const int64_t o1 = int64_t(idx[a]) * rp + idx[b], o2 = int64_t(idx[b]) * rp + idx[a];
      double s1 = 0.0, s2 = 0.0;
      for (int c = 0; c < nparts; ++c) {
        s1 += part[int64_t(c) * rp * rp + o1];
        s2 += part[int64_t(c) * rp * rp + o2];
      }
      v = 0.5 * (s1 + s2);
    }
    B[a][b] = v;
    V[a][b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int npair = ne / 2;
  for (int sweep = 0; sweep < 60 && ne >= 2; ++sweep) {
    // convergence: off-diagonal mass against the whole
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < ne * ne; e += blockDim.x) {
      const int a = e / ne, b = e % ne;
      const double v = B[a][b] * B[a][b];
      tot += v;
      if (a != b) off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) stop = !(offs > 1e-30 * red[0]);
    __syncthreads();
    if (stop) break;
    for (int st = 0; st < ne - 1; ++st) {
      if (tid < npair) {
        int a, b;
        if (tid == 0) {
          a = ne - 1;
          b = st;
        } else {
          a = (st + tid) % (ne - 1);
          b = (st - tid + ne - 1) % (ne - 1);
        }
        const double apq = B[a][b];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (B[b][b] - B[a][a]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        pa[tid] = a;
        pb[tid] = b;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows: B <- J^T B
      for (int e = tid; e < npair * ne; e += blockDim.x) {
        const int m = e / ne, col = e % ne;
        const int a = pa[m], b = pb[m];
        const double c = cs[m], s = sn[m];
        const double x = B[a][col], y = B[b][col];
        B[a][col] = c * x - s * y;
        B[b][col] = s * x + c * y;
      }
      __syncthreads();
      // columns: B <- B J, V <- V J
      for (int e = tid; e < npair * ne; e += blockDim.x) {
        const int m = e / ne, row = e % ne;
        const int a = pa[m], b = pb[m];
        const double c = cs[m], s = sn[m];
        const double x = B[row][a], y = B[row][b];
        B[row][a] = c * x - s * y;
        B[row][b] = s * x + c * y;
        const double vx = V[row][a], vy = V[row][b];
        V[row][a] = c * vx - s * vy;
        V[row][b] = s * vx + c * vy;
      }
      __syncthreads();
    }
  }
  // Sort the n real eigenvalues (the padding index, if any, is excluded).
  __shared__ int order[64];
  __shared__ double possum;
  if (tid < n) {
    const double v = B[tid][tid];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = B[j][j];
      if (u > v || (u == v && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
      if (B[j][j] > 0.0) s += B[j][j];
    possum = s;
  }
  __syncthreads();
  if (tid == 0) {
    double cum = 0.0;
    for (int l = 0; l < k; ++l) {
      const double v = l < n ? B[order[l]][order[l]] : 0.0;
      cum += v;
      evals[l] = v;
      fve[l] = possum > 0.0 ? cum / possum : 0.0;
    }
  }
  for (int e = tid; e < rp * k; e += blockDim.x) Uk[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < n * k; e += blockDim.x) {
    const int a = e / k, l = e % k;
    if (l < n) Uk[int64_t(idx[a]) * k + l] = V[a][order[l]];
  }
}

// One workgroup per eigenvector l: psi = Q U[:, l], phi = psi / sqrt(w) (0 where
// w = 0), sign rule, written column-major into efuns.
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(int64_t P, int rp, int k, const double *__restrict__ Q,
                                                   const double *__restrict__ Uk, const double *__restrict__ w,
                                                   double *__restrict__ phi, T *__restrict__ efuns) {
  __shared__ double r1[256], r2[256], r3[256];
  __shared__ long long ri[256];
  const int l = blockIdx.x, tid = threadIdx.x;
  double s1 = 0.0, s2 = 0.0, mx = 0.0;
  for (int64_t p = tid; p < P; p += blockDim.x) {
    double v = 0.0;
    for (int i = 0; i < rp; ++i) v += Q[p * rp + i] * Uk[int64_t(i) * k + l];
    const double f = w[p] > 0.0 ? v / sqrt(w[p]) : 0.0;
    phi[int64_t(l) * P + p] = f;
    s1 += w[p] * f;
    s2 += w[p] * fabs(f);
    mx = fmax(mx, fabs(f));
  }
  r1[tid] = s1;
  r2[tid] = s2;
  r3[tid] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      r1[tid] += r1[tid + s];
      r2[tid] += r2[tid + s];
      r3[tid] = fmax(r3[tid], r3[tid + s]);
    }
    __syncthreads();
  }
  const double S1 = r1[0], S2 = r2[0], MX = r3[0];
  __syncthreads();
  bool neg;
  if (fabs(S1) >= 1e-8 * S2) {
    neg = S1 < 0.0;
  } else {
    long long first = P;
    for (int64_t p = tid; p < P; p += blockDim.x)
      if (fabs(phi[int64_t(l) * P + p]) >= (1.0 - 1e-6) * MX) {
        first = p;
        break;
      }
    ri[tid] = first;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) ri[tid] = min(ri[tid], ri[tid + s]);
      __syncthreads();
    }
    neg = (ri[0] < P) && phi[int64_t(l) * P + ri[0]] < 0.0;
  }
  const double sg = neg ? -1.0 : 1.0;
  for (int64_t p = tid; p < P; p += blockDim.x) efuns[int64_t(l) * P + p] = T(sg * phi[int64_t(l) * P + p]);
}

inline unsigned nb(int64_t n) { return unsigned((n + 255) / 256); }

template <typename T>
int eig_impl(fpca_context *ctx, const fpca_grid *grid, int64_t P, const T *gamma, const double *quad_w, int k,
             int oversample, int power_iters, uint64_t seed, double *evals_h, T *efuns, double *fve_h) {
  const int r = k + oversample;
  const int rp = ((r + 15) / 16) * 16;
  // K split of the panel product: enough workgroups to fill the chip
  const int64_t colblocks = (P + 63) / 64;
  int64_t nsplit = (4 * int64_t(ctx->num_cus) + colblocks - 1) / colblocks;
  if (nsplit < 1) nsplit = 1;
  int64_t kchunk = ((P + nsplit - 1) / nsplit + 15) / 16 * 16;
  nsplit = (P + kchunk - 1) / kchunk;
  const int64_t gchunk = 256;
  const int64_t ngram = (P + gchunk - 1) / gchunk;
  const bool f32 = sizeof(T) == 4;
  size_t need = carve_bytes(P, 8) + carve_bytes(P * rp, sizeof(T)) + 3 * carve_bytes(P * rp, 8) +
                carve_bytes(ngram * rp * rp, 8) + carve_bytes(rp * rp, 8) + carve_bytes(rp, 4) +
                carve_bytes(rp * k, 8) + 2 * carve_bytes(k, 8) + carve_bytes(P * k, 8);
  if (f32) need += carve_bytes(nsplit * P * rp, 4);
  if (int rc = ws_reserve(ctx, need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  double *w = cv.take<double>(P);
  T *X = cv.take<T>(P * rp);
  double *Y = cv.take<double>(P * rp);
  double *Q = cv.take<double>(P * rp);
  double *Z = cv.take<double>(P * rp);
  double *gpart = cv.take<double>(ngram * rp * rp);
  double *Rinv = cv.take<double>(rp * rp);
  int *act = cv.take<int>(rp);
  double *Uk = cv.take<double>(rp * k);
  double *ev_d = cv.take<double>(k);
  double *fve_d = cv.take<double>(k);
  double *phi = cv.take<double>(P * k);
  float *part = f32 ? cv.take<float>(nsplit * P * rp) : nullptr;

  if (quad_w) {
    FPCA_HIP(hipMemcpyAsync(w, quad_w, sizeof(double) * P, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    double wv = 1.0;
    for (int q = 0; q < grid->d; ++q) wv /= double(grid->M[q] - 1);
    hipLaunchKernelGGL(k_default_w, dim3(nb(P)), dim3(256), 0, ctx->stream, P, wv, grid->mask, w);
    FPCA_LAUNCH_CHECK("default_w");
  }
  hipLaunchKernelGGL(k_test_matrix<T>, dim3(nb(P * rp)), dim3(256), 0, ctx->stream, seed, P, r, rp, w, X);
  FPCA_LAUNCH_CHECK("test_matrix");

  auto product = [&](double *out) -> int {
    if constexpr (sizeof(T) == 4) {
      dim3 grd((unsigned)colblocks, (unsigned)nsplit);
      switch (rp / 16) {
        case 1: hipLaunchKernelGGL(k_panel_f32<1>, grd, dim3(256), 0, ctx->stream, P, (const float *)gamma, (const float *)X, kchunk, part); break;
        case 2: hipLaunchKernelGGL(k_panel_f32<2>, grd, dim3(256), 0, ctx->stream, P, (const float *)gamma, (const float *)X, kchunk, part); break;
        case 3: hipLaunchKernelGGL(k_panel_f32<3>, grd, dim3(256), 0, ctx->stream, P, (const float *)gamma, (const float *)X, kchunk, part); break;
        default: hipLaunchKernelGGL(k_panel_f32<4>, grd, dim3(256), 0, ctx->stream, P, (const float *)gamma, (const float *)X, kchunk, part); break;
      }
      FPCA_LAUNCH_CHECK("panel_f32");
      hipLaunchKernelGGL(k_panel_reduce, dim3(nb(P * rp)), dim3(256), 0, ctx->stream, P, rp, int(nsplit), part, w, out);
      FPCA_LAUNCH_CHECK("panel_reduce");
    } else {
      hipLaunchKernelGGL(k_panel_f64, dim3(nb(P * rp)), dim3(256), 0, ctx->stream, P, rp, (const double *)gamma,
                         (const double *)X, w, out);
      FPCA_LAUNCH_CHECK("panel_f64");
    }
    return FPCA_OK;
  };
  auto cholqr = [&](const double *Yin) -> int {
    // two CholeskyQR passes: Y -> Q1 (in Z) -> Q
    const double *src = Yin;
    double *dst[2] = {Z, Q};
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_gram_part, dim3(unsigned(ngram)), dim3(256), 0, ctx->stream, P, rp, gchunk, src, src, gpart);
      FPCA_LAUNCH_CHECK("gram_part");
      hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, ctx->stream, rp, int(ngram), gpart, Rinv, act);
      FPCA_LAUNCH_CHECK("chol");
      hipLaunchKernelGGL(k_apply_rinv<T>, dim3(nb(P * rp)), dim3(256), 0, ctx->stream, P, rp, src, Rinv, w, dst[pass],
                         pass == 1 ? X : (T *)nullptr);
      FPCA_LAUNCH_CHECK("apply_rinv");
      src = dst[pass];
    }
    return FPCA_OK;
  };

  if (int rc = product(Y)) return rc;
  if (int rc = cholqr(Y)) return rc;
  for (int it = 0; it < 2 * power_iters; ++it) {
    if (int rc = product(Y)) return rc;
    if (int rc = cholqr(Y)) return rc;
  }
  if (int rc = product(Z)) return rc;  // Z = A Q
  hipLaunchKernelGGL(k_gram_part, dim3(unsigned(ngram)), dim3(256), 0, ctx->stream, P, rp, gchunk, Q, Z, gpart);
  FPCA_LAUNCH_CHECK("rr_gram");
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, ctx->stream, rp, int(ngram), gpart, act, k, ev_d, fve_d, Uk);
  FPCA_LAUNCH_CHECK("jacobi");
  hipLaunchKernelGGL(k_finalize<T>, dim3(unsigned(k)), dim3(256), 0, ctx->stream, P, rp, k, Q, Uk, w, phi, efuns);
  FPCA_LAUNCH_CHECK("finalize");
  std::vector<double> hb(2 * k);
  FPCA_HIP(hipMemcpyAsync(hb.data(), ev_d, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipMemcpyAsync(hb.data() + k, fve_d, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  for (int l = 0; l < k; ++l) {
    evals_h[l] = hb[l];
    if (fve_h) fve_h[l] = hb[k + l];
  }
  return FPCA_OK;
}

}  // namespace
}  // namespace fpca

using namespace fpca;

extern "C" int fpca_rng_normal(fpca_handle ctx, uint64_t seed, int64_t count, double *out) {
  if (int rc = check_handle(ctx)) return rc;
  if (count < 0 || (count > 0 && !out)) return set_error(FPCA_ERR_INVALID_ARG, "bad count or output");
  if (int rc = set_device(ctx)) return rc;
  if (count == 0) return FPCA_OK;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_normals, dim3(unsigned(blocks)), dim3(256), 0, ctx->stream, seed, count, out);
  FPCA_LAUNCH_CHECK("normals");
  return FPCA_OK;
}

extern "C" int fpca_eig_randomized(fpca_handle ctx, int dtype, int prec, const fpca_grid *grid, const void *gamma,
                                   const double *quad_w, int k, int oversample, int power_iters, uint64_t seed,
                                   double *evals, void *efuns, double *fve) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (!gamma || !evals || !efuns) return set_error(FPCA_ERR_INVALID_ARG, "gamma, evals and efuns are required");
  if (k < 1 || oversample < 0 || power_iters < 0)
    return set_error(FPCA_ERR_INVALID_ARG, "need k >= 1, oversample >= 0, power_iters >= 0");
  if (k + oversample > 64 || k + oversample > P)
    return set_error(FPCA_ERR_INVALID_ARG, "k + oversample = %d must be <= min(64, P)", k + oversample);
  if (dtype == FPCA_F64 && prec != FPCA_PREC_F64) return set_error(FPCA_ERR_UNSUPPORTED, "dtype F64 needs prec F64");
  if (dtype == FPCA_F32 && prec != FPCA_PREC_F32) return set_error(FPCA_ERR_UNSUPPORTED, "dtype F32 needs prec F32");
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype");
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return eig_impl<double>(ctx, grid, P, static_cast<const double *>(gamma), quad_w, k, oversample, power_iters, seed,
                            evals, static_cast<double *>(efuns), fve);
  return eig_impl<float>(ctx, grid, P, static_cast<const float *>(gamma), quad_w, k, oversample, power_iters, seed,
                         evals, static_cast<float *>(efuns), fve);
}

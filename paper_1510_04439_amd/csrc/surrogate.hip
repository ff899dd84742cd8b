// Bandwidth surrogate: summary features of the binned arrays and a small MLP
// (32 -> 128 GELU -> 128 GELU -> 1) that predicts log h of the covariance
// smoother, with hand-written forward, backward and Adam kernels. The
// cross-validation of this library supplies its training labels and remains
// the fallback selector.
#include <cmath>

#include "common.hpp"

namespace fpca {
namespace {

constexpr int NF = 32;    // features
constexpr int NH = 128;   // hidden width
constexpr int NLAG = 8;   // variogram lags per direction
// parameter layout: W1[NH][NF] b1[NH] W2[NH][NH] b2[NH] W3[NH] b3[1]
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == 20865, "parameter count");

// ------------------------------------------------------------------ features
// Accumulators (FP64): [0] sum C, [1] sum G, [2] sum Q, [3] count C > 0,
// [4] sum C diag, [5] sum G diag, [6..6+NLAG) C along coordinate 0 at lag l,
// then G, then the same along the last coordinate.
constexpr int ACC_N = 6 + 4 * NLAG;

__global__ __launch_bounds__(256) void k_feat_cov(GridDims g, const float *__restrict__ C, const float *__restrict__ G,
                                                   const float *__restrict__ Q, double *__restrict__ acc) {
  __shared__ double sh[ACC_N];
  for (int i = threadIdx.x; i < ACC_N; i += blockDim.x) sh[i] = 0.0;
  __syncthreads();
  double loc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t PP = g.P * g.P;
  const int dl = g.d - 1;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < PP; e += int64_t(gridDim.x) * blockDim.x) {
    const double c = C[e], gv = G[e];
    loc[0] += c;
    loc[1] += gv;
    if (Q) loc[2] += Q[e];
    loc[3] += c > 0.0 ? 1.0 : 0.0;
    const int64_t p = e / g.P, q = e % g.P;
    if (p == q) {
      loc[4] += c;
      loc[5] += gv;
      continue;
    }
    // which coordinates differ, and by how much
    int ndiff = 0, kd = -1, lag = 0;
    int64_t rp = p, rq = q;
    for (int k = g.d - 1; k >= 0; --k) {
      const int a = int(rp % g.M[k]), b = int(rq % g.M[k]);
      rp /= g.M[k];
      rq /= g.M[k];
      if (a != b) {
        ++ndiff;
        kd = k;
        lag = a > b ? a - b : b - a;
      }
    }
    // lags along the first and along the last coordinate (the same one when d = 1)
    if (ndiff == 1 && lag <= NLAG) {
      if (kd == 0) {
        atomicAdd(&sh[6 + lag - 1], c);
        atomicAdd(&sh[6 + NLAG + lag - 1], gv);
      }
      if (kd == dl) {
        atomicAdd(&sh[6 + 2 * NLAG + lag - 1], c);
        atomicAdd(&sh[6 + 3 * NLAG + lag - 1], gv);
      }
    }
  }
  for (int i = 0; i < 6; ++i) {
    double v = loc[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(&sh[i], v);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ACC_N; i += blockDim.x) atomicAdd(&acc[i], sh[i]);
}

// One workgroup: curve-size statistics, mean-bin statistics and the final
// feature vector.
__global__ __launch_bounds__(256) void k_feat_final(GridDims g, int64_t n, const int64_t *__restrict__ off,
                                                     const float *__restrict__ c, const float *__restrict__ s,
                                                     const float *__restrict__ s2, const double *__restrict__ acc,
                                                     int haveQ, float *__restrict__ feat) {
  __shared__ double red[8][4];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // v0 sum N, v1 sum N^2, v2 sum N(N-1), v3 max N
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double Ni = double(off[i + 1] - off[i]);
    v[0] += Ni;
    v[1] += Ni * Ni;
    v[2] += Ni * (Ni - 1.0);
    v[3] = fmax(v[3], Ni);
  }
  // v4 sum c, v5 sum c^2, v6 sum s, v7 sum s2
  for (int64_t p = threadIdx.x; p < g.P; p += blockDim.x) {
    v[4] += c[p];
    v[5] += double(c[p]) * c[p];
    v[6] += s[p];
    v[7] += s2 ? double(s2[p]) : 0.0;
  }
  for (int i = 0; i < 8; ++i) {
    double x = v[i];
    for (int o = 32; o > 0; o >>= 1) x = (i == 3) ? fmax(x, __shfl_xor(x, o)) : x + __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) red[i][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double t[8];
  for (int i = 0; i < 8; ++i)
    t[i] = (i == 3) ? fmax(fmax(red[i][0], red[i][1]), fmax(red[i][2], red[i][3]))
                    : (red[i][0] + red[i][1]) + (red[i][2] + red[i][3]);
  const double tiny = 1e-30;
  const double nn = double(n > 0 ? n : 1);
  const double meanN = t[0] / nn;
  const double sdN = sqrt(fmax(t[1] / nn - meanN * meanN, 0.0));
  const double EY2 = t[7] / fmax(t[4], tiny);
  const double EY = t[6] / fmax(t[4], tiny);
  const double g0 = acc[5] / fmax(acc[4], tiny);
  const double gbar = acc[1] / fmax(acc[0], tiny);
  const double qbar = acc[2] / fmax(acc[0], tiny);
  float f[NF];
  f[0] = float(log(nn));
  f[1] = float(log(fmax(meanN, 1.0)));
  f[2] = float(log(fmax(t[2], 1.0)));
  f[3] = float(sdN / fmax(meanN, tiny));
  f[4] = float(log(double(g.P)));
  f[5] = float(t[4] * t[4] / fmax(double(g.P) * t[5], tiny));
  f[6] = float(acc[3] / (double(g.P) * double(g.P)));
  f[7] = float(log(fmax(EY2, tiny)));
  f[8] = float(EY * EY / fmax(EY2, tiny));
  f[9] = float(log(fmax(fabs(g0), tiny)));
  f[10] = float((EY2 - g0) / fmax(EY2, tiny));
  f[11] = haveQ ? float(log(fmax(qbar - gbar * gbar, tiny))) : 0.f;
  const double gs = fabs(g0) > tiny ? g0 : tiny;
  double g1[NLAG], g2[NLAG];
  for (int l = 0; l < NLAG; ++l) {
    g1[l] = acc[6 + NLAG + l] / fmax(acc[6 + l], tiny);
    g2[l] = acc[6 + 3 * NLAG + l] / fmax(acc[6 + 2 * NLAG + l], tiny);
    f[12 + l] = float(g1[l] / gs);
    f[20 + l] = float(g2[l] / gs);
  }
  f[28] = float((g1[1] - 2.0 * g1[0] + g0) / gs);
  f[29] = float((g2[1] - 2.0 * g2[0] + g0) / gs);
  f[30] = float(log(fmax(acc[0] / (double(g.P) * double(g.P)), tiny)));
  f[31] = float(log(1.0 / double(g.M[0] - 1)));
  for (int i = 0; i < NF; ++i) feat[i] = f[i];
}

// ------------------------------------------------------------------ MLP
__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float phi = 0.39894228040143268f * expf(-0.5f * z * z);
  return Phi + z * phi;
}

// One workgroup (NH threads) per sample. x is standardized on the fly:
// (feat - mu) / sd. Saves z1, z2 (pre-activations) for the backward pass.
__global__ __launch_bounds__(NH) void k_mlp_fwd(int B, const float *__restrict__ feat, const float *__restrict__ fmu,
                                                 const float *__restrict__ fsd, const float *__restrict__ prm,
                                                 float *__restrict__ out, float *__restrict__ z1s,
                                                 float *__restrict__ z2s) {
  __shared__ float x[NF], h1[NH], red[2];
  const int b = blockIdx.x, j = threadIdx.x;
  if (j < NF) x[j] = (feat[int64_t(b) * NF + j] - fmu[j]) / fsd[j];
  __syncthreads();
  float z = prm[OFF_B1 + j];
  for (int i = 0; i < NF; ++i) z = fmaf(prm[OFF_W1 + j * NF + i], x[i], z);
  if (z1s) z1s[int64_t(b) * NH + j] = z;
  h1[j] = gelu(z);
  __syncthreads();
  float z2 = prm[OFF_B2 + j];
  for (int i = 0; i < NH; ++i) z2 = fmaf(prm[OFF_W2 + j * NH + i], h1[i], z2);
  if (z2s) z2s[int64_t(b) * NH + j] = z2;
  float o = prm[OFF_W3 + j] * gelu(z2);
  for (int s = 32; s > 0; s >>= 1) o += __shfl_xor(o, s);
  if ((j & 63) == 0) red[j >> 6] = o;
  __syncthreads();
  if (j == 0) out[b] = red[0] + red[1] + prm[OFF_B3];
}

// Per sample: the loss terms and the back-propagated deltas
//   dout = 2 (out - y) / B,  dz2 = W3 dout gelu'(z2),  dz1 = W2^T dz2 gelu'(z1).
__global__ __launch_bounds__(NH) void k_mlp_delta(int B, const float *__restrict__ prm, const float *__restrict__ out,
                                                   const float *__restrict__ target, const float *__restrict__ z1s,
                                                   const float *__restrict__ z2s, float *__restrict__ dz1s,
                                                   float *__restrict__ dz2s, float *__restrict__ dout_s) {
  __shared__ float dz2[NH];
  const int b = blockIdx.x, j = threadIdx.x;
  const float dout = 2.0f * (out[b] - target[b]) / float(B);
  if (j == 0) dout_s[b] = dout;
  const float d2 = prm[OFF_W3 + j] * dout * gelu_grad(z2s[int64_t(b) * NH + j]);
  dz2[j] = d2;
  dz2s[int64_t(b) * NH + j] = d2;
  __syncthreads();
  float dh1 = 0.f;
  for (int k = 0; k < NH; ++k) dh1 = fmaf(prm[OFF_W2 + k * NH + j], dz2[k], dh1);
  dz1s[int64_t(b) * NH + j] = dh1 * gelu_grad(z1s[int64_t(b) * NH + j]);
}

// Thread per parameter: the gradient summed over the batch in a fixed order.
__global__ __launch_bounds__(256) void k_mlp_grad(int B, const float *__restrict__ feat, const float *__restrict__ fmu,
                                                   const float *__restrict__ fsd, const float *__restrict__ z1s,
                                                   const float *__restrict__ z2s, const float *__restrict__ dz1s,
                                                   const float *__restrict__ dz2s, const float *__restrict__ dout_s,
                                                   float *__restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float s = 0.f;
  if (p < OFF_B1) {
    const int j = p / NF, i = p % NF;
    for (int b = 0; b < B; ++b) s += dz1s[int64_t(b) * NH + j] * ((feat[int64_t(b) * NF + i] - fmu[i]) / fsd[i]);
  } else if (p < OFF_W2) {
    const int j = p - OFF_B1;
    for (int b = 0; b < B; ++b) s += dz1s[int64_t(b) * NH + j];
  } else if (p < OFF_B2) {
    const int j = (p - OFF_W2) / NH, i = (p - OFF_W2) % NH;
    for (int b = 0; b < B; ++b) s += dz2s[int64_t(b) * NH + j] * gelu(z1s[int64_t(b) * NH + i]);
  } else if (p < OFF_W3) {
    const int j = p - OFF_B2;
    for (int b = 0; b < B; ++b) s += dz2s[int64_t(b) * NH + j];
  } else if (p < OFF_B3) {
    const int j = p - OFF_W3;
    for (int b = 0; b < B; ++b) s += dout_s[b] * gelu(z2s[int64_t(b) * NH + j]);
  } else {
    for (int b = 0; b < B; ++b) s += dout_s[b];
  }
  grad[p] = s;
}

// Adam (Kingma & Ba 2015) with decoupled weight decay.
__global__ void k_adam(int np, float *__restrict__ prm, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / c1, vh = vv / c2;
  prm[p] -= lr * (mh / (sqrtf(vh) + eps) + wd * prm[p]);
}

}  // namespace
}  // namespace fpca

using namespace fpca;

extern "C" {

int fpca_bw_num_params(void) { return NPARAM; }

int fpca_bw_features(fpca_handle ctx, const fpca_grid *grid, int64_t n, const int64_t *offsets, const float *c,
                     const float *s, const float *s2, const float *C, const float *G, const float *Q, float *feat) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (n < 1 || !offsets || !c || !s || !C || !G || !feat)
    return set_error(FPCA_ERR_INVALID_ARG, "n >= 1, offsets, c, s, C, G and feat are required");
  if (int rc = set_device(ctx)) return rc;
  const GridDims gd = make_dims(grid);
  if (int rc = ws3_reserve(ctx, carve_bytes(64, 8))) return rc;
  double *acc = static_cast<double *>(ctx->ws3);
  if (int rc = fill_f64(ctx, acc, 0.0, ACC_N)) return rc;
  int64_t blocks = (P * P + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_feat_cov, dim3(unsigned(blocks)), dim3(256), 0, ctx->stream, gd, C, G, Q, acc);
  FPCA_LAUNCH_CHECK("feat_cov");
  hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(256), 0, ctx->stream, gd, n, offsets, c, s, s2, acc, Q ? 1 : 0, feat);
  FPCA_LAUNCH_CHECK("feat_final");
  return FPCA_OK;
}

int fpca_bw_mlp_forward(fpca_handle ctx, int batch, const float *feat, const float *feat_mean, const float *feat_sd,
                        const float *params, float *out, float *z1, float *z2) {
  if (int rc = check_handle(ctx)) return rc;
  if (batch < 1 || !feat || !feat_mean || !feat_sd || !params || !out)
    return set_error(FPCA_ERR_INVALID_ARG, "batch >= 1 and feat, feat_mean, feat_sd, params, out are required");
  if ((z1 == nullptr) != (z2 == nullptr)) return set_error(FPCA_ERR_INVALID_ARG, "z1 and z2 go together");
  if (int rc = set_device(ctx)) return rc;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(unsigned(batch)), dim3(NH), 0, ctx->stream, batch, feat, feat_mean, feat_sd,
                     params, out, z1, z2);
  FPCA_LAUNCH_CHECK("mlp_fwd");
  return FPCA_OK;
}

int fpca_bw_mlp_backward(fpca_handle ctx, int batch, const float *feat, const float *feat_mean, const float *feat_sd,
                         const float *params, const float *out, const float *target, const float *z1,
                         const float *z2, float *work, float *grad) {
  if (int rc = check_handle(ctx)) return rc;
  if (batch < 1 || !feat || !feat_mean || !feat_sd || !params || !out || !target || !z1 || !z2 || !work || !grad)
    return set_error(FPCA_ERR_INVALID_ARG, "all arguments are required");
  if (int rc = set_device(ctx)) return rc;
  float *dz1 = work, *dz2 = work + int64_t(batch) * NH, *dout = work + 2 * int64_t(batch) * NH;
  hipLaunchKernelGGL(k_mlp_delta, dim3(unsigned(batch)), dim3(NH), 0, ctx->stream, batch, params, out, target, z1, z2,
                     dz1, dz2, dout);
  FPCA_LAUNCH_CHECK("mlp_delta");
  hipLaunchKernelGGL(k_mlp_grad, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx->stream, batch, feat, feat_mean, feat_sd,
                     z1, z2, dz1, dz2, dout, grad);
  FPCA_LAUNCH_CHECK("mlp_grad");
  return FPCA_OK;
}

int fpca_bw_adam_step(fpca_handle ctx, int step, float lr, float beta1, float beta2, float eps, float weight_decay,
                      float *params, const float *grad, float *m, float *v) {
  if (int rc = check_handle(ctx)) return rc;
  if (step < 1 || !params || !grad || !m || !v) return set_error(FPCA_ERR_INVALID_ARG, "step >= 1 and buffers required");
  if (int rc = set_device(ctx)) return rc;
  const float c1 = 1.0f - powf(beta1, float(step)), c2 = 1.0f - powf(beta2, float(step));
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx->stream, NPARAM, params, grad, m, v, lr,
                     beta1, beta2, eps, weight_decay, c1, c2);
  FPCA_LAUNCH_CHECK("adam");
  return FPCA_OK;
}

}  // extern "C"

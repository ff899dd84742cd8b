// Fused covariance smoother for d = 2 on a complete common grid (eq. 2.4 on
// the 4-dimensional grid of (s1, s2, t1, t2)), in two kernels:
//
//  stage T: one workgroup per s-row of G (a whole t-plane, held in LDS): the
//           t2 and t1 passes produce the partial moments G00, G10, G01
//           (t-exponents).
//  stage S: a workgroup owns 4 consecutive t columns, one wavefront per
//           column, lane = s2. It streams the s1 rows of the partial moments
//           through LDS (double-buffered), does the s2 pass of each row from
//           LDS, keeps the last 2R+1 results in a register window for the
//           s1 pass, and forms b0 per lane: in closed form for nodes whose
//           s- and t-windows share no grid node (the weight moments are then
//           products of 1-D sums), by an FP64 solve after the row loop for
//           the near-diagonal nodes (their response moments wait in LDS).
//           Only nodes p <= q are computed (the surface is symmetric); each
//           is written at (p,q) and (q,p) with mu(p)mu(q) subtracted and the
//           domain mask applied.
//
// The pair weights are c0 (1 - delta_pq), so the 15 weight moments are exact
// products of 1-D tap sums minus the diagonal part, evaluated in FP64 from
// small tables; only G is convolved (FP32). These systems are those of a
// complete design, well conditioned at every node; general pair weights go
// through the FP64 engine, whose windows may be nearly degenerate.
#include <cmath>

#include "common.hpp"
#include "wls.hpp"

namespace fpca {

namespace {

constexpr int RMAX = 8;
constexpr int TW = 4;  // t columns per stage-S workgroup (one per wavefront)
constexpr int ST = 64 * TW;  // threads of a stage-S workgroup
constexpr int CPL = 32 / TW;  // stage-S chunks whose t columns share a 128-byte line

struct Taps {
  float k[3][2 * RMAX + 1];  // (1-u^2)u^j at offsets -R..R
};

// Analytic weight-moment tables (FP64), per coordinate k = 0, 1 of the d = 2 grid:
//   W[k][e][x]      = sum over the window at x of (1-u^2) u^e           (e = 0,1,2)
//   Dg[k][ab][i][j] = sum_y (1-u_i^2) u_i^a (1-u_j^2) u_j^b, u_i = (y-i)/H
// with ab over (0,0),(1,0),(0,1),(2,0),(1,1),(0,2).
struct TabPtrs {
  const double *W;   // [2][3][Mmax]
  const double *Dg;  // [2][6][Mmax][Mmax]
  const double *Xc;  // [Mmax][4]: per s1 node of the tensor-product fit: 1/W0, m/v, m^2/v, pivot test passed
  int Mmax;
};

__device__ inline int ab_index(int a, int b) {
  // (0,0)0 (1,0)1 (0,1)2 (2,0)3 (1,1)4 (0,2)5
  if (a == 0 && b == 0) return 0;
  if (a == 1 && b == 0) return 1;
  if (a == 0 && b == 1) return 2;
  if (a == 2) return 3;
  if (a == 1) return 4;
  return 5;
}

__global__ void k_tables(int M0, int M1, double H0, double H1, int R0, int R1, int Mmax, double *W, double *Dg,
                         double *Xc) {
  const int k = blockIdx.y;
  const int M = k == 0 ? M0 : M1;
  const double H = k == 0 ? H0 : H1;
  const int R = k == 0 ? R0 : R1;
  // u = m / H for the offsets m = -R .. R (R <= RMAX), divided once per workgroup
  __shared__ double uo[2 * RMAX + 1];
  if (int(threadIdx.x) <= 2 * R) uo[threadIdx.x] = double(int(threadIdx.x) - R) / H;
  __syncthreads();
  if (k == 0) {
    // the first coordinate's factors of the tensor-product fit (m = W1/W0,
    // e = W2/W0, v = e - m^2), one node per thread
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < Mmax; x += gridDim.x * blockDim.x) {
      double w[3] = {0.0, 0.0, 0.0};
      if (x < M)
        for (int m = -R; m <= R; ++m) {
          if (x + m < 0 || x + m >= M) continue;
          const double u = uo[m + R];
          const double K = fabs(u) < 1.0 ? 1.0 - u * u : 0.0;
          w[0] += K;
          w[1] += K * u;
          w[2] += K * u * u;
        }
      const double r0 = w[0] > 0.0 ? 1.0 / w[0] : 0.0;
      const double mx = w[1] * r0, ex = w[2] * r0, vx = ex - mx * mx;
      const bool ok = ex > 0.0 && vx >= 1e-10 * ex;
      const double ax = ok ? mx / vx : 0.0;
      Xc[4 * x + 0] = r0;
      Xc[4 * x + 1] = ax;
      Xc[4 * x + 2] = mx * ax;
      Xc[4 * x + 3] = ok ? 1.0 : 0.0;
    }
  }
  const int64_t nW = 3 * int64_t(Mmax), nD = 6 * int64_t(Mmax) * Mmax;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nW + nD; e += int64_t(gridDim.x) * blockDim.x) {
    if (e < nW) {
      const int ex = int(e / Mmax), x = int(e % Mmax);
      double s = 0.0;
      if (x < M)
        for (int m = -R; m <= R; ++m) {
          if (x + m < 0 || x + m >= M) continue;
          const double u = uo[m + R];
          const double K = fabs(u) < 1.0 ? 1.0 - u * u : 0.0;
          s += K * (ex == 0 ? 1.0 : (ex == 1 ? u : u * u));
        }
      W[int64_t(k) * nW + e] = s;
    } else {
      const int64_t f = e - nW;
      const int ab = int(f / (int64_t(Mmax) * Mmax));
      const int i = int((f / Mmax) % Mmax), j = int(f % Mmax);
      const int a = (ab == 1 || ab == 4) ? 1 : (ab == 3 ? 2 : 0);
      const int b = (ab == 2 || ab == 4) ? 1 : (ab == 5 ? 2 : 0);
      double s = 0.0;
      // only nodes within R of both i and j contribute
      if (i < M && j < M)
        for (int y = max(0, max(i, j) - R); y <= min(M - 1, min(i, j) + R); ++y) {
          const double ui = uo[y - i + R], uj = uo[y - j + R];
          const double Ki = fabs(ui) < 1.0 ? 1.0 - ui * ui : 0.0;
          const double Kj = fabs(uj) < 1.0 ? 1.0 - uj * uj : 0.0;
          if (Ki == 0.0 || Kj == 0.0) continue;
          s += Ki * (a == 0 ? 1.0 : (a == 1 ? ui : ui * ui)) * Kj * (b == 0 ? 1.0 : (b == 1 ? uj : uj * uj));
        }
      Dg[int64_t(k) * nD + f] = s;
    }
  }
}

// ---------------------------------------------------------------- stage T
// U layout: 3 arrays of P x P (row s, column t): G00, G10, G01 (exponents of
// u in (t1, t2)).
template <int R>
__global__ __launch_bounds__(512) void k_stage_t(int M1, int M2, int64_t P, const float *__restrict__ G, Taps tp,
                                                  float *__restrict__ U) {
  constexpr int NB = 4;  // consecutive outputs per thread
  constexpr int WIN = NB + 2 * R;
  extern __shared__ float lds[];
  const int LD = M2 + 1;  // padded t-plane row: both passes are bank-conflict free
  const int plane = M1 * LD;
  float *rowG = lds;
  float *A = lds + plane;  // t2-pass planes GK, GU
  const int64_t s = blockIdx.x;
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < P; e += blockDim.x) {
    const int t1 = int(e / M2), t2 = int(e % M2);
    rowG[t1 * LD + t2] = G[s * P + e];
  }
  __syncthreads();
  // t2 pass: thread -> (strip of NB outputs along t2, line t1), t1 fastest
  const int nst2 = (M2 + NB - 1) / NB;
  for (int sidx = tid; sidx < nst2 * M1; sidx += blockDim.x) {
    const int t1 = sidx % M1, t20 = (sidx / M1) * NB;
    float wg[WIN];
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
      const int t2 = t20 - R + i;
      wg[i] = (t2 >= 0 && t2 < M2) ? rowG[t1 * LD + t2] : 0.f;
    }
#pragma unroll
    for (int o = 0; o < NB; ++o) {
      float gk = 0.f, gu = 0.f;
#pragma unroll
      for (int m = 0; m <= 2 * R; ++m) {
        gk = fmaf(tp.k[0][m], wg[o + m], gk);
        gu = fmaf(tp.k[1][m], wg[o + m], gu);
      }
      if (t20 + o < M2) {
        const int e = t1 * LD + t20 + o;
        A[e] = gk;
        A[plane + e] = gu;
      }
    }
  }
  __syncthreads();
  // t1 pass: thread -> (t2, strip of NB outputs along t1), t2 fastest; results to HBM row s
  const int64_t PP = P * P;
  const int nst1 = (M1 + NB - 1) / NB;
  for (int sidx = tid; sidx < nst1 * M2; sidx += blockDim.x) {
    const int t2 = sidx % M2, t10 = (sidx / M2) * NB;
    float out[3][NB];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int o = 0; o < NB; ++o) out[q][o] = 0.f;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      float w[WIN];
#pragma unroll
      for (int i = 0; i < WIN; ++i) {
        const int t1 = t10 - R + i;
        w[i] = (t1 >= 0 && t1 < M1) ? A[a * plane + t1 * LD + t2] : 0.f;
      }
#pragma unroll
      for (int o = 0; o < NB; ++o)
#pragma unroll
        for (int m = 0; m <= 2 * R; ++m) {
          const float v = w[o + m];
          // GK -> G00, G10; GU -> G01
          if (a == 0) {
            out[0][o] = fmaf(tp.k[0][m], v, out[0][o]);
            out[1][o] = fmaf(tp.k[1][m], v, out[1][o]);
          } else {
            out[2][o] = fmaf(tp.k[0][m], v, out[2][o]);
          }
        }
    }
#pragma unroll
    for (int o = 0; o < NB; ++o) {
      if (t10 + o >= M1) continue;
      float *u = U + s * P + int64_t(t10 + o) * M2 + t2;
#pragma unroll
      for (int q = 0; q < 3; ++q) u[q * PP] = out[q][o];
    }
  }
}

// ---------------------------------------------------------------- stage S
template <int R>
__global__ __launch_bounds__(ST) void k_stage_s(int M1, int M2, int64_t P, const float *__restrict__ U, Taps tp,
                                                  const float *__restrict__ mu, const uint8_t *__restrict__ mask,
                                                  double c0, TabPtrs tab, int nchunks, float *__restrict__ gamma,
                                                  int8_t *__restrict__ status) {
  constexpr int NU = 3;
  constexpr int W = 2 * R + 1;
  // Staged input row (double-buffered); rows s2 = -R .. 63 + R of it (R zero
  // rows at both ends) so that the s2 pass reads its 2R+1 neighbours
  // without tests.
  constexpr int SW = 64 + 2 * R;
  __shared__ float stage[2][NU][SW][TW + 1];
  // response moments of the near-diagonal nodes, per wavefront: rows
  // t1-2R .. t1, lanes t2-2R .. t2+2R
  __shared__ float nearT[TW][2 * R + 1][4 * R + 1][5];
  // The row loop's transposed writes (Gamma(p, t) for the TW columns t of the
  // workgroup) gathered per output row, so that wavefront 0 writes each p's
  // TW consecutive values at once, one row later; status -1: not emitted.
  __shared__ float tq_v[2][64][TW];
  __shared__ int8_t tq_s[2][64][TW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Chunk order: the chunks sharing a 128-byte line of a row (CPL chunks of
  // TW floats) land on one XCD (dispatch is round-robin over 8 XCDs), and the
  // chunks with the most work (largest t1) come first.
  int chunk;
  {
    const int b = blockIdx.x;
    const int nlines = (nchunks + CPL - 1) / CPL;
    const int L = (b / (8 * CPL)) * 8 + (b % 8);
    const int sib = (b / 8) % CPL;
    int line = nlines - 1 - L;
    chunk = line * CPL + sib;
    if (L >= nlines || chunk >= nchunks || chunk < 0) chunk = -1;
  }
  if (chunk < 0) return;  // uniform across the workgroup
  const int64_t t0 = int64_t(chunk) * TW;
  const int64_t t = t0 + wave;
  const bool wave_ok = t < P;
  const int t1 = wave_ok ? int(t / M2) : -1;
  const int t2 = wave_ok ? int(t % M2) : 0;
  // last output row of any wave in this workgroup
  int xmax = int(min(int64_t(P - 1), t0 + TW - 1) / M2);
  const int64_t PP = P * P;

  // Per-lane factors of the analytic weight moments: window sums W[e] of
  // the s2, t1 and t2 coordinates and the diagonal-overlap sums Dg[ab] of
  // the second grid coordinate at (s2, t2). Loaded where needed (before and
  // after the row loop), so they hold no registers during it.
  auto load_factors = [&](double *ws2, double *wt1, double *wt2, double *dg2) {
    const int Mm = tab.Mmax;
    const double *W1 = tab.W, *W2 = tab.W + 3 * Mm;
    const double *D2 = tab.Dg + 6 * int64_t(Mm) * Mm;
    const int s2 = lane < M2 ? lane : 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      ws2[e] = W2[e * Mm + s2];
      wt1[e] = W1[e * Mm + (t1 < 0 ? 0 : t1)];
      wt2[e] = W2[e * Mm + t2];
    }
    if (dg2)
#pragma unroll
      for (int ab = 0; ab < 6; ++ab) dg2[ab] = D2[(int64_t(ab) * Mm + s2) * Mm + t2];
  };
  // Tensor-product design (windows of s and t that share no node): with
  // per-coordinate window sums W0, W1, W2, m = W1/W0, e = W2/W0, v = e - m^2,
  // the fit's centered second-moment matrix is diagonal and
  //   b0 = [T0 (1 + sum_k m_k^2/v_k) - sum_k (m_k/v_k) T1_k] / S0,
  // with the pivots of the scaled system equal to v_k / e_k. The s2, t1, t2
  // parts are fixed per lane; the s1 part is added per row.
  double tz_c = 0.0, tz_a[3] = {0.0, 0.0, 0.0}, tz_inv = 0.0;
  bool tz_ok = true;
  {
    double ws2[3], wt1[3], wt2[3];
    load_factors(ws2, wt1, wt2, nullptr);
    const double *tb[3] = {ws2, wt1, wt2};
    double prod = c0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double w0 = tb[k][0], mk = tb[k][1] / w0, ek = tb[k][2] / w0;
      const double vk = ek - mk * mk;
      tz_ok = tz_ok && ek > 0.0 && vk >= 1e-10 * ek;
      tz_a[k] = mk / vk;
      tz_c += mk * tz_a[k];
      prod *= w0;
    }
    tz_inv = 1.0 / prod;
  }

  // s2-pass results of the last W input rows (the s1 window, oldest first):
  //   0: K*U0, 1: uK*U0, 2: K*U1, 3: K*U2 along s2
  constexpr int NA = 4;
  float win[NA][W];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int i = 0; i < W; ++i) win[a][i] = 0.f;
  for (int e = tid; e < 2 * NU * SW * (TW + 1); e += ST) (&stage[0][0][0][0])[e] = 0.f;
  for (int e = tid; e < 2 * 64 * TW; e += ST) (&tq_s[0][0][0])[e] = -1;

  // Each thread stages NU values per row (64 s2 x TW t per array);
  // the next row is fetched into registers while the current one is used.
  static_assert(64 * TW == ST, "one staged value per thread and array");
  const int ls2 = tid / TW, ltt = tid % TW;
  const bool lok = ls2 < M2 && t0 + ltt < P;
  float pre[NU];
  auto fetch = [&](int r) {
#pragma unroll
    for (int a = 0; a < NU; ++a)
      pre[a] = (r < M1 && lok) ? U[a * PP + (int64_t(r) * M2 + ls2) * P + t0 + ltt] : 0.f;
  };
  // Gamma(p,t) = Gamma(t,p) = b0 - mu_p mu_t (0 outside the domain), status at both.
  // eb >= 0: the transposed write goes through tq_v / tq_s[eb] (row loop)
  auto emit = [&](int64_t p, double b0, int8_t st, int eb) {
    if (mu) b0 -= double(mu[p]) * double(mu[t]);
    if (mask && (!mask[p] || !mask[t])) b0 = 0.0;
    const float v = float(b0);
    gamma[t * P + p] = v;
    if (status) status[t * P + p] = st;
    if (eb >= 0) {
      tq_v[eb][lane][wave] = v;
      tq_s[eb][lane][wave] = st;
    } else {
      gamma[p * P + t] = v;
      if (status) status[p * P + t] = st;
    }
  };
  // wavefront 0: the gathered transposed writes of output row x (buffer eb)
  const bool vec4 = P % TW == 0 && (reinterpret_cast<uintptr_t>(gamma) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(status) & 3) == 0;
  auto flush = [&](int eb, int x) {
    if (x < 0 || lane >= M2) return;
    const int64_t p = int64_t(x) * M2 + lane;
    float v[TW];
    int8_t sv[TW];
    bool all = true, any = false;
#pragma unroll
    for (int w = 0; w < TW; ++w) {
      v[w] = tq_v[eb][lane][w];
      sv[w] = tq_s[eb][lane][w];
      all = all && sv[w] >= 0;
      any = any || sv[w] >= 0;
    }
    if (!any) return;
    float *g = gamma + p * P + t0;
    int8_t *sp = status ? status + p * P + t0 : nullptr;
    if (all && vec4) {
      static_assert(TW == 4, "one 16-byte and one 4-byte store per p");
      *reinterpret_cast<float4 *>(g) = make_float4(v[0], v[1], v[2], v[3]);
      if (sp)
        *reinterpret_cast<uint32_t *>(sp) = uint32_t(uint8_t(sv[0])) | (uint32_t(uint8_t(sv[1])) << 8) |
                                            (uint32_t(uint8_t(sv[2])) << 16) | (uint32_t(uint8_t(sv[3])) << 24);
    } else {
#pragma unroll
      for (int w = 0; w < TW; ++w)
        if (sv[w] >= 0) {
          g[w] = v[w];
          if (sp) sp[w] = sv[w];
        }
    }
  };
  const int rlast = xmax + R;  // last input row any wavefront needs
  fetch(0);
  __syncthreads();  // the zeroed padding rows
  for (int r = 0; r <= rlast; ++r) {
    const int buf = r & 1;
#pragma unroll
    for (int a = 0; a < NU; ++a) stage[buf][a][R + ls2][ltt] = pre[a];
    __syncthreads();
    if (r < rlast) fetch(r + 1);
    // the previous row's transposed writes; this row's slots start empty
    if (wave == 0) flush(buf ^ 1, r - 1 - R);
    tq_s[buf][lane][wave] = -1;
    // s2 pass of input row r (lanes = s2) from the staged row
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) {
      const float u0 = stage[buf][0][lane + i][wave];
      const float u1 = stage[buf][1][lane + i][wave];
      const float u2 = stage[buf][2][lane + i][wave];
      a0 = fmaf(tp.k[0][i], u0, a0);
      a1 = fmaf(tp.k[1][i], u0, a1);
      a2 = fmaf(tp.k[0][i], u1, a2);
      a3 = fmaf(tp.k[0][i], u2, a3);
    }
#pragma unroll
    for (int i = 0; i < W - 1; ++i) {
      win[0][i] = win[0][i + 1];
      win[1][i] = win[1][i + 1];
      win[2][i] = win[2][i + 1];
      win[3][i] = win[3][i + 1];
    }
    win[0][W - 1] = a0;
    win[1][W - 1] = a1;
    win[2][W - 1] = a2;
    win[3][W - 1] = a3;
    const int x = r - R;
    if (x < 0 || !wave_ok || x > t1) continue;  // no output row for this wavefront
    // s1 pass over the window: input rows x-R .. x+R
    double m[20];
    {
      float T0 = 0.f, Ts1 = 0.f, Ts2 = 0.f, Tt1 = 0.f, Tt2 = 0.f;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        T0 = fmaf(tp.k[0][i], win[0][i], T0);
        Ts1 = fmaf(tp.k[1][i], win[0][i], Ts1);
        Ts2 = fmaf(tp.k[0][i], win[1][i], Ts2);
        Tt1 = fmaf(tp.k[0][i], win[2][i], Tt1);
        Tt2 = fmaf(tp.k[0][i], win[3][i], Tt2);
      }
      m[15] = T0;
      m[16] = Ts1;
      m[17] = Ts2;
      m[18] = Tt1;
      m[19] = Tt2;
    }
    if (lane >= M2) continue;
    const int64_t p = int64_t(x) * M2 + lane;
    if (p > t) continue;
    if (abs(x - t1) <= 2 * R && abs(lane - t2) <= 2 * R) {
      // near the s = t diagonal: solved after the row loop
      float *nq = nearT[wave][x - (t1 - 2 * R)][lane - (t2 - 2 * R)];
#pragma unroll
      for (int k = 0; k < 5; ++k) nq[k] = float(m[15 + k]);
      continue;
    }
    const double *xc = tab.Xc + 4 * x;  // 1/W0, m/v, m^2/v, ok of row x
    const double inv = tz_inv * xc[0];
    if (tz_ok && xc[3] != 0.0) {
      emit(p, (m[15] * (1.0 + tz_c + xc[2]) - xc[1] * m[16] - tz_a[0] * m[17] - tz_a[1] * m[18] -
               tz_a[2] * m[19]) * inv,
           FPCA_STATUS_OK, buf);
    } else {
      emit(p, m[15] * inv, FPCA_STATUS_FALLBACK, buf);
    }
  }
  __syncthreads();
  if (wave == 0) flush(rlast & 1, rlast - R);

  // Nodes whose s- and t-windows share grid nodes (|s1 - t1| <= 2R and
  // |s2 - t2| <= 2R): the diagonal exclusion couples s and t, full system.
  if (!wave_ok) return;
  double ws2[3], wt1[3], wt2[3], dg2[6];
  load_factors(ws2, wt1, wt2, dg2);
  const int dl = lane - (t2 - 2 * R);
  for (int x = max(0, t1 - 2 * R); x <= t1; ++x) {
    if (lane >= M2 || dl < 0 || dl > 4 * R) continue;
    const int64_t p = int64_t(x) * M2 + lane;
    if (p > t) continue;
    const int Mm = tab.Mmax;
    const double *W1 = tab.W, *D1 = tab.Dg;
    const double wx[3] = {W1[x], W1[Mm + x], W1[2 * Mm + x]};
    auto d1 = [&](int a1, int b1) { return D1[(int64_t(ab_index(a1, b1)) * Mm + x) * Mm + t1]; };
    // moment q has u-exponents (a1, a2, b1, b2) in (s1, s2, t1, t2)
    const int E[15][4] = {{0, 0, 0, 0}, {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1},
                          {2, 0, 0, 0}, {1, 1, 0, 0}, {1, 0, 1, 0}, {1, 0, 0, 1}, {0, 2, 0, 0},
                          {0, 1, 1, 0}, {0, 1, 0, 1}, {0, 0, 2, 0}, {0, 0, 1, 1}, {0, 0, 0, 2}};
    double m[20];
#pragma unroll
    for (int mq = 0; mq < 15; ++mq) {
      const double af = ws2[E[mq][1]] * wt1[E[mq][2]] * wt2[E[mq][3]];
      m[mq] = c0 * (wx[E[mq][0]] * af - d1(E[mq][0], E[mq][2]) * dg2[ab_index(E[mq][1], E[mq][3])]);
    }
    const float *nq = nearT[wave][x - (t1 - 2 * R)][dl];
#pragma unroll
    for (int k = 0; k < 5; ++k) m[15 + k] = nq[k];
    int8_t st;
    const double b0 = wls_b0<4>(m, &st);
    emit(p, b0, st, -1);
  }
}

int tap_radius(double h, int M) { return int(std::floor(h * double(M - 1))); }

}  // namespace

bool smooth_cov_fused_d2_supported(const fpca_grid *grid, const double *bw) {
  if (grid->d != 2) return false;
  const int M1 = grid->M[0], M2 = grid->M[1];
  if (M2 > 64 || int64_t(M1) * M2 > 4096) return false;
  const int R1 = tap_radius(bw[0], M1), R2 = tap_radius(bw[1], M2);
  if (R1 != R2 || R1 < 1 || R1 > RMAX) return false;
  // the same taps serve both coordinates
  if (std::fabs(bw[0] * (M1 - 1) - bw[1] * (M2 - 1)) > 1e-12 * bw[0] * (M1 - 1)) return false;
  return true;
}

int smooth_cov_fused_d2(fpca_context *ctx, const fpca_grid *grid, double c0, const float *G, const double *bw,
                        const float *mu, float *gamma, int8_t *status) {
  const int M1 = grid->M[0], M2 = grid->M[1];
  const int64_t P = int64_t(M1) * M2;
  const int R = tap_radius(bw[0], M1);
  const double H = bw[0] * double(M1 - 1);
  Taps tp{};
  for (int j = 0; j < 3; ++j)
    for (int m = -R; m <= R; ++m) {
      const double u = double(m) / H;
      const double K = std::fabs(u) < 1.0 ? 1.0 - u * u : 0.0;
      tp.k[j][m + R] = float(K * (j == 0 ? 1.0 : (j == 1 ? u : u * u)));
    }
  constexpr int NU = 3;
  const int Mmax = M1 > M2 ? M1 : M2;
  const size_t bytesU = carve_bytes(size_t(NU) * P * P, 4);
  const size_t bytesT = carve_bytes(2 * 3 * Mmax, 8) + carve_bytes(2 * 6 * size_t(Mmax) * Mmax, 8) +
                        carve_bytes(4 * size_t(Mmax), 8);
  if (int rc = ws_reserve(ctx, bytesU + bytesT)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  float *U = cv.take<float>(size_t(NU) * P * P);
  TabPtrs tab{nullptr, nullptr, nullptr, Mmax};
  double *Wt = cv.take<double>(2 * 3 * Mmax);
  double *Dt = cv.take<double>(2 * 6 * size_t(Mmax) * Mmax);
  double *Xt = cv.take<double>(4 * size_t(Mmax));
  const double H2 = bw[1] * double(M2 - 1);
  hipLaunchKernelGGL(k_tables, dim3(128, 2), dim3(256), 0, ctx->stream, M1, M2, H, H2, R, tap_radius(bw[1], M2), Mmax,
                     Wt, Dt, Xt);
  FPCA_LAUNCH_CHECK("tables");
  tab.W = Wt;
  tab.Dg = Dt;
  tab.Xc = Xt;
  const size_t lds_t = 3 * size_t(M1) * (M2 + 1) * sizeof(float);
#define STAGE_T(RR)                                                                                          \
  do {                                                                                                       \
    static int lds_set = 0; /* the attribute is set once per size (not inside a captured stream) */         \
    if (lds_set < int(lds_t)) {                                                                              \
      FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_stage_t<RR>),                          \
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_t)));                 \
      lds_set = int(lds_t);                                                                                  \
    }                                                                                                        \
    hipLaunchKernelGGL((k_stage_t<RR>), dim3(unsigned(P)), dim3(512), lds_t, ctx->stream, M1, M2, P, G, tp, U); \
  } while (0)
  switch (R) {
    case 1: STAGE_T(1); break;
    case 2: STAGE_T(2); break;
    case 3: STAGE_T(3); break;
    case 4: STAGE_T(4); break;
    case 5: STAGE_T(5); break;
    case 6: STAGE_T(6); break;
    case 7: STAGE_T(7); break;
    default: STAGE_T(8); break;
  }
#undef STAGE_T
  FPCA_LAUNCH_CHECK("stage_t");
  const int nchunks = int((P + TW - 1) / TW);
  const int nlines = (nchunks + CPL - 1) / CPL;
  const int grid_s = ((nlines + 7) / 8) * 8 * CPL;
#define STAGE_S(RR)                                                                                          \
  hipLaunchKernelGGL((k_stage_s<RR>), dim3(grid_s), dim3(ST), 0, ctx->stream, M1, M2, P, U, tp, mu, grid->mask, \
                     c0, tab, nchunks, gamma, status)
  switch (R) {
    case 1: STAGE_S(1); break;
    case 2: STAGE_S(2); break;
    case 3: STAGE_S(3); break;
    case 4: STAGE_S(4); break;
    case 5: STAGE_S(5); break;
    case 6: STAGE_S(6); break;
    case 7: STAGE_S(7); break;
    default: STAGE_S(8); break;
  }
#undef STAGE_S
  FPCA_LAUNCH_CHECK("stage_s");
  return FPCA_OK;
}

}  // namespace fpca

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

typedef double v4d __attribute__((ext_vector_type(4)));

// Four consecutive values as FP64 from one 16-byte (float) or two 16-byte
// (double) loads; the address is 16-byte aligned.
__device__ inline void load4(const float *p, double *o) {
  const float4 v = *reinterpret_cast<const float4 *>(p);
  o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
}
__device__ inline void load4(const double *p, double *o) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
  o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
}
constexpr int MB = 8;             // MFMA steps (4 nodes each) whose operands are loaded together

// Common grid: one wavefront's part of Phi^T Phi, the shared matrix of the
// curves observed at every node: the 16 x 16 tiles (0,0), (0,1), (1,1) over
// the nodes n0 .. n1-1 with FP64 MFMA (16 x 16 x 4: lane l carries
// Phi[16 tr + l % 16][node + l / 16] as the A operand and the same for tc as
// the B operand), the operands of MB steps loaded before they are used.
template <typename T, bool VEC>
__device__ inline void gram_wave(int64_t P, const T *__restrict__ efuns, int k, int64_t n0, int64_t n1, v4d &d00,
                                 v4d &d01, v4d &d11) {
  const int lane = threadIdx.x & 63;
  const int nt = k > 16 ? 2 : 1;
  const int row = lane & 15, kk = lane >> 4;
  const bool r0 = row < k, r1 = 16 + row < k;
  const T *f0p = efuns + int64_t(r0 ? row : 0) * P;
  const T *f1p = efuns + int64_t(r1 ? 16 + row : 0) * P;
  for (int64_t q = n0; q < n1; q += 4 * MB) {
    double f0[MB], f1[MB];
    if (VEC && q + 4 * MB <= n1) {
      // step 4b + j takes node q + 16 b + 4 kk + j: each lane's four nodes of
      // a 16-node block in one vector load
#pragma unroll
      for (int bl = 0; bl < MB / 4; ++bl) {
        const int64_t p = q + 16 * bl + 4 * kk;
        load4(f0p + p, f0 + 4 * bl);
        load4(f1p + p, f1 + 4 * bl);
      }
#pragma unroll
      for (int s = 0; s < MB; ++s) {
        f0[s] = r0 ? f0[s] : 0.0;
        f1[s] = r1 ? f1[s] : 0.0;
      }
    } else {
      // every load is issued (addresses clamped into the range), then masked
#pragma unroll
      for (int s = 0; s < MB; ++s) {
        const int64_t p = q + 16 * (s >> 2) + 4 * kk + (s & 3);
        const int64_t pc = min(p, n1 - 1);
        const double v0 = double(f0p[pc]), v1 = double(f1p[pc]);
        const bool in = p < n1;
        f0[s] = (in && r0) ? v0 : 0.0;
        f1[s] = (in && r1) ? v1 : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < MB; ++s) {
      d00 = __builtin_amdgcn_mfma_f64_16x16x4f64(f0[s], f0[s], d00, 0, 0, 0);
      if (nt > 1) {  // tile (1, 0) is the transpose of (0, 1)
        d01 = __builtin_amdgcn_mfma_f64_16x16x4f64(f0[s], f1[s], d01, 0, 0, 0);
        d11 = __builtin_amdgcn_mfma_f64_16x16x4f64(f1[s], f1[s], d11, 0, 0, 0);
      }
    }
  }
}

// Words of the LDS pool of k_pace_cg_rhs: workgroup 0 holds A (k x k + 1
// padding) and the two Gauss-Jordan buffers (k x 2k each), whose space first
// holds four slots of the Gram tiles; the other workgroups hold their
// wavefronts' tiles, the inverse and the right-hand sides.
constexpr int CG_A = PACE_KMAX * (PACE_KMAX + 1);
constexpr int CG_M = PACE_KMAX * 2 * PACE_KMAX;
constexpr int CG_POOL = CG_A + 2 * CG_M;
static_assert(4 * 3 * 256 <= 2 * CG_M, "the Gram slots fit in the Gauss-Jordan buffers");

constexpr int CG_NGW = 8;  // workgroups of k_pace_cg_rhs that form partial sums of Phi^T Phi

// Common grid: partial sums of Phi^T Phi (the shared matrix) over the share
// b of CG_NGW of the nodes, by the NT threads of one workgroup: its
// wavefronts take contiguous parts of that share (gram_wave), their tiles are
// added in a fixed order (wavefronts 4g + w into LDS slot w, g = 0, 1, ...,
// then the four slots) into part[b][tile].
template <typename T, bool VEC, int NT>
__device__ void cg_gram_part(int64_t P, const T *__restrict__ efuns, int k, int b, double *slot,
                             double *__restrict__ part) {
  constexpr int NW = NT / 64;
  static_assert(NW % 4 == 0, "wavefronts come in fours");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = lane & 15, kk = lane >> 4;
  constexpr int NWT = CG_NGW * NW;
  const int64_t per = ((P + NWT * 4 * MB - 1) / (NWT * 4 * MB)) * 4 * MB;  // nodes per wavefront
  const int64_t n0 = min(P, (int64_t(b) * NW + wave) * per), n1 = min(P, n0 + per);
  v4d d00 = {0, 0, 0, 0}, d01 = d00, d11 = d00;
  gram_wave<T, VEC>(P, efuns, k, n0, n1, d00, d01, d11);
  // D[i][j] of a tile sits in lane j + 16 (i % 4), element i / 4
  for (int g = 0; g < NW / 4; ++g) {
    if ((wave >> 2) == g) {
      double *sw = slot + (wave & 3) * 3 * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = (kk + 4 * v) * 16 + row;
        sw[e] = (g ? sw[e] : 0.0) + d00[v];
        sw[256 + e] = (g ? sw[256 + e] : 0.0) + d01[v];
        sw[512 + e] = (g ? sw[512 + e] : 0.0) + d11[v];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < 3 * 256; e += NT)
    part[int64_t(b) * 3 * 256 + e] = ((slot[e] + slot[768 + e]) + slot[1536 + e]) + slot[2304 + e];
}

// Common grid: the shared matrix Phi^T Phi + sigma^2 Lambda^{-1} from the
// CG_NGW partial sums (added in workgroup order) and its inverse, to Lout, by
// the NT threads of one workgroup.
template <int NT>
__device__ void cg_inverse(int k, const PaceDiag &dg, const double *__restrict__ part, double *pool,
                           double *__restrict__ Lout, int *__restrict__ ok) {
  const int tid = threadIdx.x;
  double *A = pool;                    // [PACE_KMAX][PACE_KMAX + 1]
  double *M0 = pool + CG_A;            // [PACE_KMAX][2 PACE_KMAX]
  double *M1 = M0 + CG_M;
  for (int e = tid; e < k * k; e += NT) {
    const int r = e / k, c = e % k;
    // the upper tiles only: entry (r, c) of tile (1, 0) is (c, r) of tile (0, 1)
    const int rr = (r >> 4) > (c >> 4) ? c : r, cc = (r >> 4) > (c >> 4) ? r : c;
    const int tr = rr >> 4, tc = cc >> 4;
    const int t = tr == 0 ? (tc == 0 ? 0 : 1) : 2;
    const int ei = (rr & 15) * 16 + (cc & 15);
    double v[CG_NGW];
#pragma unroll
    for (int b = 0; b < CG_NGW; ++b) v[b] = part[(int64_t(b) * 3 + t) * 256 + ei];
    double sum = 0.0;
#pragma unroll
    for (int b = 0; b < CG_NGW; ++b) sum += v[b];
    const bool kr = dg.v[r] >= 0.0, kc = dg.v[c] >= 0.0;
    A[r * (PACE_KMAX + 1) + c] = (kr && kc) ? sum + (r == c ? dg.v[r] : 0.0) : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  // A^{-1} by Gauss-Jordan elimination on [A | I] (k x 2k), two LDS buffers
  // so that each step reads the previous one: one barrier per step. A is
  // symmetric positive definite when every kept component has lambda > 0;
  // the pivots are those of its LDL^T factorization, so a pivot <= 0 means it
  // is not: ok[0] = 0 (every curve then takes its own factorization).
  constexpr int LDM = 2 * PACE_KMAX;
  for (int e = tid; e < k * 2 * k; e += NT) {
    const int r = e / (2 * k), j = e % (2 * k);
    M0[r * LDM + j] = j < k ? A[r * (PACE_KMAX + 1) + j] : (j - k == r ? 1.0 : 0.0);
  }
  __syncthreads();
  bool good = true;
  for (int c = 0; c < k; ++c) {
    const double *Mo = (c & 1) ? M1 : M0;
    double *Mn = (c & 1) ? M0 : M1;
    const double piv = Mo[c * LDM + c];
    good = good && piv > 0.0;
    const double inv = 1.0 / piv;
    for (int e = tid; e < k * 2 * k; e += NT) {
      const int r = e / (2 * k), j = e % (2 * k);
      const double pj = Mo[c * LDM + j] * inv;
      Mn[r * LDM + j] = r == c ? pj : fma(-Mo[r * LDM + c], pj, Mo[r * LDM + j]);
    }
    __syncthreads();
  }
  const double *Mf = (k & 1) ? M1 : M0;
  for (int e = tid; e < k * k; e += NT) Lout[e] = Mf[(e / k) * LDM + k + e % k];
  if (tid == 0) ok[0] = good ? 1 : 0;
}

// Common grid, curves observed at every node: the right-hand sides
// Phi^T (Y_i - mu) of 16 curves per workgroup as one FP64 MFMA product
// (rows = curves, columns = components, K = nodes). Each of the eight
// wavefronts streams an eighth of the nodes straight from memory into the
// operands (lane l: Y[curve l % 16][node + l / 16] minus mu, and the basis at
// the same node for components l % 16 and 16 + l % 16), MB steps loaded
// before they are used; the wavefronts' tiles are summed in a fixed order. A
// curve with a missing value
// gets a NaN first score: k_pace solves it on its own. The scores are the
// shared inverse times the right-hand sides. Workgroups 1..CG_NGW form
// partial sums of the shared matrix (cg_gram_part) and count themselves on
// ready[1]; workgroup 0 adds them, inverts the matrix (cg_inverse) and
// publishes the inverse through ready[0] (both zero at the launch: k_pace
// clears them at the end of every call), while the others form their
// right-hand sides. A workgroup that
// finds a flag unset after its spin limit gives up the shared factor: its
// curves go to k_pace.
constexpr int RH_CURVES = 16;

// Clears the flag through which k_pace_cg_rhs publishes the shared inverse
// and the count of its partial sums (a kernel rather than a memset, so that
// the call can be captured in a graph). The flags start at zero and every
// call's k_pace clears them again, so this runs only after a call that was
// cut short between its two kernels.
__global__ void k_pace_clear(int *__restrict__ ready) {
  if (threadIdx.x < 2) ready[threadIdx.x] = 0;
}

constexpr int RH_THREADS = 512;  // 8 wavefronts

template <typename T, bool VEC>
__global__ __launch_bounds__(RH_THREADS) void k_pace_cg_rhs(int64_t n, int64_t P, const T *__restrict__ y,
                                                      const T *__restrict__ mu, const T *__restrict__ efuns, int k,
                                                      PaceDiag dg, double *__restrict__ gpart,
                                                      double *__restrict__ Lcg, int *__restrict__ cg_ok,
                                                      int *__restrict__ ready, T *__restrict__ scores) {
  static_assert(4 * 2 * 256 + RH_CURVES * (PACE_KMAX + 1) + CG_A <= CG_POOL, "the right-hand sides fit the pool");
  __shared__ double pool[CG_POOL];
  auto red = reinterpret_cast<double(*)[2][256]>(pool);                             // [4][2][256]
  auto Ai = reinterpret_cast<double(*)[PACE_KMAX + 1]>(pool + 4 * 2 * 256);        // [PACE_KMAX][..]
  auto rhs = reinterpret_cast<double(*)[PACE_KMAX + 1]>(pool + 4 * 2 * 256 + CG_A);  // [RH_CURVES][..]
  constexpr int NW = RH_THREADS / 64;
  __shared__ int miss[RH_CURVES];
  __shared__ int s_ok;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (blockIdx.x == 0) {
    // the partial sums of the CG_NGW workgroups that follow (counted on ready[1])
    if (tid == 0) {
      long long it = 0;
      bool got = true;
      while (__hip_atomic_load(ready + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < CG_NGW) {
        if (++it > (1LL << 20)) {
          got = false;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (got) got = __hip_atomic_load(ready + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == CG_NGW;
      s_ok = got ? 1 : 0;
    }
    __syncthreads();
    if (s_ok) {
      cg_inverse<RH_THREADS>(k, dg, gpart, pool, Lcg, cg_ok);
    } else if (tid == 0) {
      cg_ok[0] = 0;  // no shared factor: k_pace solves every curve
    }
    // every lane's stores are released before the flag is set
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_store(ready, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  if (blockIdx.x <= CG_NGW) {
    cg_gram_part<T, VEC, RH_THREADS>(P, efuns, k, blockIdx.x - 1, pool, gpart);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(ready + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int64_t c0 = int64_t(blockIdx.x - 1 - CG_NGW) * RH_CURVES;
  if (tid < RH_CURVES) miss[tid] = 0;
  __syncthreads();
  const int nt = k > 16 ? 2 : 1;
  const int row = lane & 15, kk = lane >> 4;
  const int64_t c = c0 + row;
  const bool cin = c < n;
  const T *yr = y + (cin ? c : 0) * P;
  const bool r0 = row < k, r1 = 16 + row < k;
  const T *f0p = efuns + int64_t(r0 ? row : 0) * P;
  const T *f1p = efuns + int64_t(r1 ? 16 + row : 0) * P;
  const int64_t per = ((P + NW * 4 * MB - 1) / (NW * 4 * MB)) * 4 * MB;
  const int64_t n0 = wave * per, n1 = min(P, n0 + per);
  v4d d0 = {0, 0, 0, 0}, d1 = d0;
  bool bad = false;
  for (int64_t q = n0; q < n1; q += 4 * MB) {
    double a[MB], b0[MB], b1[MB];
    if (VEC && q + 4 * MB <= n1) {
      // step 4b + j takes node q + 16 b + 4 kk + j: each lane's four nodes of
      // a 16-node block in one vector load per array
      double ml[MB];
#pragma unroll
      for (int bl = 0; bl < MB / 4; ++bl) {
        const int64_t p = q + 16 * bl + 4 * kk;
        load4(yr + p, a + 4 * bl);
        load4(mu + p, ml + 4 * bl);
        load4(f0p + p, b0 + 4 * bl);
        load4(f1p + p, b1 + 4 * bl);
      }
#pragma unroll
      for (int s = 0; s < MB; ++s) {
        const double yv = cin ? a[s] : 0.0;
        bad |= !isfinite(yv);
        a[s] = cin ? yv - ml[s] : 0.0;
        b0[s] = r0 ? b0[s] : 0.0;
        b1[s] = r1 ? b1[s] : 0.0;
      }
    } else {
      // every load is issued (addresses clamped into the range), then masked
#pragma unroll
      for (int s = 0; s < MB; ++s) {
        const int64_t p = q + 16 * (s >> 2) + 4 * kk + (s & 3);
        const int64_t pc = min(p, n1 - 1);
        const double yl = double(yr[pc]), ml = double(mu[pc]), v0 = double(f0p[pc]), v1 = double(f1p[pc]);
        const bool in = p < n1 && cin;
        const double yv = in ? yl : 0.0;
        bad |= !isfinite(yv);
        a[s] = in ? yv - ml : 0.0;
        b0[s] = (p < n1 && r0) ? v0 : 0.0;
        b1[s] = (p < n1 && r1) ? v1 : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < MB; ++s) {
      d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b0[s], d0, 0, 0, 0);
      if (nt > 1) d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b1[s], d1, 0, 0, 0);
    }
  }
  if (bad) miss[row] = 1;
  // D[i][j] sits in lane j + 16 (i % 4), element i / 4 (i: curve, j:
  // component); waves 4g .. 4g + 3 add into the four slots in turn
  for (int g = 0; g < NW / 4; ++g) {
    if ((wave >> 2) == g) {
      const int w = wave & 3;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = (kk + 4 * v) * 16 + row;
        red[w][0][e] = (g ? red[w][0][e] : 0.0) + d0[v];
        red[w][1][e] = (g ? red[w][1][e] : 0.0) + d1[v];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < RH_CURVES * PACE_KMAX; e += RH_THREADS) {
    const int ci = e / PACE_KMAX, l = e % PACE_KMAX;
    if (l >= k) continue;
    const int tc = l >> 4, ei = ci * 16 + (l & 15);
    double sum = 0.0;
    for (int w = 0; w < 4; ++w) sum += red[w][tc][ei];
    rhs[ci][l] = dg.v[l] >= 0.0 ? sum : 0.0;
  }
  // the shared inverse from workgroup 0 (long done by now, as a rule)
  if (tid == 0) {
    // spin on relaxed loads, then one acquiring load (one cache invalidation
    // for the workgroup; the barrier below orders the other waves' loads)
    long long it = 0;
    bool got = true;
    while (__hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      if (++it > (1LL << 20)) {
        got = false;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (got) got = __hip_atomic_load(ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 1;
    s_ok = (got && cg_ok[0] == 1) ? 1 : 0;
  }
  __syncthreads();
  if (s_ok == 0) {
    // no shared factor (or it never came): k_pace solves these curves
    if (tid < RH_CURVES && c0 + tid < n) scores[(c0 + tid) * k] = T(__builtin_nan(""));
    return;
  }
  for (int e = tid; e < k * k; e += RH_THREADS) Ai[e / k][e % k] = Lcg[e];
  __syncthreads();
  // scores = A^{-1} rhs, one thread per (curve, component)
  if (tid < RH_CURVES * k) {
    const int ci = tid / k, l = tid % k;
    const int64_t cc = c0 + ci;
    if (cc < n) {
      double v = 0.0;
      for (int m = 0; m < k; ++m) v = fma(Ai[l][m], rhs[ci][m], v);
      if (miss[ci]) {
        if (l == 0) scores[cc * k] = T(__builtin_nan(""));  // marker: k_pace solves this curve
      } else {
        scores[cc * k + l] = T(v);
      }
    }
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
                                                       T *__restrict__ scores, int *__restrict__ ready) {
  // k_pace_cg_rhs has finished: its two flags return to zero for the next call
  if (ready && blockIdx.x == 0 && threadIdx.x < 2) ready[threadIdx.x] = 0;
  __shared__ double ph[PACE_CH][PACE_KMAX + 1];
  __shared__ double yc[PACE_CH];
  __shared__ double A[PACE_KMAX][PACE_KMAX + 1];
  __shared__ double rhs[PACE_KMAX];
  __shared__ unsigned char tri_r[PACE_TRI], tri_c[PACE_TRI];
  const int tid = threadIdx.x;
  const int64_t P = g.P;
  const int nmat = k * (k + 1) / 2, nacc = nmat + k;
  const bool fast = design == FPCA_COMMON_GRID && Lcg && cg_ok && cg_ok[0] == 1;
  bool built = false;  // the triangle's index tables, formed at the first curve this workgroup solves
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    int64_t a, b;
    if (design == FPCA_IRREGULAR) {
      a = off[i];
      b = off[i + 1];
    } else {
      a = i * P;
      b = a + P;
    }
    // with the shared factor, k_pace_cg_rhs has solved every complete curve
    // and marked the others with a NaN first score
    if (fast) {
      const double s0 = double(scores[i * k]);
      if (s0 == s0) continue;  // uniform: every thread reads the same value
    }
    if (!built) {
      if (tid == 0)
        for (int r = 0, e = 0; r < k; ++r)
          for (int c = r; c < k; ++c, ++e) {
            tri_r[e] = (unsigned char)r;
            tri_c[e] = (unsigned char)c;
          }
      __syncthreads();
      built = true;
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

// Scratch of the common-grid design: the shared k x k inverse, its
// positive-definiteness flag, the two flags of k_pace_cg_rhs and the partial
// sums of Phi^T Phi (8,192 + 256 + 256 + 49,152 bytes).
constexpr size_t PACE_PART_BYTES = size_t(CG_NGW) * 3 * 256 * sizeof(double);
constexpr size_t PACE_SCRATCH_BYTES = PACE_KMAX * PACE_KMAX * sizeof(double) + 256 + 256 + PACE_PART_BYTES;

// One copy per GPU of the scratch used by fpca_pace_scores_noalloc. In host
// code `scratch` names a host-side stand-in: kernels get the device address
// looked up for each device by pace_scratch_init.
constexpr int PACE_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[PACE_MAX_DEVICES] = {};
// the fixed array's two flags are zero (as they start): see pace_flags_clean
bool g_scratch_clean[PACE_MAX_DEVICES] = {};

// `fixed`: caller-provided scratch of PACE_SCRATCH_BYTES (the allocation-free
// entry point), or NULL to carve it from the handle's arena.
template <typename T>
int pace_impl(fpca_context *ctx, const fpca_grid *grid, int design, int64_t n, const int64_t *offsets, const T *t,
              const T *y, const T *mu, const T *efuns, int k, const PaceDiag &dg, T *scores, void *fixed) {
  if (n == 0) return FPCA_OK;
  const GridDims g = make_dims(grid);
  const double *Lcg = nullptr;
  const int *cg_ok = nullptr;
  int *ready_out = nullptr;   // the flags k_pace clears (common grid)
  bool *clean_out = nullptr;  // set again once that k_pace is queued
  if (design == FPCA_COMMON_GRID) {
    if (!fixed)
      if (int rc = ws_reserve(ctx, PACE_SCRATCH_BYTES)) return rc;
    Carver cv{static_cast<char *>(fixed ? fixed : ctx->ws), 0, fixed ? PACE_SCRATCH_BYTES : ctx->ws_size};
    double *L = cv.take<double>(PACE_KMAX * PACE_KMAX);
    int *okf = cv.take<int>(1);
    int *ready_fixed = cv.take<int>(2);
    // the flags: in the fixed array, or in the handle's flag words
    int *ready = fixed ? ready_fixed : ctx->d_flags + 16;
    bool *clean = fixed ? &g_scratch_clean[ctx->device] : &ctx->pace_flags_clean;
    double *gpart = cv.take<double>(PACE_PART_BYTES / sizeof(double));
    // vector loads when every row starts on a 16-byte boundary
    const bool vec = g.P % 4 == 0 && (reinterpret_cast<uintptr_t>(efuns) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(y) & 15) == 0 && (reinterpret_cast<uintptr_t>(mu) & 15) == 0;
    if (!*clean) {
      hipLaunchKernelGGL(k_pace_clear, dim3(1), dim3(64), 0, ctx->stream, ready);
      FPCA_LAUNCH_CHECK("pace_clear");
    }
    *clean = false;
    ready_out = ready;
    clean_out = clean;
    Lcg = L;
    cg_ok = okf;
    // workgroup 0 inverts the shared matrix, the next CG_NGW form its partial
    // sums, the others take 16 curves each
    const dim3 rgrid(unsigned((n + RH_CURVES - 1) / RH_CURVES + 1 + CG_NGW));
    if (vec)
      hipLaunchKernelGGL((k_pace_cg_rhs<T, true>), rgrid, dim3(RH_THREADS), 0, ctx->stream, n, g.P, y, mu, efuns, k,
                         dg, gpart, L, okf, ready, scores);
    else
      hipLaunchKernelGGL((k_pace_cg_rhs<T, false>), rgrid, dim3(RH_THREADS), 0, ctx->stream, n, g.P, y, mu, efuns, k,
                         dg, gpart, L, okf, ready, scores);
    FPCA_LAUNCH_CHECK("pace_cg_rhs");
  }
  // grid-stride over the curves; on the common grid most of them are done
  // (k_pace_cg_rhs solved them) and a workgroup only checks their marker
  const unsigned blocks = unsigned(n < 2048 ? n : 2048);
  hipLaunchKernelGGL(k_pace<T>, dim3(blocks), dim3(PACE_THREADS), 0, ctx->stream, g, n, design, offsets, t, y, mu,
                     efuns, k, dg, Lcg, cg_ok, scores, ready_out);
  FPCA_LAUNCH_CHECK("pace");
  if (clean_out) *clean_out = true;
  return FPCA_OK;
}

// Reconstruction on the grid (the display after eq. 2.7):
//   xhat[i][p] = mu[p] + sum_l xi[i][l] phi_l[p].
// Thread per node p of a 256-node block with its k basis values in registers
// (KB of them: k rounded up to a multiple of 8, the rest zero), the block's
// RC_CURVES score rows in LDS (zero past k); writes are contiguous along p.
// 64 curves per block: each block reads its nodes' basis values once per 64
// output rows.
constexpr int RC_CURVES = 64;

template <typename T, int KB>
__global__ __launch_bounds__(256) void k_reconstruct(int64_t P, int64_t n, int k, const T *__restrict__ mu,
                                                     const T *__restrict__ efuns, const T *__restrict__ xi,
                                                     T *__restrict__ xhat) {
  __shared__ double xs[RC_CURVES][KB];
  const int64_t i0 = int64_t(blockIdx.y) * RC_CURVES;
  const int nc = int(min(int64_t(RC_CURVES), n - i0));
  for (int e = threadIdx.x; e < nc * KB; e += blockDim.x) {
    const int c = e / KB, l = e % KB;
    xs[c][l] = l < k ? double(xi[(i0 + c) * k + l]) : 0.0;
  }
  __syncthreads();
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double ph[KB];
#pragma unroll
  for (int l = 0; l < KB; ++l) ph[l] = l < k ? double(efuns[int64_t(l) * P + p]) : 0.0;
  const double m = double(mu[p]);
  for (int c = 0; c < nc; ++c) {
    double v = m;
#pragma unroll
    for (int l = 0; l < KB; ++l) v = fma(xs[c][l], ph[l], v);
    xhat[(i0 + c) * P + p] = T(v);
  }
}

template <typename T>
int reconstruct_impl(fpca_context *ctx, int64_t P, int64_t n, int k, const T *mu, const T *efuns, const T *xi,
                     T *xhat) {
  if (n == 0 || P == 0) return FPCA_OK;
  const int64_t gy = (n + RC_CURVES - 1) / RC_CURVES;
  if (gy > 65535) return set_error(FPCA_ERR_UNSUPPORTED, "n = %lld curves exceeds %d", (long long)n, 65535 * RC_CURVES);
  const dim3 grid(unsigned((P + 255) / 256), unsigned(gy));
  switch ((k + 7) / 8) {
    case 1:
      hipLaunchKernelGGL((k_reconstruct<T, 8>), grid, dim3(256), 0, ctx->stream, P, n, k, mu, efuns, xi, xhat);
      break;
    case 2:
      hipLaunchKernelGGL((k_reconstruct<T, 16>), grid, dim3(256), 0, ctx->stream, P, n, k, mu, efuns, xi, xhat);
      break;
    case 3:
      hipLaunchKernelGGL((k_reconstruct<T, 24>), grid, dim3(256), 0, ctx->stream, P, n, k, mu, efuns, xi, xhat);
      break;
    default:
      hipLaunchKernelGGL((k_reconstruct<T, PACE_KMAX>), grid, dim3(256), 0, ctx->stream, P, n, k, mu, efuns, xi,
                         xhat);
      break;
  }
  FPCA_LAUNCH_CHECK("reconstruct");
  return FPCA_OK;
}


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
  g_scratch_clean[device] = true;  // a __device__ array starts zeroed
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

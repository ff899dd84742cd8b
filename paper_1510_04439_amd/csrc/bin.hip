// Linear binning (Section 3.2) of observations for the mean (eq. 2.3) and the
// raw covariance (eq. 2.4).
//
// Mean: each observation scatters its 2^d multilinear weights with atomics
// (into per-workgroup LDS sums on small grids, added without atomics after).
// Covariance, irregular design: the ordered-pair sums are assembled by the
// Gram identity
//   G = sum_i w_i (z_i z_i^T - sum_j Y_ij^2 b_ij b_ij^T),  z_i = sum_j b_ij Y_ij,
// (b_ij the binning-weight vector of t_ij): per-curve rows scaled by sqrt(w_i),
// one symmetric Gram product on MFMA, then the j = l terms subtracted.
// Covariance, common grid: G = Y^T Y / (P(P-1)) with the diagonal removed.
#include <cmath>

#include "binrule.hpp"
#include "common.hpp"

namespace fpca {
int gram_i32(fpca_context *ctx, const int32_t *A, int64_t K, int64_t N, int64_t *C);
}

namespace fpca {
namespace {

__device__ inline void atomic_add_t(float *p, double v) { atomicAdd(p, float(v)); }
__device__ inline void atomic_add_t(double *p, double v) { atomicAdd(p, v); }

// One workgroup per curve (grid-stride); threads over the curve's observations.
template <typename T>
__global__ __launch_bounds__(256) void k_bin_mean(GridDims g, int64_t n, const int64_t *__restrict__ off,
                                                   const T *__restrict__ t, const T *__restrict__ y,
                                                   T *c, T *s, T *s2, int32_t *idx,
                                                   unsigned long long *cnt, int *flags) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t a = off[i], b = off[i + 1];
    if (b <= a) continue;
    const double w = 1.0 / double(b - a);
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      int k[3];
      double rho[3];
      if (!locate(t + j * g.d, g, k, rho)) {
        atomicOr(flags, 1);
        if (idx) idx[j] = -1;
        continue;
      }
      const double yv = double(y[j]);
      int64_t lower = 0;
      for (int q = 0; q < g.d; ++q) lower += int64_t(k[q]) * g.stride[q];
      for (int cc = 0; cc < (1 << g.d); ++cc) {
        int64_t p;
        double W;
        corner(g, k, rho, cc, &p, &W);
        const double ww = w * W;
        atomic_add_t(&c[p], ww);
        atomic_add_t(&s[p], ww * yv);
        if (s2) atomic_add_t(&s2[p], ww * yv * yv);
      }
      if (idx) idx[j] = int32_t(lower);
      if (cnt) atomicAdd(&cnt[lower], 1ull);
    }
  }
}

// Mean binning on small grids (MB_PMAX nodes or fewer): the same scatter into
// FP64 accumulators in LDS (one set per workgroup, grid-stride over the
// curves), then each workgroup writes its sums to part[blockIdx][a][p]; the
// finish kernel adds the workgroups' sums in workgroup order. On a small
// grid every observation lands on a few hundred nodes, where global atomics
// from all workgroups queue on the same addresses.
constexpr int MB_PMAX = 2048;
constexpr int MB_WGS = 256;  // workgroups of the scatter
template <typename T>
__global__ __launch_bounds__(256) void k_bin_mean_lds(GridDims g, int64_t n, const int64_t *__restrict__ off,
                                                       const T *__restrict__ t, const T *__restrict__ y, int narr,
                                                       double *__restrict__ part, int32_t *idx,
                                                       unsigned long long *cnt, int *flags) {
  __shared__ double acc[3][MB_PMAX];
  const int P = int(g.P);
  for (int e = threadIdx.x; e < narr * P; e += blockDim.x) acc[e / P][e % P] = 0.0;
  __syncthreads();
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t a = off[i], b = off[i + 1];
    if (b <= a) continue;
    const double w = 1.0 / double(b - a);
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      int k[3];
      double rho[3];
      if (!locate(t + j * g.d, g, k, rho)) {
        atomicOr(flags, 1);
        if (idx) idx[j] = -1;
        continue;
      }
      const double yv = double(y[j]);
      int64_t lower = 0;
      for (int q = 0; q < g.d; ++q) lower += int64_t(k[q]) * g.stride[q];
      for (int cc = 0; cc < (1 << g.d); ++cc) {
        int64_t p;
        double W;
        corner(g, k, rho, cc, &p, &W);
        const double ww = w * W;
        atomicAdd(&acc[0][p], ww);
        atomicAdd(&acc[1][p], ww * yv);
        if (narr > 2) atomicAdd(&acc[2][p], ww * yv * yv);
      }
      if (idx) idx[j] = int32_t(lower);
      if (cnt) atomicAdd(&cnt[lower], 1ull);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < narr * P; e += blockDim.x)
    part[int64_t(blockIdx.x) * narr * P + e] = acc[e / P][e % P];
}

// Sum over the nwg workgroups' partials of element e: 16 lanes per element,
// lane g adds partials g, g + 16, ... (up to 16 loads in flight), then the 16
// lane sums are combined pairwise in a fixed order.
constexpr int WS_LANES = 16;
template <typename PT>
__device__ inline double sum_over_wgs(const PT *__restrict__ part, int64_t stride, int nwg, int64_t e, bool in,
                                      double (*red)[256 / WS_LANES]) {
  const int g = threadIdx.x / (256 / WS_LANES), el = threadIdx.x % (256 / WS_LANES);
  double sacc = 0.0;
  for (int w0 = g; w0 < nwg; w0 += WS_LANES * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int w = w0 + WS_LANES * u;
      v[u] = (in && w < nwg) ? double(part[int64_t(w) * stride + e]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) sacc += v[u];
  }
  red[g][el] = sacc;
  __syncthreads();
#pragma unroll
  for (int wd = WS_LANES / 2; wd > 0; wd >>= 1) {
    if (g < wd) red[g][el] += red[g + wd][el];
    __syncthreads();
  }
  return red[0][el];
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin_mean_finish(int64_t P, int narr, int nwg,
                                                          const double *__restrict__ part, T *c, T *s, T *s2) {
  __shared__ double red[WS_LANES][256 / WS_LANES];
  const int64_t e = int64_t(blockIdx.x) * (256 / WS_LANES) + threadIdx.x % (256 / WS_LANES);
  const bool in = e < narr * P;
  const double sum = sum_over_wgs(part, int64_t(narr) * P, nwg, e, in, red);
  if (in && threadIdx.x < 256 / WS_LANES) {
    const int a = int(e / P);
    const int64_t p = e % P;
    (a == 0 ? c : (a == 1 ? s : s2))[p] = T(sum);
  }
}

// Common grid, mean: column sums of the n x P matrix (and of its squares) in
// FP64 over chunks of CS_ROWS rows. A workgroup covers 256 columns (four per
// lane) of one chunk; wavefront w loads its CS_ROWS/4 rows at once, and the
// four wavefronts' sums are added in order through LDS. The chunk's sums go
// to part[chunk][P]; the finish kernel adds the chunks (no atomics).
constexpr int CS_ROWS = 64;
template <typename T>
__global__ __launch_bounds__(256) void k_colsum(int64_t n, int64_t P, const T *__restrict__ Y,
                                                 double *__restrict__ part1, double *__restrict__ part2) {
  constexpr int RW = CS_ROWS / 4;  // rows per wavefront
  __shared__ double red[2][4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = int64_t(blockIdx.x) * 256 + 4 * lane;
  const int64_t r0 = int64_t(blockIdx.y) * CS_ROWS + wave * RW;
  const bool vec = (P % 4 == 0) && p0 + 3 < P;
  T v[RW][4];
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    const int64_t r = r0 + u;
    if (r < n && vec) {
      if constexpr (sizeof(T) == 4) {
        const float4 x = *reinterpret_cast<const float4 *>(Y + r * P + p0);
        v[u][0] = x.x; v[u][1] = x.y; v[u][2] = x.z; v[u][3] = x.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[u][e] = Y[r * P + p0 + e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[u][e] = (r < n && p0 + e < P) ? Y[r * P + p0 + e] : T(0);
    }
  }
  double s[4] = {0.0, 0.0, 0.0, 0.0}, q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < RW; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double x = double(v[u][e]);
      s[e] += x;
      q[e] += x * x;
    }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    red[0][wave][4 * lane + e] = s[e];
    red[1][wave][4 * lane + e] = q[e];
  }
  __syncthreads();
  const int c = threadIdx.x;
  const int64_t p = int64_t(blockIdx.x) * 256 + c;
  if (p < P) {
    const int64_t o = int64_t(blockIdx.y) * P + p;
    part1[o] = (red[0][0][c] + red[0][1][c]) + (red[0][2][c] + red[0][3][c]);
    if (part2) part2[o] = (red[1][0][c] + red[1][1][c]) + (red[1][2][c] + red[1][3][c]);
  }
}

// c = n/P, s = (column sums)/P, s2 = (column sums of squares)/P: eight lanes
// per column add every eighth chunk (loads in flight together), then the
// eight sums are combined pairwise.
template <typename T>
__global__ __launch_bounds__(256) void k_colsum_finish(int64_t n, int64_t P, int nchunks,
                                                        const double *__restrict__ part1,
                                                        const double *__restrict__ part2, T *c, T *s, T *s2) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t p = gid >> 3;
  const int g = int(gid & 7);
  double a = 0.0, b = 0.0;
  if (p < P) {
    for (int k0 = g; k0 < nchunks; k0 += 64) {
      double va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + 8 * u;
        va[u] = k < nchunks ? part1[int64_t(k) * P + p] : 0.0;
        vb[u] = (s2 && k < nchunks) ? part2[int64_t(k) * P + p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a += va[u];
        b += vb[u];
      }
    }
  }
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if (p < P && g == 0) {
    c[p] = T(double(n) / double(P));
    s[p] = T(a / double(P));
    if (s2) s2[p] = T(b / double(P));
  }
}

// Row position of each curve when curves are grouped by fold (stable within a
// fold), and the first row of every fold. One workgroup.
__global__ __launch_bounds__(1024) void k_fold_rows(int64_t n, int n_folds, const int32_t *__restrict__ fold,
                                                    int64_t *pos, int64_t *fold_start, int *flags) {
  __shared__ int64_t scan[1024];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int f = 0; f < n_folds; ++f) {
    if (threadIdx.x == 0) fold_start[f] = base;
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
      const int64_t i = c0 + threadIdx.x;
      const int in = (i < n && fold[i] == f) ? 1 : 0;
      scan[threadIdx.x] = in;
      __syncthreads();
      for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
      }
      if (in) pos[i] = base + scan[threadIdx.x] - 1;
      __syncthreads();
      if (threadIdx.x == 1023) base += scan[1023];
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) fold_start[n_folds] = base;
  // curves whose fold id is out of range are left out of every fold
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    if (fold[i] < 0 || fold[i] >= n_folds) {
      pos[i] = -1;
      atomicOr(flags, 2);
    }
  }
}

// Per-curve rows of the Gram identity, scaled by sqrt(w_i), w_i = 1/(N_i(N_i-1)):
//   Z[r,p] = sqrt(w_i) sum_j W_p(t_ij) Y_ij,  Cr[r,p] = sqrt(w_i) sum_j W_p(t_ij),
//   Z2[r,p] = sqrt(w_i) sum_j W_p(t_ij) Y_ij^2, cntrow[r,p] = #obs with lower corner p,
// where r is the curve's row (grouped by fold). Rows must be zeroed first.
template <typename T>
__global__ __launch_bounds__(256) void k_bin_rows(GridDims g, int64_t n, const int64_t *__restrict__ off,
                                                   const T *__restrict__ t, const T *__restrict__ y,
                                                   const int64_t *__restrict__ pos, T *Z, T *Cr, T *Z2,
                                                   int32_t *cntrow, int *flags) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t a = off[i], b = off[i + 1];
    const int64_t Ni = b - a;
    const int64_t r = pos ? pos[i] : i;
    if (Ni < 2 || r < 0) continue;
    const double sw = sqrt(1.0 / (double(Ni) * double(Ni - 1)));
    T *zr = Z + r * g.P;
    T *cr = Cr + r * g.P;
    T *z2 = Z2 ? Z2 + r * g.P : nullptr;
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      int k[3];
      double rho[3];
      if (!locate(t + j * g.d, g, k, rho)) {
        atomicOr(flags, 1);
        continue;
      }
      const double yv = double(y[j]);
      for (int cc = 0; cc < (1 << g.d); ++cc) {
        int64_t p;
        double W;
        corner(g, k, rho, cc, &p, &W);
        atomic_add_t(&cr[p], sw * W);
        atomic_add_t(&zr[p], sw * W * yv);
        if (z2) atomic_add_t(&z2[p], sw * W * yv * yv);
      }
      if (cntrow) {
        int64_t lower = 0;
        for (int q = 0; q < g.d; ++q) lower += int64_t(k[q]) * g.stride[q];
        atomicAdd(&cntrow[r * g.P + lower], 1);
      }
    }
  }
}

// Removes the j = l terms of the Gram identity: for each observation and each
// pair (u, v) of its corners, subtract w_i W_u W_v (times Y^2 for G and Y^4
// for Q) in slab 0 and in the slab of the curve's fold. Also removes the
// self-pairs from the integer pair counts.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_diag(GridDims g, int64_t n, const int64_t *__restrict__ off,
                                                    const T *__restrict__ t, const T *__restrict__ y,
                                                    const int32_t *__restrict__ fold, int n_folds, T *C, T *G,
                                                    T *Q, int64_t slab, unsigned long long *cnt) {
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t a = off[i], b = off[i + 1];
    const int64_t Ni = b - a;
    if (Ni < 2) continue;
    const int f = fold ? fold[i] : -1;
    if (fold && (f < 0 || f >= n_folds)) continue;
    const double w = 1.0 / (double(Ni) * double(Ni - 1));
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      int k[3];
      double rho[3];
      if (!locate(t + j * g.d, g, k, rho)) continue;
      const double yv = double(y[j]);
      const double y2 = yv * yv;
      const int nc = 1 << g.d;
      int64_t pu[8];
      double Wu[8];
      for (int cc = 0; cc < nc; ++cc) corner(g, k, rho, cc, &pu[cc], &Wu[cc]);
      for (int u = 0; u < nc; ++u)
        for (int v = 0; v < nc; ++v) {
          const int64_t e = pu[u] * g.P + pu[v];
          const double ww = w * Wu[u] * Wu[v];
          if (ww == 0.0) continue;
          for (int sl = 0; sl < (fold ? 2 : 1); ++sl) {
            const int64_t o = sl == 0 ? e : (int64_t(f) + 1) * slab + e;
            atomic_add_t(&C[o], -ww);
            atomic_add_t(&G[o], -ww * y2);
            if (Q) atomic_add_t(&Q[o], -ww * y2 * y2);
          }
        }
      if (cnt) {
        int64_t lower = 0;
        for (int q = 0; q < g.d; ++q) lower += int64_t(k[q]) * g.stride[q];
        atomicAdd(&cnt[lower * g.P + lower], (unsigned long long)(-1ll));
      }
    }
  }
}

// The same j = l terms on small grids without folds: every such pair (u, v)
// joins two corners of one cell, so it is node u and one of the 3^d
// neighbours u + sum_q dq stride_q (dq in {-1, 0, 1}). Each workgroup
// (grid-stride over the curves) adds the terms into FP32 sums per (node,
// neighbour) in LDS (in the storage type T: FP32 sums for FP32 data, FP64
// for FP64) and writes them to part[blockIdx][a][node][neighbour];
// k_pair_diag_finish adds the workgroups' sums in workgroup order (FP64) and
// subtracts them from C, G and Q.
constexpr size_t PD_LDS_MAX = 128 * 1024;  // bytes of LDS for the sums
constexpr int PD_WGS = 256;                // workgroups of the scatter
template <typename T>
__global__ __launch_bounds__(256) void k_pair_diag_lds(GridDims g, int64_t n, const int64_t *__restrict__ off,
                                                        const T *__restrict__ t, const T *__restrict__ y, int narr,
                                                        T *__restrict__ part, unsigned long long *cnt) {
  extern __shared__ __align__(8) unsigned char pacc_raw[];
  T *pacc = reinterpret_cast<T *>(pacc_raw);  // [narr][P][nb]
  const int P = int(g.P);
  int nb = 1;
  for (int q = 0; q < g.d; ++q) nb *= 3;
  const int tot = narr * P * nb;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) pacc[e] = T(0);
  __syncthreads();
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t a = off[i], b = off[i + 1];
    const int64_t Ni = b - a;
    if (Ni < 2) continue;
    const double w = 1.0 / (double(Ni) * double(Ni - 1));
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) {
      int k[3];
      double rho[3];
      if (!locate(t + j * g.d, g, k, rho)) continue;
      const double yv = double(y[j]);
      const double y2 = yv * yv;
      const int nc = 1 << g.d;
      int64_t pu[8];
      double Wu[8];
      for (int cc = 0; cc < nc; ++cc) corner(g, k, rho, cc, &pu[cc], &Wu[cc]);
      for (int u = 0; u < nc; ++u)
        for (int v = 0; v < nc; ++v) {
          const double ww = w * Wu[u] * Wu[v];
          if (ww == 0.0) continue;
          // digit q of bi: the step of coordinate q from corner u to corner v
          // (corner() takes coordinate q from bit d-1-q of the corner index)
          int bi = 0, m = 1;
          for (int q = 0; q < g.d; ++q, m *= 3) {
            const int sh = g.d - 1 - q;
            bi += (((v >> sh) & 1) - ((u >> sh) & 1) + 1) * m;
          }
          T *ac = pacc + int64_t(pu[u]) * nb + bi;
          atomicAdd(ac, T(ww));
          atomicAdd(ac + int64_t(P) * nb, T(ww * y2));
          if (narr > 2) atomicAdd(ac + 2 * int64_t(P) * nb, T(ww * y2 * y2));
        }
      if (cnt) {
        int64_t lower = 0;
        for (int q = 0; q < g.d; ++q) lower += int64_t(k[q]) * g.stride[q];
        atomicAdd(&cnt[lower * g.P + lower], (unsigned long long)(-1ll));
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < tot; e += blockDim.x) part[int64_t(blockIdx.x) * tot + e] = pacc[e];
}

template <typename T>
__global__ __launch_bounds__(256) void k_pair_diag_finish(GridDims g, int narr, int nwg,
                                                           const T *__restrict__ part, T *C, T *G, T *Q) {
  __shared__ double red[WS_LANES][256 / WS_LANES];
  const int P = int(g.P);
  int nb = 1;
  for (int q = 0; q < g.d; ++q) nb *= 3;
  // element (node, neighbour) of this lane group
  const int64_t e = int64_t(blockIdx.x) * (256 / WS_LANES) + threadIdx.x % (256 / WS_LANES);
  const bool in = e < int64_t(P) * nb;
  const int p = in ? int(e / nb) : 0, bi = in ? int(e % nb) : 0;
  // the neighbour's node, if it exists
  int64_t qn = p;
  int m = bi;
  bool ok = in;
  for (int q = 0; q < g.d; ++q) {
    const int dq = m % 3 - 1;
    m /= 3;
    const int kq = int((p / g.stride[q]) % g.M[q]);
    if (kq + dq < 0 || kq + dq >= g.M[q]) ok = false;
    qn += int64_t(dq) * g.stride[q];
  }
  const int64_t tot = int64_t(narr) * P * nb;
  for (int a = 0; a < narr; ++a) {
    const double sum = sum_over_wgs(part + int64_t(a) * P * nb, tot, nwg, e, ok, red);
    if (ok && threadIdx.x < 256 / WS_LANES && sum != 0.0) {
      T *A = a == 0 ? C : (a == 1 ? G : Q);
      const int64_t o = int64_t(p) * P + qn;
      A[o] = T(double(A[o]) - sum);
    }
    __syncthreads();  // red is reused for the next array
  }
}

// Slab 0 = sum of the fold slabs.
template <typename T>
__global__ void k_sum_slabs(T *A, int64_t slab, int nf) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (; e < slab; e += step) {
    T s = T(0);
    for (int f = 1; f <= nf; ++f) s += A[f * slab + e];
    A[e] = s;
  }
}

template <typename T>
__global__ void k_square(const T *__restrict__ a, T *__restrict__ b, int64_t n) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (; e < n; e += step) b[e] = a[e] * a[e];
}

template <typename T>
__global__ void k_set_diag(T *A, int64_t P, T v) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < P) A[p * P + p] = v;
}

inline unsigned grid1(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return unsigned(b > cap ? cap : b);
}

template <typename T>
int gram(fpca_context *ctx, const T *A, int64_t K, int64_t N, T *C, double alpha, bool zero_diag, int prec) {
  if constexpr (sizeof(T) == 4)
    return syrk_f32(ctx, A, K, N, C, N, float(alpha), zero_diag, prec);
  else
    return syrk_f64(ctx, A, K, N, C, N, alpha, zero_diag);
}

template <typename T>
int bin_impl(fpca_context *ctx, const fpca_grid *grid, int kind, int design, int prec, int64_t n,
             const int64_t *offsets, const T *t, const T *y, const int32_t *fold, int n_folds, T *W, T *S,
             T *SQ, int32_t *bin_index, int64_t *cell_count) {
  GridDims g = make_dims(grid);
  const int64_t P = g.P;
  if (kind == FPCA_BIN_MEAN) {
    if (design == FPCA_IRREGULAR) {
      const bool lds = P <= MB_PMAX && n > 0;  // the finish kernel writes every node
      if (!lds) {
        if (int rc = fill_bytes_zero(ctx, W, P * sizeof(T))) return rc;
        if (int rc = fill_bytes_zero(ctx, S, P * sizeof(T))) return rc;
        if (SQ)
          if (int rc = fill_bytes_zero(ctx, SQ, P * sizeof(T))) return rc;
      }
      if (cell_count)
        if (int rc = fill_i64(ctx, cell_count, 0, P)) return rc;
      if (n == 0) return FPCA_OK;
      if (lds) {
        const int narr = SQ ? 3 : 2;
        const int nwg = int(n < MB_WGS ? n : MB_WGS);
        if (int rc = ws_reserve(ctx, carve_bytes(size_t(nwg) * narr * P, 8))) return rc;
        double *part = static_cast<double *>(ctx->ws);
        hipLaunchKernelGGL(k_bin_mean_lds<T>, dim3(unsigned(nwg)), dim3(256), 0, ctx->stream, g, n, offsets, t, y,
                           narr, part, bin_index, reinterpret_cast<unsigned long long *>(cell_count), ctx->d_flags);
        FPCA_LAUNCH_CHECK("bin_mean_lds");
        hipLaunchKernelGGL(k_bin_mean_finish<T>, dim3(unsigned((narr * P + 15) / 16)), dim3(256), 0, ctx->stream, P,
                           narr, nwg, part, W, S, SQ);
        FPCA_LAUNCH_CHECK("bin_mean_finish");
        return FPCA_OK;
      }
      unsigned blocks = unsigned(n < 16384 ? n : 16384);
      hipLaunchKernelGGL(k_bin_mean<T>, dim3(blocks), dim3(256), 0, ctx->stream, g, n, offsets, t, y, W, S, SQ,
                         bin_index, reinterpret_cast<unsigned long long *>(cell_count), ctx->d_flags);
      FPCA_LAUNCH_CHECK("bin_mean");
      return FPCA_OK;
    }
    // common grid
    const int nchunks = int(n > 0 ? (n + CS_ROWS - 1) / CS_ROWS : 0);
    const size_t part = carve_bytes(size_t(nchunks > 0 ? nchunks : 1) * P, 8);
    if (int rc = ws_reserve(ctx, 2 * part)) return rc;
    Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
    double *part1 = cv.take<double>(size_t(nchunks > 0 ? nchunks : 1) * P);
    double *part2 = cv.take<double>(size_t(nchunks > 0 ? nchunks : 1) * P);
    if (n > 0) {
      dim3 grd((unsigned)((P + 255) / 256), (unsigned)nchunks);
      hipLaunchKernelGGL(k_colsum<T>, grd, dim3(256), 0, ctx->stream, n, P, y, part1, SQ ? part2 : nullptr);
      FPCA_LAUNCH_CHECK("colsum");
    }
    hipLaunchKernelGGL(k_colsum_finish<T>, dim3(unsigned((8 * P + 255) / 256)), dim3(256), 0, ctx->stream, n, P,
                       nchunks, part1, part2, W, S, SQ);
    FPCA_LAUNCH_CHECK("colsum_finish");
    return FPCA_OK;
  }

  // ---------------- covariance
  const int nsl = (fold && n_folds > 0) ? n_folds + 1 : 1;
  const int64_t slab = P * P;
  if (design == FPCA_COMMON_GRID) {
    const double w = 1.0 / (double(P) * double(P - 1));
    if (int rc = gram<T>(ctx, y, n, P, S, w, true, prec)) return rc;
    if (W) {  // the pair weights n w (1 - delta_pq) are materialized only when asked for
      if constexpr (sizeof(T) == 4) {
        if (int rc = fill_f32(ctx, W, float(double(n) * w), slab)) return rc;
      } else {
        if (int rc = fill_f64(ctx, W, double(n) * w, slab)) return rc;
      }
      hipLaunchKernelGGL(k_set_diag<T>, dim3(grid1(P)), dim3(256), 0, ctx->stream, W, P, T(0));
      FPCA_LAUNCH_CHECK("set_diag");
    }
    if (SQ) {
      if (int rc = ws_reserve(ctx, carve_bytes(size_t(n) * P, sizeof(T)))) return rc;
      T *Y2 = static_cast<T *>(ctx->ws);
      hipLaunchKernelGGL(k_square<T>, dim3(grid1(n * P)), dim3(256), 0, ctx->stream, y, Y2, n * P);
      FPCA_LAUNCH_CHECK("square");
      if (int rc = gram<T>(ctx, Y2, n, P, SQ, w, true, prec)) return rc;
    }
    return FPCA_OK;
  }

  // irregular design: rows, Gram products, j = l correction
  const int64_t nrows = n;
  size_t need = 2 * carve_bytes(size_t(nrows) * P, sizeof(T));
  if (SQ) need += carve_bytes(size_t(nrows) * P, sizeof(T));
  if (cell_count) need += carve_bytes(size_t(nrows) * P, sizeof(int32_t));
  if (nsl > 1) need += carve_bytes(n, 8) + carve_bytes(n_folds + 1, 8);
  if (int rc = ws_reserve(ctx, need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  T *Z = cv.take<T>(size_t(nrows) * P);
  T *Cr = cv.take<T>(size_t(nrows) * P);
  T *Z2 = SQ ? cv.take<T>(size_t(nrows) * P) : nullptr;
  int32_t *cntrow = cell_count ? cv.take<int32_t>(size_t(nrows) * P) : nullptr;
  int64_t *pos = nullptr, *fstart = nullptr;
  if (nsl > 1) {
    pos = cv.take<int64_t>(n);
    fstart = cv.take<int64_t>(n_folds + 1);
  }
  const int64_t rowbytes = nrows * P * int64_t(sizeof(T));
  if (int rc = fill_bytes_zero(ctx, Z, rowbytes)) return rc;
  if (int rc = fill_bytes_zero(ctx, Cr, rowbytes)) return rc;
  if (Z2)
    if (int rc = fill_bytes_zero(ctx, Z2, rowbytes)) return rc;
  if (cntrow)
    if (int rc = fill_bytes_zero(ctx, cntrow, nrows * P * 4)) return rc;
  if (nsl > 1 && n > 0) {
    hipLaunchKernelGGL(k_fold_rows, dim3(1), dim3(1024), 0, ctx->stream, n, n_folds, fold, pos, fstart,
                       ctx->d_flags);
    FPCA_LAUNCH_CHECK("fold_rows");
  }
  unsigned blocks = unsigned(n < 16384 ? (n > 0 ? n : 1) : 16384);
  if (n > 0) {
    hipLaunchKernelGGL(k_bin_rows<T>, dim3(blocks), dim3(256), 0, ctx->stream, g, n, offsets, t, y, pos, Z, Cr, Z2,
                       cntrow, ctx->d_flags);
    FPCA_LAUNCH_CHECK("bin_rows");
  }
  if (nsl == 1) {
    if (int rc = gram<T>(ctx, Cr, n, P, W, 1.0, false, prec)) return rc;
    if (int rc = gram<T>(ctx, Z, n, P, S, 1.0, false, prec)) return rc;
    if (SQ)
      if (int rc = gram<T>(ctx, Z2, n, P, SQ, 1.0, false, prec)) return rc;
  } else {
    // fold f occupies rows [fstart[f], fstart[f+1]); the boundaries are read
    // back once (n_folds+1 integers) to size each product.
    std::vector<int64_t> hs(n_folds + 1);
    FPCA_HIP(hipMemcpyAsync(hs.data(), fstart, sizeof(int64_t) * (n_folds + 1), hipMemcpyDeviceToHost,
                            ctx->stream));
    FPCA_HIP(hipStreamSynchronize(ctx->stream));
    for (int f = 0; f < n_folds; ++f) {
      const int64_t r0 = hs[f], kf = hs[f + 1] - hs[f];
      T *Wf = W + (int64_t(f) + 1) * slab;
      T *Sf = S + (int64_t(f) + 1) * slab;
      if (kf == 0) {
        if (int rc = fill_bytes_zero(ctx, Wf, slab * sizeof(T))) return rc;
        if (int rc = fill_bytes_zero(ctx, Sf, slab * sizeof(T))) return rc;
        if (SQ)
          if (int rc = fill_bytes_zero(ctx, SQ + (int64_t(f) + 1) * slab, slab * sizeof(T))) return rc;
        continue;
      }
      if (int rc = gram<T>(ctx, Cr + r0 * P, kf, P, Wf, 1.0, false, prec)) return rc;
      if (int rc = gram<T>(ctx, Z + r0 * P, kf, P, Sf, 1.0, false, prec)) return rc;
      if (SQ)
        if (int rc = gram<T>(ctx, Z2 + r0 * P, kf, P, SQ + (int64_t(f) + 1) * slab, 1.0, false, prec)) return rc;
    }
    for (T *A : {W, S, SQ}) {
      if (!A) continue;
      hipLaunchKernelGGL(k_sum_slabs<T>, dim3(grid1(slab)), dim3(256), 0, ctx->stream, A, slab, n_folds);
      FPCA_LAUNCH_CHECK("sum_slabs");
    }
  }
  if (cell_count) {
    if (int rc = gram_i32(ctx, cntrow, n, P, cell_count)) return rc;
  }
  if (n > 0) {
    int nb = 1;
    for (int q = 0; q < g.d; ++q) nb *= 3;
    const int narr = SQ ? 3 : 2;
    const size_t lds = size_t(narr) * size_t(P) * nb * sizeof(T);
    if (nsl == 1 && lds <= PD_LDS_MAX) {
      static size_t lds_set = 0;  // the attribute is set once per size (not inside a captured stream)
      if (lds > lds_set) {
        FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_pair_diag_lds<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(PD_LDS_MAX)));
        lds_set = PD_LDS_MAX;
      }
      const int nwg = int(n < PD_WGS ? n : PD_WGS);
      if (int rc = ws_reserve(ctx, carve_bytes(size_t(nwg) * narr * P * nb, sizeof(T)))) return rc;
      T *part = static_cast<T *>(ctx->ws);
      hipLaunchKernelGGL(k_pair_diag_lds<T>, dim3(unsigned(nwg)), dim3(256), lds, ctx->stream, g, n, offsets, t, y,
                         narr, part, reinterpret_cast<unsigned long long *>(cell_count));
      FPCA_LAUNCH_CHECK("pair_diag_lds");
      hipLaunchKernelGGL(k_pair_diag_finish<T>, dim3(unsigned((int64_t(P) * nb + 15) / 16)), dim3(256), 0,
                         ctx->stream, g, narr, nwg, part, W, S, SQ);
      FPCA_LAUNCH_CHECK("pair_diag_finish");
      return FPCA_OK;
    }
    hipLaunchKernelGGL(k_pair_diag<T>, dim3(blocks), dim3(256), 0, ctx->stream, g, n, offsets, t, y,
                       nsl > 1 ? fold : nullptr, n_folds, W, S, SQ, slab,
                       reinterpret_cast<unsigned long long *>(cell_count));
    FPCA_LAUNCH_CHECK("pair_diag");
  }
  return FPCA_OK;
}

}  // namespace
}  // namespace fpca

using namespace fpca;

extern "C" int fpca_bin(fpca_handle ctx, const fpca_grid *grid, int kind, int design, int dtype, int prec,
                        int64_t n, const int64_t *offsets, const void *t, const void *y,
                        const int32_t *fold_of_curve, int n_folds, void *weights, void *sums, void *sq_sums,
                        int32_t *bin_index, int64_t *cell_count) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (kind != FPCA_BIN_MEAN && kind != FPCA_BIN_COV) return set_error(FPCA_ERR_INVALID_ARG, "bad kind %d", kind);
  if (design != FPCA_IRREGULAR && design != FPCA_COMMON_GRID)
    return set_error(FPCA_ERR_INVALID_ARG, "bad design %d", design);
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (n < 0) return set_error(FPCA_ERR_INVALID_ARG, "n < 0");
  if (!sums) return set_error(FPCA_ERR_INVALID_ARG, "sums are required");
  if (!weights && !(kind == FPCA_BIN_COV && design == FPCA_COMMON_GRID))
    return set_error(FPCA_ERR_INVALID_ARG, "weights are required (optional only for common-grid COV binning)");
  if (!y && n > 0) return set_error(FPCA_ERR_INVALID_ARG, "y is required");
  if (design == FPCA_IRREGULAR) {
    if (!offsets || (!t && n > 0)) return set_error(FPCA_ERR_INVALID_ARG, "irregular design needs offsets and t");
  } else {
    if (offsets || t) return set_error(FPCA_ERR_INVALID_ARG, "common-grid design takes no offsets or t");
    if (bin_index) return set_error(FPCA_ERR_INVALID_ARG, "bin_index is defined for irregular designs only");
    if (cell_count) return set_error(FPCA_ERR_UNSUPPORTED, "cell_count is defined for irregular designs only");
    if (fold_of_curve) return set_error(FPCA_ERR_UNSUPPORTED, "folds need the irregular design");
  }
  if (fold_of_curve && n_folds < 1) return set_error(FPCA_ERR_INVALID_ARG, "n_folds must be >= 1 with folds");
  if (kind == FPCA_BIN_MEAN && fold_of_curve) return set_error(FPCA_ERR_UNSUPPORTED, "folds apply to COV binning");
  if (kind == FPCA_BIN_COV) {
    if (P > 8192) return set_error(FPCA_ERR_UNSUPPORTED, "covariance binning needs P <= 8192 (P = %lld)", (long long)P);
    if (dtype == FPCA_F64 && prec != FPCA_PREC_F64)
      return set_error(FPCA_ERR_UNSUPPORTED, "dtype F64 needs prec F64");
    if (dtype == FPCA_F32 && prec != FPCA_PREC_F32 && prec != FPCA_PREC_BF16X3)
      return set_error(FPCA_ERR_UNSUPPORTED, "dtype F32 needs prec F32 or BF16X3");
    if (bin_index) return set_error(FPCA_ERR_INVALID_ARG, "bin_index is produced by MEAN binning");
  }
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return bin_impl<double>(ctx, grid, kind, design, prec, n, offsets, static_cast<const double *>(t),
                            static_cast<const double *>(y), fold_of_curve, n_folds, static_cast<double *>(weights),
                            static_cast<double *>(sums), static_cast<double *>(sq_sums), bin_index, cell_count);
  return bin_impl<float>(ctx, grid, kind, design, prec, n, offsets, static_cast<const float *>(t),
                         static_cast<const float *>(y), fold_of_curve, n_folds, static_cast<float *>(weights),
                         static_cast<float *>(sums), static_cast<float *>(sq_sums), bin_index, cell_count);
}

// Both binnings of complete common-grid curves. FP32 data with BF16x3
// products: the Gram product's split pass over Y also leaves the mean's FP64
// column-sum chunks (the same sums as k_colsum, bit for bit), so Y is read
// once; k_colsum_finish then forms the mean's arrays. Otherwise the two
// binnings run one after the other.
extern "C" int fpca_bin_common(fpca_handle ctx, const fpca_grid *grid, int dtype, int prec, int64_t n, const void *y,
                               void *mean_weights, void *mean_sums, void *mean_sq_sums, void *cov_weights,
                               void *cov_sums) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (dtype != FPCA_F32 || prec != FPCA_PREC_BF16X3) {
    if (int rc = fpca_bin(ctx, grid, FPCA_BIN_MEAN, FPCA_COMMON_GRID, dtype, prec, n, nullptr, nullptr, y, nullptr,
                          0, mean_weights, mean_sums, mean_sq_sums, nullptr, nullptr))
      return rc;
    return fpca_bin(ctx, grid, FPCA_BIN_COV, FPCA_COMMON_GRID, dtype, prec, n, nullptr, nullptr, y, nullptr, 0,
                    cov_weights, cov_sums, nullptr, nullptr, nullptr);
  }
  if (n < 0) return set_error(FPCA_ERR_INVALID_ARG, "n < 0");
  if (!mean_weights || !mean_sums || !cov_sums)
    return set_error(FPCA_ERR_INVALID_ARG, "mean_weights, mean_sums and cov_sums are required");
  if (!y && n > 0) return set_error(FPCA_ERR_INVALID_ARG, "y is required");
  if (P > 8192) return set_error(FPCA_ERR_UNSUPPORTED, "covariance binning needs P <= 8192 (P = %lld)", (long long)P);
  if (int rc = set_device(ctx)) return rc;
  const float *Y = static_cast<const float *>(y);
  float *W = static_cast<float *>(mean_weights), *S = static_cast<float *>(mean_sums);
  float *SQ = static_cast<float *>(mean_sq_sums);
  const int nchunks = int((n + 63) / 64);  // the Gram split's 64-row K blocks
  const size_t part = carve_bytes(size_t(nchunks > 0 ? nchunks : 1) * P, 8);
  if (int rc = ws_reserve(ctx, 2 * part)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  double *part1 = cv.take<double>(size_t(nchunks > 0 ? nchunks : 1) * P);
  double *part2 = cv.take<double>(size_t(nchunks > 0 ? nchunks : 1) * P);
  const double w = 1.0 / (double(P) * double(P - 1));
  if (int rc = syrk_f32(ctx, Y, n, P, static_cast<float *>(cov_sums), P, float(w), true, FPCA_PREC_BF16X3, part1,
                        SQ ? part2 : nullptr))
    return rc;
  hipLaunchKernelGGL(k_colsum_finish<float>, dim3(unsigned((8 * P + 255) / 256)), dim3(256), 0, ctx->stream, n, P,
                     nchunks, part1, part2, W, S, SQ);
  FPCA_LAUNCH_CHECK("colsum_finish");
  if (cov_weights) {
    float *CW = static_cast<float *>(cov_weights);
    if (int rc = fill_f32(ctx, CW, float(double(n) * w), P * P)) return rc;
    hipLaunchKernelGGL(k_set_diag<float>, dim3(grid1(P)), dim3(256), 0, ctx->stream, CW, P, 0.f);
    FPCA_LAUNCH_CHECK("set_diag");
  }
  return FPCA_OK;
}

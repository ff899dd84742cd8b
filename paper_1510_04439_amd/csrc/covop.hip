// The smoothed covariance of complete common-grid data as an operator: its
// products with a block of vectors are formed without the P x P covariance
// ever being stored (Section 3.2's blockwise processing, Section 3.4's
// products of the covariance with the projection matrix).
//
// With every curve observed at every node, the pair weights of eq. 2.4 are one
// constant off the diagonal p = q and zero on it, and the pair sums are
// G = (Y^T Y - diag) / (P(P-1)). Write Z_{i,0} for curve i filtered by the
// product taps K and Z_{i,k} for the taps K u_k (u_k = m / H_k along
// coordinate k, H_k = h_k (M_k - 1)), and W_e(x) = sum_m K(m) (m/H)^e for the
// 1-D window sums at x. Where the s- and t-windows of a covariance node share
// no grid node (|s_k - t_k| > 2 R_k for some k), no diagonal pair enters the
// window: the weight moments are a tensor product and the local-linear
// intercept has a closed form, which factors over the two ends:
//   b0(s,t) = (1/n) sum_i [ L_i(s) L_i(t) - B_i(s) B_i(t) ]
//   B_i(x) = (A(x) Z_{i,0}(x) - sum_k (a_k/v_k) Z_{i,k}(x)) / S(x),
//   L_i(x) = Z_{i,0}(x) / S(x) + B_i(x)   (curve i's own local-linear smooth),
// with a_k = W_1/W_0, v_k = W_2/W_0 - a_k^2 at x_k, A = sum_k a_k^2/v_k and
// S = prod_k W_0(x_k). Away from the band |s - t|_inf <= 2R the smoothed
// covariance therefore has rank at most 2n + 1 (with the mean term) and
//   Gamma X = (1/n) (L (L^T X) - B (B^T X)) - mu (mu^T X) + Delta X,
// where Delta is nonzero on the band only: there the (2d+1)-moment system is
// solved per node with the diagonal pairs removed,
//   weight moments   = prod_k W(s_k) W(t_k) - prod_k E_k(s_k, t_k),
//   response moments = (1/n) [ sum_i Z_a(s) Z_b(t) - sum_p f(p; s,t) Y2(p) ],
// (E_k the 1-D sums over shared nodes of K(p-s)K(p-t) times powers of u and
// v, Y2(p) = sum_i Y_ip^2, f the product of the per-coordinate factors), and
// Delta = b0_band - b0_closed form. Delta is either recomputed in every
// product (tile by tile, nothing of the covariance kept) or formed once and
// kept in tile blocks (the band only). Everything is FP64.
//
// Band tiles are boxes of 64 nodes (64; 8 x 8; 4 x 4 x 4). One workgroup per
// s-tile visits the t-tiles within reach of the band; per tile pair:
//   1. the 2d+1 response moments of the full pair sums as products over the
//      curves, in chunks of 16 curves staged in LDS;
//   2. the diagonal correction by mode products of the Y2 box with the 1-D
//      factors of each coordinate (separable sums over the shared nodes);
//   3. the weight moments from 1-D tables, the FP64 solve and Delta;
//   4. Delta times the t-tile's rows of X added to the s-tile's outputs (or
//      the block stored).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "common.hpp"
#include "covop.hpp"
#include "wls.hpp"

namespace fpca {
namespace {

constexpr int BT = 512;  // band kernel threads
constexpr int NC = 16;   // curves per staged chunk
constexpr int ZP = 66;   // padded row of 64 nodes in LDS

struct CovGeo {
  int d;
  int M[3];
  int R[3];
  int64_t stride[3];
  int64_t P;
  int n;
  double inv_n;
  const double *K[3];  // K(m), m = -R..R
  const double *U[3];  // m / H
  const double *W[3];  // W[x*3 + e]
  const double *E[3];  // E[(x*(4R+1) + delta + 2R)*6 + ab], ab: 00 10 01 20 11 02
  int tb[3], nt[3], span[3];
  int nslot;
};

template <int d>
constexpr int tile_ext() {
  return d == 1 ? 64 : (d == 2 ? 8 : 4);
}

// ------------------------------------------------------------------ set-up
__global__ void k_transpose(int64_t n, int64_t P, const double *__restrict__ Y, double *__restrict__ Yn) {
  __shared__ double t[32][33];
  const int64_t p0 = int64_t(blockIdx.x) * 32, i0 = int64_t(blockIdx.y) * 32;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int64_t i = i0 + r, p = p0 + threadIdx.x;
    t[r][threadIdx.x] = (i < n && p < P) ? Y[i * P + p] : 0.0;
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int64_t p = p0 + r, i = i0 + threadIdx.x;
    if (p < P && i < n) Yn[p * n + i] = t[threadIdx.x][r];
  }
}

__global__ void k_sq(int64_t P, int n, const double *__restrict__ Yn, double *__restrict__ Y2) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v = Yn[p * n + i];
    s = fma(v, v, s);
  }
  Y2[p] = s;
}

struct FilterMap {
  int nmap;
  int fo[4], fi[4], e[4];
};

// One 1-D pass along coordinate k of node-major arrays [P][F][n]: map j of
// blockIdx.y takes family fi through the taps K (e = 0) or K u (e = 1) into
// family fo.
__global__ void k_filter(CovGeo g, int k, const double *__restrict__ in, int Fin, double *__restrict__ out,
                         int Fout, FilterMap fm) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int n = g.n;
  if (idx >= g.P * n) return;
  const int j = blockIdx.y;
  const int64_t p = idx / n;
  const int i = int(idx - p * n);
  const int64_t st = g.stride[k];
  const int R = g.R[k];
  const int xk = int((p / st) % g.M[k]);
  const int lo = -min(R, xk), hi = min(R, g.M[k] - 1 - xk);
  const int fi = fm.fi[j], fo = fm.fo[j];
  const bool wu = fm.e[j] != 0;
  const double *Kk = g.K[k], *Uk = g.U[k];
  double acc = 0.0;
  for (int m = lo; m <= hi; ++m) {
    const double w = wu ? Kk[m + R] * Uk[m + R] : Kk[m + R];
    acc = fma(w, in[((p + int64_t(m) * st) * Fin + fi) * n + i], acc);
  }
  out[(p * Fout + fo) * n + i] = acc;
}

// L and B of every curve at every node from the filtered families.
__global__ void k_lr_prep(CovGeo g, const double *__restrict__ Zn, double *__restrict__ Ln, double *__restrict__ Bn) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int n = g.n;
  if (idx >= g.P * n) return;
  const int64_t p = idx / n;
  const int i = int(idx - p * n);
  const int F = g.d + 1;
  double S = 1.0, A = 0.0, bsum = 0.0;
  for (int k = 0; k < g.d; ++k) {
    const int x = int((p / g.stride[k]) % g.M[k]);
    const double w0 = g.W[k][x * 3], w1 = g.W[k][x * 3 + 1], w2 = g.W[k][x * 3 + 2];
    const double a = w1 / w0, v = w2 / w0 - a * a;
    S *= w0;
    A += a * a / v;
    bsum += (a / v) * Zn[(p * F + 1 + k) * n + i];
  }
  const double z0 = Zn[(p * F) * n + i];
  const double B = (A * z0 - bsum) / S;
  Ln[p * n + i] = z0 / S + B;
  Bn[p * n + i] = B;
}

// ------------------------------------------------------------------ low rank
// Partial products over 64 rows: part[blk][i][c] = sum_t L[t][i] X[t][c],
// part[blk][n + i][c] likewise with B, part[blk][2n][c] = sum_t mu[t] X[t][c].
__global__ __launch_bounds__(256) void k_lr_partial(CovGeo g, int r, const double *__restrict__ X,
                                                    const double *__restrict__ Ln, const double *__restrict__ Bn,
                                                    const double *__restrict__ mu, double *__restrict__ part) {
  __shared__ double Xs[64][64];
  __shared__ double ms[64];
  const int n = g.n;
  const int64_t blk = blockIdx.x, row0 = blk * 64;
  const int nrows = int(min<int64_t>(64, g.P - row0));
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int t = e >> 6, c = e & 63;
    Xs[t][c] = (t < nrows && c < r) ? X[(row0 + t) * r + c] : 0.0;
  }
  if (threadIdx.x < 64) ms[threadIdx.x] = threadIdx.x < nrows ? mu[row0 + threadIdx.x] : 0.0;
  __syncthreads();
  const int il = threadIdx.x & 63, cq = threadIdx.x >> 6;
  const int i = blockIdx.y * 64 + il;
  const int64_t base = blk * (2 * int64_t(n) + 1);
  if (i < n) {
    double u[16], v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) u[j] = v[j] = 0.0;
    for (int t = 0; t < nrows; ++t) {
      const double l = Ln[(row0 + t) * n + i], b = Bn[(row0 + t) * n + i];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double x = Xs[t][cq + 4 * j];
        u[j] = fma(l, x, u[j]);
        v[j] = fma(b, x, v[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c = cq + 4 * j;
      if (c < r) {
        part[(base + i) * 64 + c] = u[j];
        part[(base + n + i) * 64 + c] = v[j];
      }
    }
  }
  if (blockIdx.y == 0 && threadIdx.x < r) {
    double s = 0.0;
    for (int t = 0; t < nrows; ++t) s = fma(ms[t], Xs[t][threadIdx.x], s);
    part[(base + 2 * n) * 64 + threadIdx.x] = s;
  }
}

// tot[j][c] = sum over the row blocks of part[b][j][c]: one workgroup per row
// j; thread (group g, column c) adds blocks g, g + 4, ... (eight loads in
// flight), then the four groups are added in order.
__global__ __launch_bounds__(256) void k_lr_reduce(int64_t nblk, int rows, int r, const double *__restrict__ part,
                                                   double *__restrict__ tot) {
  __shared__ double gs[4][64];
  const int j = blockIdx.x, c = threadIdx.x & 63, g = threadIdx.x >> 6;
  double s = 0.0;
  if (c < r) {
    int64_t b = g;
    for (; b + 28 < nblk; b += 32) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[((b + 4 * u) * rows + j) * 64 + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < nblk; b += 4) s += part[(b * rows + j) * 64 + c];
  }
  gs[g][c] = s;
  __syncthreads();
  if (g == 0 && c < r) tot[int64_t(j) * 64 + c] = ((gs[0][c] + gs[1][c]) + gs[2][c]) + gs[3][c];
}

// out[s][c] = (1/n) sum_i (L[s][i] U[i][c] - B[s][i] V[i][c]) - mu[s] m[c]
__global__ __launch_bounds__(256) void k_lr_out(CovGeo g, int r, const double *__restrict__ Ln,
                                                const double *__restrict__ Bn, const double *__restrict__ mu,
                                                const double *__restrict__ tot, double *__restrict__ out) {
  __shared__ double Us[32][64], Vs[32][64];
  __shared__ double Ls[64][33], Bs[64][33];
  const int n = g.n;
  const int64_t row0 = int64_t(blockIdx.x) * 64;
  const int nrows = int(min<int64_t>(64, g.P - row0));
  const int sl = threadIdx.x >> 2, cq = threadIdx.x & 3;
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  for (int i0 = 0; i0 < n; i0 += 32) {
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 64; e += 256) {
      const int ii = e >> 6, c = e & 63;
      const bool ok = i0 + ii < n && c < r;
      Us[ii][c] = ok ? tot[int64_t(i0 + ii) * 64 + c] : 0.0;
      Vs[ii][c] = ok ? tot[int64_t(n + i0 + ii) * 64 + c] : 0.0;
    }
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int t = e >> 5, ii = e & 31;
      const bool ok = t < nrows && i0 + ii < n;
      Ls[t][ii] = ok ? Ln[(row0 + t) * n + i0 + ii] : 0.0;
      Bs[t][ii] = ok ? Bn[(row0 + t) * n + i0 + ii] : 0.0;
    }
    __syncthreads();
    for (int ii = 0; ii < 32; ++ii) {
      const double l = Ls[sl][ii], b = Bs[sl][ii];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = fma(l, Us[ii][cq + 4 * j], fma(-b, Vs[ii][cq + 4 * j], acc[j]));
    }
  }
  if (sl < nrows) {
    const double m = mu[row0 + sl];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c = cq + 4 * j;
      if (c < r) out[(row0 + sl) * r + c] = acc[j] * g.inv_n - m * tot[int64_t(2 * n) * 64 + c];
    }
  }
}

// ------------------------------------------------------------------ band
// Per-coordinate exponent index of each weight moment (S0, S1[D], S2 upper
// triangle row by row) for D = 2d coordinates s_0..s_{d-1}, t_0..t_{d-1}:
// 0 = (0,0), 1 = (1,0), 2 = (0,1), 3 = (2,0), 4 = (1,1), 5 = (0,2) as powers of
// (u_k, v_k).
template <int d>
__device__ constexpr int mom_ab(int q, int k) {
  constexpr int D = 2 * d;
  if (q == 0) return 0;
  if (q <= D) {
    const int j = q - 1;
    return (j % d == k) ? (j < d ? 1 : 2) : 0;
  }
  int idx = q - 1 - D;
  int j = 0;
  while (idx >= D - j) {
    idx -= D - j;
    ++j;
  }
  const int l = j + idx;
  const int kj = j % d, kl = l % d;
  const bool sj = j < d, sl = l < d;
  if (kj == kl) {
    if (kj != k) return 0;
    if (j == l) return sj ? 3 : 5;
    return 4;
  }
  if (k == kj) return sj ? 1 : 2;
  if (k == kl) return sl ? 1 : 2;
  return 0;
}

// m[q] = prod_k P_k[ab(q,k)] - prod_k E_k[ab(q,k)] with every index fixed at
// compile time (the per-coordinate factors stay in registers).
template <int d, int q>
__device__ inline double weight_moment(const double (&Pk)[3][6], const double (&Ek)[3][6]) {
  constexpr int a0 = mom_ab<d>(q, 0);
  constexpr int a1 = d > 1 ? mom_ab<d>(q, 1) : 0;
  constexpr int a2 = d > 2 ? mom_ab<d>(q, 2) : 0;
  double pp = Pk[0][a0], ee = Ek[0][a0];
  if constexpr (d > 1) {
    pp *= Pk[1][a1];
    ee *= Ek[1][a1];
  }
  if constexpr (d > 2) {
    pp *= Pk[2][a2];
    ee *= Ek[2][a2];
  }
  return pp - ee;
}

template <int d, int... q>
__device__ inline void fill_weight_moments(const double (&Pk)[3][6], const double (&Ek)[3][6], double *m,
                                           std::integer_sequence<int, q...>) {
  ((m[q] = weight_moment<d, q>(Pk, Ek)), ...);
}

struct BandArgs {
  CovGeo g;
  const double *Zn;
  const double *Y2;
  const double *X;  // fused product: P x r
  int r;
  double *out;
  double *band;  // stored blocks
};

// Local node li of a tile (coordinate d-1 fastest) and its grid coordinates.
template <int d>
__device__ inline void tile_node(int li, const int *lo, const CovGeo &g, int *x, bool *ok, int64_t *p) {
  constexpr int TB = tile_ext<d>();
  int rem = li;
  bool v = true;
  int64_t q = 0;
#pragma unroll
  for (int k = d - 1; k >= 0; --k) {
    x[k] = lo[k] + rem % TB;
    rem /= TB;
    v = v && x[k] < g.M[k];
    q += int64_t(x[k]) * g.stride[k];
  }
  *ok = v;
  *p = q;
}

constexpr int ZH = 34;  // padded row of the 32 t-nodes of a half tile

template <int d>
constexpr int band_union_doubles() {
  constexpr int zc = (d + 1) * NC * (ZP + ZH);
  constexpr int dx = 64 * 33 + 32 * 64;
  return zc > dx ? zc : dx;
}

template <int d>
constexpr int band_lds_doubles() {
  // union region (curve chunks | Delta and X tiles) + Y2 box + mode-product buffers
  constexpr int extra = d == 3 ? (3 * 16 * 16 * 3 + 16 * 16 * 3 + 16 * 16 * 5) : (d == 2 ? 64 * 8 * 3 : 0);
  return band_union_doubles<d>() + 4096 + extra;
}

// Per s-tile: every t-tile within reach of the band, each in two halves of 32
// t-nodes (4 nodes per thread keep the FP64 solve within the registers).
template <int d, bool STORE>
__global__ __launch_bounds__(BT) void k_band(BandArgs A) {
  constexpr int D = 2 * d;
  constexpr int NT = 2 * d + 1;  // response moments
  constexpr int NS = 1 + D + D * (D + 1) / 2;
  constexpr int TB = tile_ext<d>();
  constexpr int UN = band_union_doubles<d>();
  extern __shared__ double sm[];
  double *Zs = sm;                      // [d+1][NC][ZP]: the 64 s-nodes
  double *Zt = sm + (d + 1) * NC * ZP;  // [d+1][NC][ZH]: the 32 t-nodes of the half
  double *Dl = sm;                      // [64][33]
  double *Xl = sm + 64 * 33;            // [32][64]
  double *Yb = sm + UN;                 // Y2 box
  double *Fb = Yb + 4096;               // d = 3: F[3][16][16][3]; d = 2: V[64][8][3]
  double *V3 = Fb + 3 * 16 * 16 * 3;    // d = 3: [16][16][3]
  double *V2 = V3 + 16 * 16 * 3;        // d = 3: [16][16][5]
  __shared__ long long sidx[64], tidx[64];
  __shared__ int sok[64], tok[64];

  const CovGeo &g = A.g;
  const int n = g.n;
  const int tid = threadIdx.x;
  const int a = tid >> 4, b = tid & 15;  // s-locals 2a, 2a+1; t-locals 32 hh + 2b, + 1
  int sa[3] = {0, 0, 0}, s0[3] = {0, 0, 0};
  {
    int64_t rem = blockIdx.x;
#pragma unroll
    for (int k = d - 1; k >= 0; --k) {
      sa[k] = int(rem % g.nt[k]);
      rem /= g.nt[k];
      s0[k] = sa[k] * TB;
    }
  }
  if (tid < 64) {
    int x[3];
    bool ok;
    int64_t p;
    tile_node<d>(tid, s0, g, x, &ok, &p);
    sok[tid] = ok;
    sidx[tid] = ok ? p : 0;
  }
  int sl[2][3];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    int rem = 2 * a + x;
#pragma unroll
    for (int k = d - 1; k >= 0; --k) {
      sl[x][k] = rem % TB;
      rem /= TB;
    }
  }
  const int ro = tid >> 3, cg = tid & 7;  // fused product: s-row and column group
  double acco[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acco[j] = 0.0;

  for (int o = 0; o < g.nslot; ++o) {
    int t0[3] = {0, 0, 0};
    bool inside = true;
    {
      int rem = o;
#pragma unroll
      for (int k = d - 1; k >= 0; --k) {
        const int w = 2 * g.span[k] + 1;
        const int c = sa[k] + rem % w - g.span[k];
        rem /= w;
        inside = inside && c >= 0 && c < g.nt[k];
        t0[k] = c * TB;
      }
    }
    if (!inside) continue;  // uniform across the workgroup
    __syncthreads();        // readers of the previous tile pair's tables are done
    if (tid < 64) {
      int x[3];
      bool ok;
      int64_t p;
      tile_node<d>(tid, t0, g, x, &ok, &p);
      tok[tid] = ok;
      tidx[tid] = ok ? p : 0;
    }
    // Y2 over the nodes shared by some s- and t-window of the tile pair, and
    // (d = 3) the 1-D factor tables F[k][q = sl*4 + tl][p][ab]
    int plo[3], np[3];
    bool any = true;
#pragma unroll
    for (int k = 0; k < d; ++k) {
      const int shi = min(s0[k] + TB - 1, g.M[k] - 1), thi = min(t0[k] + TB - 1, g.M[k] - 1);
      plo[k] = max(max(s0[k], t0[k]) - g.R[k], 0);
      const int phi = min(min(shi, thi) + g.R[k], g.M[k] - 1);
      np[k] = phi - plo[k] + 1;
      any = any && np[k] > 0;
    }
    if (any) {
      int nbx = 1;
#pragma unroll
      for (int k = 0; k < d; ++k) nbx *= np[k];
      for (int e = tid; e < nbx; e += BT) {
        int rem = e;
        int64_t p = 0;
#pragma unroll
        for (int k = d - 1; k >= 0; --k) {
          p += int64_t(plo[k] + rem % np[k]) * g.stride[k];
          rem /= np[k];
        }
        Yb[e] = A.Y2[p];
      }
      if constexpr (d == 3) {
        for (int e = tid; e < 3 * 16 * 16 * 3; e += BT) {
          const int k = e / 768, rem = e - k * 768;
          const int q = rem / 48, rem2 = rem - q * 48;
          const int pi = rem2 / 3, ab = rem2 - pi * 3;
          double f = 0.0;
          if (pi < np[k]) {
            const int R = g.R[k];
            const int s = s0[k] + (q >> 2), t = t0[k] + (q & 3), p = plo[k] + pi;
            const int ds = p - s, dt = p - t;
            if (ds >= -R && ds <= R && dt >= -R && dt <= R) {
              f = g.K[k][ds + R] * g.K[k][dt + R];
              if (ab == 1) f *= g.U[k][ds + R];
              if (ab == 2) f *= g.U[k][dt + R];
            }
          }
          Fb[e] = f;
        }
      }
    }

    for (int hh = 0; hh < 2; ++hh) {
      int tl[2][3];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        int rem = 32 * hh + 2 * b + y;
#pragma unroll
        for (int k = d - 1; k >= 0; --k) {
          tl[y][k] = rem % TB;
          rem /= TB;
        }
      }
      // ---- 1. response moments of the full pair sums
      double acc[2][2][NT];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int q = 0; q < NT; ++q) acc[x][y][q] = 0.0;
      for (int i0 = 0; i0 < n; i0 += NC) {
        __syncthreads();
        constexpr int ps = (d + 1) * NC * 64, pt = (d + 1) * NC * 32;
        for (int e = tid; e < ps + pt; e += BT) {
          const bool side = e >= ps;
          const int rem = side ? e - ps : e;
          const int node = rem / ((d + 1) * NC);
          const int fi = rem - node * ((d + 1) * NC);
          const int f = fi / NC, ii = fi - f * NC;
          const int tn = 32 * hh + node;
          const bool ok = (side ? tok[tn] : sok[node]) && i0 + ii < n;
          const long long p = side ? tidx[tn] : sidx[node];
          const double v = ok ? A.Zn[(p * (d + 1) + f) * n + i0 + ii] : 0.0;
          if (side)
            Zt[(f * NC + ii) * ZH + node] = v;
          else
            Zs[(f * NC + ii) * ZP + node] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int ii = 0; ii < NC; ++ii) {
          double zs[2][d + 1], zt[2][d + 1];
#pragma unroll
          for (int f = 0; f <= d; ++f) {
            const double2 s2 = *reinterpret_cast<const double2 *>(&Zs[(f * NC + ii) * ZP + 2 * a]);
            const double2 t2 = *reinterpret_cast<const double2 *>(&Zt[(f * NC + ii) * ZH + 2 * b]);
            zs[0][f] = s2.x;
            zs[1][f] = s2.y;
            zt[0][f] = t2.x;
            zt[1][f] = t2.y;
          }
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
              acc[x][y][0] = fma(zs[x][0], zt[y][0], acc[x][y][0]);
#pragma unroll
              for (int k = 0; k < d; ++k) {
                acc[x][y][1 + k] = fma(zs[x][k + 1], zt[y][0], acc[x][y][1 + k]);
                acc[x][y][1 + d + k] = fma(zs[x][0], zt[y][k + 1], acc[x][y][1 + d + k]);
              }
            }
        }
      }

      // closed-form (tensor-product) intercept from the full moments
      double low[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          double S = 1.0, fac = 1.0, lin = 0.0;
#pragma unroll
          for (int k = 0; k < d; ++k) {
            const int xs = min(s0[k] + sl[x][k], g.M[k] - 1), xt = min(t0[k] + tl[y][k], g.M[k] - 1);
            const double *Wk = g.W[k];
            const double s0w = Wk[xs * 3], s1w = Wk[xs * 3 + 1], s2w = Wk[xs * 3 + 2];
            const double t0w = Wk[xt * 3], t1w = Wk[xt * 3 + 1], t2w = Wk[xt * 3 + 2];
            const double as = s1w / s0w, vs = s2w / s0w - as * as;
            const double at = t1w / t0w, vt = t2w / t0w - at * at;
            S *= s0w * t0w;
            fac += as * as / vs + at * at / vt;
            lin += (as / vs) * acc[x][y][1 + k] + (at / vt) * acc[x][y][1 + d + k];
          }
          low[x][y] = (acc[x][y][0] * fac - lin) * g.inv_n / S;
        }

      // ---- 2. diagonal correction: subtract sum_p f(p; s,t) Y2(p) from acc
      if (any) {
        if constexpr (d == 1) {
          const int R = g.R[0];
          const double *K0 = g.K[0], *U0 = g.U[0];
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
              const int s = s0[0] + sl[x][0], t = t0[0] + tl[y][0];
              const int lo = max(max(s, t) - R, 0), hi = min(min(s, t) + R, g.M[0] - 1);
              double c0 = 0.0, c1 = 0.0, c2 = 0.0;
              for (int p = lo; p <= hi; ++p) {
                const double kk = K0[p - s + R] * K0[p - t + R] * Yb[p - plo[0]];
                c0 += kk;
                c1 = fma(kk, U0[p - s + R], c1);
                c2 = fma(kk, U0[p - t + R], c2);
              }
              acc[x][y][0] -= c0;
              acc[x][y][1] -= c1;
              acc[x][y][2] -= c2;
            }
        } else if constexpr (d == 2) {
          const int R0 = g.R[0], R1 = g.R[1];
          const double *K0 = g.K[0], *U0 = g.U[0], *K1 = g.K[1], *U1 = g.U[1];
          double *V = Fb;  // [np0][8][3]
          for (int hs = 0; hs < 4; ++hs) {
#pragma unroll
            for (int x = 0; x < 2; ++x) {
              const int s1 = s0[1] + 2 * hs + x;
              // V[p0][tl][ab] = sum_p1 f1(p1; s1, t1)^{ab} Y2(p0, p1)
              for (int e = tid; e < np[0] * 8 * 3; e += BT) {
                const int p0i = e / 24, rem = e - p0i * 24;
                const int tlc = rem / 3, ab = rem - tlc * 3;
                const int t1 = t0[1] + tlc;
                double sacc = 0.0;
                for (int p1i = 0; p1i < np[1]; ++p1i) {
                  const int p1 = plo[1] + p1i;
                  const int ds = p1 - s1, dt = p1 - t1;
                  if (ds < -R1 || ds > R1 || dt < -R1 || dt > R1) continue;
                  double f = K1[ds + R1] * K1[dt + R1];
                  if (ab == 1) f *= U1[ds + R1];
                  if (ab == 2) f *= U1[dt + R1];
                  sacc = fma(f, Yb[p0i * np[1] + p1i], sacc);
                }
                V[e] = sacc;
              }
              __syncthreads();
              if ((a & 3) == hs) {
                const int s0c = s0[0] + sl[x][0];
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                  const int t0c = t0[0] + tl[y][0];
                  const int tlc = tl[y][1];
                  double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                  for (int p0i = 0; p0i < np[0]; ++p0i) {
                    const int p0 = plo[0] + p0i;
                    const int ds = p0 - s0c, dt = p0 - t0c;
                    if (ds < -R0 || ds > R0 || dt < -R0 || dt > R0) continue;
                    const double f = K0[ds + R0] * K0[dt + R0];
                    const double *v = &V[(p0i * 8 + tlc) * 3];
                    c[0] = fma(f, v[0], c[0]);
                    c[1] = fma(f * U0[ds + R0], v[0], c[1]);
                    c[2] = fma(f * U0[dt + R0], v[0], c[2]);
                    c[3] = fma(f, v[1], c[3]);
                    c[4] = fma(f, v[2], c[4]);
                  }
                  // order of acc: T0, s0, s1, t0, t1
                  acc[x][y][0] -= c[0];
                  acc[x][y][1] -= c[1];
                  acc[x][y][3] -= c[2];
                  acc[x][y][2] -= c[3];
                  acc[x][y][4] -= c[4];
                }
              }
              __syncthreads();
            }
          }
        } else {
          // s-locals: s2 = 2 (a & 1) + x, s1 = (a >> 1) & 3, s0 = a >> 3;
          // t-locals: t2 = 2 (b & 1) + y, t1 = (b >> 1) & 3, t0 = 2 hh + (b >> 3)
          const int s1l = (a >> 1) & 3, s0l = a >> 3;
          const int t1l = (b >> 1) & 3, t0l = 2 * hh + (b >> 3);
          for (int hs = 0; hs < 2; ++hs)
            for (int ht = 0; ht < 2; ++ht) {
#pragma unroll
              for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                  const int q2 = (2 * hs + x) * 4 + 2 * ht + y;
                  // (a) V3[p0][p1][ab] = sum_p2 F2[q2][p2][ab] Y2(p0,p1,p2)
                  for (int e = tid; e < np[0] * np[1] * 3; e += BT) {
                    const int p01 = e / 3, ab = e - p01 * 3;
                    const double *Fr = &Fb[(2 * 256 + q2 * 16) * 3 + ab];
                    const double *Yr = &Yb[p01 * np[2]];
                    double sacc = 0.0;
                    for (int p2 = 0; p2 < np[2]; ++p2) sacc = fma(Fr[p2 * 3], Yr[p2], sacc);
                    V3[e] = sacc;
                  }
                  __syncthreads();
                  // (b) V2[p0][q1][c5]; c5 = (ab1, ab2): 00 00, 10 00, 01 00, 00 10, 00 01
                  for (int e = tid; e < np[0] * 16 * 5; e += BT) {
                    const int p0 = e / 80, rem = e - p0 * 80;
                    const int q1 = rem / 5, c5 = rem - q1 * 5;
                    const int ab1 = c5 < 3 ? c5 : 0, ab2 = c5 < 3 ? 0 : c5 - 2;
                    const double *Fr = &Fb[(256 + q1 * 16) * 3 + ab1];
                    const double *Vr = &V3[(p0 * np[1]) * 3 + ab2];
                    double sacc = 0.0;
                    for (int p1 = 0; p1 < np[1]; ++p1) sacc = fma(Fr[p1 * 3], Vr[p1 * 3], sacc);
                    V2[e] = sacc;
                  }
                  __syncthreads();
                  // (c) the owners of (s2, t2): sum over p0
                  if ((a & 1) == hs && (b & 1) == ht) {
                    const int q0 = s0l * 4 + t0l, q1 = s1l * 4 + t1l;
                    double c[7] = {0, 0, 0, 0, 0, 0, 0};
                    for (int p0 = 0; p0 < np[0]; ++p0) {
                      const double *Fr = &Fb[(q0 * 16 + p0) * 3];
                      const double *Vr = &V2[(p0 * 16 + q1) * 5];
                      c[0] = fma(Fr[0], Vr[0], c[0]);  // T0
                      c[1] = fma(Fr[1], Vr[0], c[1]);  // s0
                      c[2] = fma(Fr[2], Vr[0], c[2]);  // t0
                      c[3] = fma(Fr[0], Vr[1], c[3]);  // s1
                      c[4] = fma(Fr[0], Vr[2], c[4]);  // t1
                      c[5] = fma(Fr[0], Vr[3], c[5]);  // s2
                      c[6] = fma(Fr[0], Vr[4], c[6]);  // t2
                    }
                    // order of acc: T0, s0, s1, s2, t0, t1, t2
                    acc[x][y][0] -= c[0];
                    acc[x][y][1] -= c[1];
                    acc[x][y][2] -= c[3];
                    acc[x][y][3] -= c[5];
                    acc[x][y][4] -= c[2];
                    acc[x][y][5] -= c[4];
                    acc[x][y][6] -= c[6];
                  }
                }
            }
        }
      }

      // ---- 3. weight moments, the solve and Delta
      double delta[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int si = 2 * a + x, ti = 32 * hh + 2 * b + y;
          bool inb = sok[si] && tok[ti];
          double Pk[3][6], Ek[3][6];
#pragma unroll
          for (int k = 0; k < d; ++k) {
            const int xs = min(s0[k] + sl[x][k], g.M[k] - 1), xt = min(t0[k] + tl[y][k], g.M[k] - 1);
            const int dl = xt - xs;
            const int R2 = 2 * g.R[k];
            inb = inb && dl >= -R2 && dl <= R2;
            const double *Wk = g.W[k];
            const double ws0 = Wk[xs * 3], ws1 = Wk[xs * 3 + 1], ws2 = Wk[xs * 3 + 2];
            const double wt0 = Wk[xt * 3], wt1 = Wk[xt * 3 + 1], wt2 = Wk[xt * 3 + 2];
            Pk[k][0] = ws0 * wt0;
            Pk[k][1] = ws1 * wt0;
            Pk[k][2] = ws0 * wt1;
            Pk[k][3] = ws2 * wt0;
            Pk[k][4] = ws1 * wt1;
            Pk[k][5] = ws0 * wt2;
            const int dc = min(max(dl, -R2), R2);
            const double *Er = &g.E[k][(int64_t(xs) * (2 * R2 + 1) + dc + R2) * 6];
#pragma unroll
            for (int j = 0; j < 6; ++j) Ek[k][j] = Er[j];
          }
          double dv = 0.0;
          if (inb) {
            double m[NS + NT];
            fill_weight_moments<d>(Pk, Ek, m, std::make_integer_sequence<int, NS>{});
#pragma unroll
            for (int q = 0; q < NT; ++q) m[NS + q] = acc[x][y][q] * g.inv_n;
            int8_t st;
            const double b0 = wls_b0<D>(m, &st);
            dv = b0 - low[x][y];
          }
          delta[x][y] = dv;
          // one element's solve at a time: no interleaving of their registers
          __builtin_amdgcn_sched_barrier(0);
        }

      // ---- 4. output
      if constexpr (STORE) {
        double *blk = A.band + (int64_t(blockIdx.x) * g.nslot + o) * 4096;
#pragma unroll
        for (int x = 0; x < 2; ++x)
          *reinterpret_cast<double2 *>(&blk[(2 * a + x) * 64 + 32 * hh + 2 * b]) =
              make_double2(delta[x][0], delta[x][1]);
      } else {
        __syncthreads();  // all readers of the curve chunks are done
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) Dl[(2 * a + x) * 33 + 2 * b + y] = delta[x][y];
        for (int e = tid; e < 32 * 64; e += BT) {
          const int t = e >> 6, c = e & 63;
          const int tn = 32 * hh + t;
          Xl[e] = (tok[tn] && c < A.r) ? A.X[tidx[tn] * A.r + c] : 0.0;
        }
        __syncthreads();
        for (int t = 0; t < 32; ++t) {
          const double dd = Dl[ro * 33 + t];
#pragma unroll
          for (int j = 0; j < 8; ++j) acco[j] = fma(dd, Xl[t * 64 + cg + 8 * j], acco[j]);
        }
      }
    }
  }
  if constexpr (!STORE) {
    if (sok[ro]) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = cg + 8 * j;
        if (c < A.r) A.out[sidx[ro] * A.r + c] += acco[j];
      }
    }
  }
}

// Product with the stored band blocks.
template <int d>
__global__ __launch_bounds__(BT) void k_band_apply(BandArgs A) {
  constexpr int TB = tile_ext<d>();
  extern __shared__ double sm[];
  double *Dl = sm;            // [64][65]
  double *Xl = sm + 64 * 65;  // [64][64]
  __shared__ long long sidx[64], tidx[64];
  __shared__ int sok[64], tok[64];
  const CovGeo &g = A.g;
  const int tid = threadIdx.x;
  int sa[3] = {0, 0, 0}, s0[3] = {0, 0, 0};
  {
    int64_t rem = blockIdx.x;
#pragma unroll
    for (int k = d - 1; k >= 0; --k) {
      sa[k] = int(rem % g.nt[k]);
      rem /= g.nt[k];
      s0[k] = sa[k] * TB;
    }
  }
  if (tid < 64) {
    int x[3];
    bool ok;
    int64_t p;
    tile_node<d>(tid, s0, g, x, &ok, &p);
    sok[tid] = ok;
    sidx[tid] = ok ? p : 0;
  }
  const int ro = tid >> 3, cg = tid & 7;
  double acco[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acco[j] = 0.0;
  for (int o = 0; o < g.nslot; ++o) {
    int t0[3] = {0, 0, 0};
    bool inside = true;
    {
      int rem = o;
#pragma unroll
      for (int k = d - 1; k >= 0; --k) {
        const int w = 2 * g.span[k] + 1;
        const int c = sa[k] + rem % w - g.span[k];
        rem /= w;
        inside = inside && c >= 0 && c < g.nt[k];
        t0[k] = c * TB;
      }
    }
    if (!inside) continue;
    __syncthreads();
    if (tid < 64) {
      int x[3];
      bool ok;
      int64_t p;
      tile_node<d>(tid, t0, g, x, &ok, &p);
      tok[tid] = ok;
      tidx[tid] = ok ? p : 0;
    }
    const double *blk = A.band + (int64_t(blockIdx.x) * g.nslot + o) * 4096;
    for (int e = tid; e < 4096; e += BT) Dl[(e >> 6) * 65 + (e & 63)] = blk[e];
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += BT) {
      const int t = e >> 6, c = e & 63;
      Xl[e] = (tok[t] && c < A.r) ? A.X[tidx[t] * A.r + c] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < 64; ++t) {
      const double dd = Dl[ro * 65 + t];
#pragma unroll
      for (int j = 0; j < 8; ++j) acco[j] = fma(dd, Xl[t * 64 + cg + 8 * j], acco[j]);
    }
  }
  if (sok[ro]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cg + 8 * j;
      if (c < A.r) A.out[sidx[ro] * A.r + c] += acco[j];
    }
  }
}

// ------------------------------------------------------------------ host
CovGeo make_geo(const fpca_covop_s *op) {
  CovGeo g{};
  g.d = op->d;
  int64_t st = 1;
  for (int k = 2; k >= 0; --k) {
    g.M[k] = k < op->d ? op->M[k] : 1;
    g.R[k] = k < op->d ? op->R[k] : 0;
  }
  for (int k = op->d - 1; k >= 0; --k) {
    g.stride[k] = st;
    st *= op->M[k];
  }
  g.P = op->P;
  g.n = int(op->n);
  g.inv_n = 1.0 / double(op->n);
  for (int k = 0; k < op->d; ++k) {
    g.K[k] = op->tab + op->tab_K[k];
    g.U[k] = op->tab + op->tab_U[k];
    g.W[k] = op->tab + op->tab_W[k];
    g.E[k] = op->tab + op->tab_E[k];
    g.tb[k] = op->tb[k];
    g.nt[k] = op->nt[k];
    g.span[k] = op->span[k];
  }
  g.nslot = op->nslot;
  return g;
}

unsigned nb256(int64_t n) { return unsigned((n + 255) / 256); }

template <int d>
int launch_band(fpca_covop_s *op, bool store, const double *X, int r, double *out) {
  BandArgs A{};
  A.g = make_geo(op);
  A.Zn = op->Zn;
  A.Y2 = op->Y2;
  A.X = X;
  A.r = r;
  A.out = out;
  A.band = op->band;
  const size_t lds = size_t(band_lds_doubles<d>()) * 8;
  if (store) {
    FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band<d, true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL((k_band<d, true>), dim3(unsigned(op->n_stiles)), dim3(BT), lds, op->ctx->stream, A);
  } else {
    FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band<d, false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL((k_band<d, false>), dim3(unsigned(op->n_stiles)), dim3(BT), lds, op->ctx->stream, A);
  }
  FPCA_LAUNCH_CHECK("covop band");
  return FPCA_OK;
}

template <int d>
int launch_band_apply(fpca_covop_s *op, const double *X, int r, double *out) {
  BandArgs A{};
  A.g = make_geo(op);
  A.X = X;
  A.r = r;
  A.out = out;
  A.band = op->band;
  const size_t lds = size_t(64 * 65 + 64 * 64) * 8;
  FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band_apply<d>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL((k_band_apply<d>), dim3(unsigned(op->n_stiles)), dim3(BT), lds, op->ctx->stream, A);
  FPCA_LAUNCH_CHECK("covop band apply");
  return FPCA_OK;
}

int band_dispatch(fpca_covop_s *op, bool store, const double *X, int r, double *out) {
  switch (op->d) {
    case 1: return launch_band<1>(op, store, X, r, out);
    case 2: return launch_band<2>(op, store, X, r, out);
    default: return launch_band<3>(op, store, X, r, out);
  }
}

}  // namespace

int covop_apply_internal(fpca_covop_s *op, int r, const double *X, double *out) {
  fpca_context *ctx = op->ctx;
  const CovGeo g = make_geo(op);
  const int rows = int(2 * op->n + 1);
  hipLaunchKernelGGL(k_lr_partial, dim3(unsigned(op->lr_blocks), unsigned((op->n + 63) / 64)), dim3(256), 0,
                     ctx->stream, g, r, X, op->Ln, op->Bn, op->mu, op->lr_part);
  FPCA_LAUNCH_CHECK("covop lr partial");
  hipLaunchKernelGGL(k_lr_reduce, dim3(unsigned(rows)), dim3(256), 0, ctx->stream, op->lr_blocks, rows, r,
                     op->lr_part, op->lr_tot);
  FPCA_LAUNCH_CHECK("covop lr reduce");
  hipLaunchKernelGGL(k_lr_out, dim3(unsigned((op->P + 63) / 64)), dim3(256), 0, ctx->stream, g, r, op->Ln, op->Bn,
                     op->mu, op->lr_tot, out);
  FPCA_LAUNCH_CHECK("covop lr out");
  if (op->mode == FPCA_COVOP_STORE_BAND) {
    switch (op->d) {
      case 1: return launch_band_apply<1>(op, X, r, out);
      case 2: return launch_band_apply<2>(op, X, r, out);
      default: return launch_band_apply<3>(op, X, r, out);
    }
  }
  return band_dispatch(op, false, X, r, out);
}

}  // namespace fpca

using namespace fpca;

extern "C" int fpca_covop_create(fpca_handle ctx, const fpca_grid *grid, int64_t n, const double *Y,
                                 const double *mu, const double *bandwidth, int mode, fpca_covop *op_out) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (!op_out) return set_error(FPCA_ERR_INVALID_ARG, "op is required");
  *op_out = nullptr;
  if (!Y || !mu || !bandwidth) return set_error(FPCA_ERR_INVALID_ARG, "Y, mu and bandwidth are required");
  if (grid->mask) return set_error(FPCA_ERR_UNSUPPORTED, "the covariance operator takes the full rectangle only");
  if (n < 1 || n > (int64_t(1) << 20)) return set_error(FPCA_ERR_INVALID_ARG, "need 1 <= n <= 2^20");
  if (mode != FPCA_COVOP_RECOMPUTE && mode != FPCA_COVOP_STORE_BAND)
    return set_error(FPCA_ERR_INVALID_ARG, "bad mode %d", mode);
  const int d = grid->d;
  const int rmax = d == 3 ? 6 : (d == 2 ? 28 : 2016);
  auto *op = new fpca_covop_s();
  op->ctx = ctx;
  op->d = d;
  op->P = P;
  op->n = n;
  op->mode = mode;
  std::vector<double> htab;
  for (int k = 0; k < d; ++k) {
    const int M = grid->M[k];
    const double h = bandwidth[k];
    if (!(h > 0.0) || !std::isfinite(h)) {
      delete op;
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidths must be positive and finite");
    }
    const double H = h * double(M - 1);
    const int R = std::min(int(std::floor(H)), M - 1);
    if (R < 1 || R > rmax) {
      delete op;
      return set_error(FPCA_ERR_UNSUPPORTED, "coordinate %d: window of %d grid steps (need 1..%d)", k, R, rmax);
    }
    op->M[k] = M;
    op->R[k] = R;
    op->H[k] = H;
    // taps, window sums and shared-node sums
    std::vector<double> K(2 * R + 1), U(2 * R + 1);
    for (int m = -R; m <= R; ++m) {
      const double u = double(m) / H;
      K[m + R] = std::fabs(u) < 1.0 ? 1.0 - u * u : 0.0;
      U[m + R] = u;
    }
    std::vector<double> W(size_t(M) * 3), E(size_t(M) * (4 * R + 1) * 6, 0.0);
    for (int x = 0; x < M; ++x) {
      double w0 = 0, w1 = 0, w2 = 0;
      for (int m = -std::min(R, x); m <= std::min(R, M - 1 - x); ++m) {
        w0 += K[m + R];
        w1 += K[m + R] * U[m + R];
        w2 += K[m + R] * U[m + R] * U[m + R];
      }
      W[x * 3] = w0;
      W[x * 3 + 1] = w1;
      W[x * 3 + 2] = w2;
      const double a = w1 / w0, v = w2 / w0 - a * a;
      if (!(w0 > 0.0) || !(v >= 1e-8 * (w2 / w0))) {
        delete op;
        return set_error(FPCA_ERR_UNSUPPORTED, "coordinate %d: degenerate window at node %d", k, x);
      }
      for (int dl = -2 * R; dl <= 2 * R; ++dl) {
        const int t = x + dl;
        if (t < 0 || t >= M) continue;
        double e[6] = {0, 0, 0, 0, 0, 0};
        for (int p = std::max(std::max(x, t) - R, 0); p <= std::min(std::min(x, t) + R, M - 1); ++p) {
          const double kk = K[p - x + R] * K[p - t + R], us = U[p - x + R], vt = U[p - t + R];
          e[0] += kk;
          e[1] += kk * us;
          e[2] += kk * vt;
          e[3] += kk * us * us;
          e[4] += kk * us * vt;
          e[5] += kk * vt * vt;
        }
        for (int j = 0; j < 6; ++j) E[(size_t(x) * (4 * R + 1) + dl + 2 * R) * 6 + j] = e[j];
      }
    }
    op->tab_K[k] = int64_t(htab.size());
    htab.insert(htab.end(), K.begin(), K.end());
    op->tab_U[k] = int64_t(htab.size());
    htab.insert(htab.end(), U.begin(), U.end());
    op->tab_W[k] = int64_t(htab.size());
    htab.insert(htab.end(), W.begin(), W.end());
    op->tab_E[k] = int64_t(htab.size());
    htab.insert(htab.end(), E.begin(), E.end());
    const int TB = d == 1 ? 64 : (d == 2 ? 8 : 4);
    op->tb[k] = TB;
    op->nt[k] = (M + TB - 1) / TB;
    op->span[k] = (2 * R + TB - 1) / TB;
  }
  op->n_stiles = 1;
  op->nslot = 1;
  for (int k = 0; k < d; ++k) {
    op->n_stiles *= op->nt[k];
    op->nslot *= 2 * op->span[k] + 1;
  }
  op->lr_blocks = (P + 63) / 64;
  const int F = d + 1;
  const size_t bytes_main = carve_bytes(size_t(P) * F * n, 8) + 2 * carve_bytes(size_t(P) * n, 8) +
                            2 * carve_bytes(P, 8) + carve_bytes(htab.size(), 8) +
                            carve_bytes(size_t(op->lr_blocks) * (2 * n + 1) * 64, 8) +
                            carve_bytes(size_t(2 * n + 1) * 64, 8);
  const size_t bytes_band =
      mode == FPCA_COVOP_STORE_BAND ? carve_bytes(size_t(op->n_stiles) * op->nslot * 4096, 8) : 0;
  auto fail = [&](int rc) {
    if (op->Zn) (void)hipFree(op->Zn);
    if (op->band) (void)hipFree(op->band);
    delete op;
    return rc;
  };
  if (int rc = set_device(ctx)) return fail(rc);
  {
    size_t free_b = 0, total_b = 0;
    FPCA_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t temp = carve_bytes(size_t(P) * F * n, 8) + carve_bytes(size_t(P) * n, 8);
    if (bytes_main + bytes_band + temp > free_b)
      return fail(set_error(FPCA_ERR_WORKSPACE, "covariance operator needs %zu bytes, %zu free",
                            bytes_main + bytes_band + temp, free_b));
  }
  void *mem = nullptr;
  if (hipMalloc(&mem, bytes_main) != hipSuccess) return fail(set_error(FPCA_ERR_WORKSPACE, "hipMalloc failed"));
  Carver cv{static_cast<char *>(mem), 0, bytes_main};
  op->Zn = cv.take<double>(size_t(P) * F * n);
  op->Ln = cv.take<double>(size_t(P) * n);
  op->Bn = cv.take<double>(size_t(P) * n);
  op->Y2 = cv.take<double>(P);
  op->mu = cv.take<double>(P);
  op->tab = cv.take<double>(htab.size());
  op->lr_part = cv.take<double>(size_t(op->lr_blocks) * (2 * n + 1) * 64);
  op->lr_tot = cv.take<double>(size_t(2 * n + 1) * 64);
  if (bytes_band && hipMalloc(reinterpret_cast<void **>(&op->band), bytes_band) != hipSuccess)
    return fail(set_error(FPCA_ERR_WORKSPACE, "hipMalloc of the band failed"));
  hipStream_t s = ctx->stream;
  if (hipMemcpyAsync(op->tab, htab.data(), htab.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(op->mu, mu, size_t(P) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return fail(set_error(FPCA_ERR_DEVICE, "copy failed"));
  // temporaries: the transposed curves and a second family buffer
  double *Yn = nullptr, *tmp = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&Yn), size_t(P) * n * 8) != hipSuccess)
    return fail(set_error(FPCA_ERR_WORKSPACE, "hipMalloc failed"));
  if (hipMalloc(reinterpret_cast<void **>(&tmp), size_t(P) * F * n * 8) != hipSuccess) {
    (void)hipFree(Yn);
    return fail(set_error(FPCA_ERR_WORKSPACE, "hipMalloc failed"));
  }
  const CovGeo g = make_geo(op);
  int rc = FPCA_OK;
  do {
    hipLaunchKernelGGL(k_transpose, dim3(unsigned((P + 31) / 32), unsigned((n + 31) / 32)), dim3(32, 8), 0, s, n, P,
                       Y, Yn);
    if (hipGetLastError() != hipSuccess) {
      rc = set_error(FPCA_ERR_DEVICE, "transpose launch failed");
      break;
    }
    hipLaunchKernelGGL(k_sq, dim3(nb256(P)), dim3(256), 0, s, P, int(n), Yn, op->Y2);
    // separable passes, last coordinate first; the last pass lands in Zn
    const double *in = Yn;
    int Fin = 1;
    for (int pass = 0; pass < d && rc == FPCA_OK; ++pass) {
      const int k = d - 1 - pass;
      double *dst = ((d - 1 - pass) % 2 == 0) ? op->Zn : tmp;
      FilterMap fm{};
      fm.nmap = 0;
      fm.fo[fm.nmap] = 0, fm.fi[fm.nmap] = 0, fm.e[fm.nmap] = 0, ++fm.nmap;
      fm.fo[fm.nmap] = k + 1, fm.fi[fm.nmap] = 0, fm.e[fm.nmap] = 1, ++fm.nmap;
      for (int j = k + 1; j < d; ++j) fm.fo[fm.nmap] = j + 1, fm.fi[fm.nmap] = j + 1, fm.e[fm.nmap] = 0, ++fm.nmap;
      hipLaunchKernelGGL(k_filter, dim3(nb256(P * n), unsigned(fm.nmap)), dim3(256), 0, s, g, k, in, Fin, dst, F, fm);
      if (hipGetLastError() != hipSuccess) rc = set_error(FPCA_ERR_DEVICE, "filter launch failed");
      in = dst;
      Fin = F;
    }
    if (rc != FPCA_OK) break;
    hipLaunchKernelGGL(k_lr_prep, dim3(nb256(P * n)), dim3(256), 0, s, g, op->Zn, op->Ln, op->Bn);
    if (hipGetLastError() != hipSuccess) {
      rc = set_error(FPCA_ERR_DEVICE, "prep launch failed");
      break;
    }
    if (mode == FPCA_COVOP_STORE_BAND) rc = band_dispatch(op, true, nullptr, 0, nullptr);
  } while (false);
  // the temporaries are freed once the stream has used them
  const hipError_t e1 = hipStreamSynchronize(s);
  (void)hipFree(Yn);
  (void)hipFree(tmp);
  if (rc != FPCA_OK) return fail(rc);
  if (e1 != hipSuccess) return fail(hip_fail(e1, "covariance operator set-up"));
  *op_out = op;
  return FPCA_OK;
}

extern "C" int fpca_covop_apply(fpca_covop op, int r, const double *X, double *out) {
  if (!op) return set_error(FPCA_ERR_INVALID_ARG, "null operator");
  if (int rc = check_handle(op->ctx)) return rc;
  if (r < 1 || r > 64) return set_error(FPCA_ERR_INVALID_ARG, "need 1 <= r <= 64");
  if (!X || !out) return set_error(FPCA_ERR_INVALID_ARG, "X and out are required");
  if (int rc = set_device(op->ctx)) return rc;
  return covop_apply_internal(op, r, X, out);
}

extern "C" int fpca_covop_destroy(fpca_covop op) {
  if (!op) return FPCA_OK;
  if (op->ctx) (void)hipSetDevice(op->ctx->device);
  if (op->ctx && op->ctx->stream) (void)hipStreamSynchronize(op->ctx->stream);
  if (op->Zn) (void)hipFree(op->Zn);
  if (op->band) (void)hipFree(op->band);
  delete op;
  return FPCA_OK;
}

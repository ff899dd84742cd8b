// Random-projection eigendecomposition of the matrixized covariance
// (Sections 3.1 and 3.4): A = W^1/2 Gamma W^1/2 is never formed; every product
// A X is computed as W^1/2 (Gamma (W^1/2 X)).
//
//   test matrix  : counter-based normals (splitmix64 + Box-Muller), P x r
//   products     : Gamma X on MFMA (FP32) with split K, FP64 reduction
//   orthonormal  : CholeskyQR in FP64 between products, CholeskyQR2 before
//                  the Rayleigh-Ritz step (columns that become numerically
//                  dependent are dropped: their basis vector is set to 0);
//                  row kernels on 16-row chunks, a fixed-order sum of the
//                  partial Gram matrices, a one-workgroup factorization
//   Rayleigh-Ritz: B = Q^T A Q in FP64, eigenpairs by a one-workgroup
//                  parallel-ordered cyclic Jacobi method in FP64
//   finalize     : psi = Q U, phi = psi / sqrt(w), sign rule, FVE.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "covop.hpp"

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

// Quadrature weights, their square roots and the scaled test matrix in one
// pass, thread per (p, j): w_p = quad_w[p] if given, else the Riemann weight
// wv (0 outside the mask); X[p][j] = sqrt(w_p) * normal number j*P + p of the
// seed's stream for j < r, 0 for the padding columns.
template <typename T>
__global__ void k_setup(uint64_t seed, int64_t P, int r, int rp, const double *__restrict__ quad_w, double wv,
                        const uint8_t *__restrict__ mask, double *__restrict__ w, double *__restrict__ sw, T *X) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P * rp) return;
  const int64_t p = e / rp;
  const int j = int(e % rp);
  const double wp = quad_w ? quad_w[p] : ((mask && !mask[p]) ? 0.0 : wv);
  const double s = sqrt(wp);
  if (j == 0) {
    w[p] = wp;
    sw[p] = s;
  }
  X[e] = T(j < r ? s * normal_at(seed, uint64_t(j) * uint64_t(P) + uint64_t(p)) : 0.0);
}

// Partial products of Y^T = X^T Gamma over one K chunk (Gamma symmetric):
// workgroup = (64 nodes, K chunk); 4 wavefronts x 16 nodes; MFMA 16x16x4 FP32
// with the basis as the A operand and Gamma rows as the B operand. Tiles of 32
// Gamma rows are prefetched into registers while the previous tile is used.
template <int RB, bool VEC>
__global__ __launch_bounds__(256) void k_panel_f32(int64_t P, const float *__restrict__ G,
                                                    const float *__restrict__ X, int64_t kchunk,
                                                    float *__restrict__ part) {
  constexpr int RP = RB * 16;
  constexpr int KT = 32;
  __shared__ float As[2][KT][64 + 4];
  __shared__ float Xs[2][KT][RP + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = int64_t(blockIdx.x) * 64;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk;
  const int64_t k1 = min(P, k0 + kchunk);
  float4_t acc[2][RB];  // two sets alternate over K steps: independent MFMA chains
#pragma unroll
  for (int b = 0; b < RB; ++b) acc[0][b] = acc[1][b] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int ar = tid >> 4, ac = (tid & 15) * 4;  // rows ar and ar+16, columns ac..ac+3
  float ra[2][4], rx[2][4];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t q = kb + ar + 16 * h;
      if (VEC && q < k1 && c0 + ac + 3 < P) {
        const float4 v = *reinterpret_cast<const float4 *>(G + q * P + c0 + ac);
        ra[h][0] = v.x; ra[h][1] = v.y; ra[h][2] = v.z; ra[h][3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[h][e] = (q < k1 && c0 + ac + e < P) ? G[q * P + c0 + ac + e] : 0.f;
      }
      // basis rows kb..kb+31 are contiguous: KT*RP floats
      const int o = (tid + 256 * h) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = (o + e) / RP, cc = (o + e) % RP;
        const int64_t qq = kb + rr;
        rx[h][e] = (o + e < KT * RP && qq < k1) ? X[qq * RP + cc] : 0.f;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int e = 0; e < 4; ++e) As[buf][ar + 16 * h][ac + e] = ra[h][e];
      const int o = (tid + 256 * h) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (o + e < KT * RP) Xs[buf][(o + e) / RP][(o + e) % RP] = rx[h][e];
    }
  };
  int buf = 0;
  if (k0 < k1) {
    load(k0);
    store(0);
  }
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += KT) {
    const bool more = kb + KT < k1;
    if (more) load(kb + KT);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int krow = kk + (lane >> 4);
      const float b = As[buf][krow][wave * 16 + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < RB; ++mb) {
        const float a = Xs[buf][krow][mb * 16 + (lane & 15)];
        acc[(kk >> 2) & 1][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[(kk >> 2) & 1][mb], 0, 0, 0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // D[j][p]: row j = mb*16 + 4*(lane/16) + v, column p = c0 + wave*16 + lane%16.
  const int64_t p = c0 + wave * 16 + (lane & 15);
  if (p < P) {
    float *dst = part + (int64_t(blockIdx.y) * P + p) * RP;
#pragma unroll
    for (int mb = 0; mb < RB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[mb * 16 + 4 * (lane >> 4) + v] = acc[0][mb][v] + acc[1][mb][v];
  }
}

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// The same partial products as k_panel_f32 on BF16x3 MFMA: each FP32 value x
// is split as hi = bf16(x), lo = bf16(x - hi) while it is staged in LDS, and
// a 16x16 block takes lo*hi + hi*lo + hi*hi on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation (the lo*lo term, below 2^-16 of the product, is dropped).
// Gamma is symmetric, so the 64 output nodes p of a workgroup read their own
// rows: thread (p, g) takes 8 consecutive nodes q of row p per 32 (one
// 32-byte run), and the 16 rows of a wavefront's B operand come from LDS as
// one 16-byte read per lane. Tiles of 64 nodes (two MFMA k-steps) in two LDS
// buffers, loaded into registers two tiles ahead of their products. Rows
// past P are read from row P - 1 and feed only outputs past P, which are not
// written.
template <int RB, bool VEC>
__global__ __launch_bounds__(256) void k_panel_bf16x3(int64_t P, const float *__restrict__ G,
                                                       const float *__restrict__ X, int64_t kchunk,
                                                       float *__restrict__ part) {
  constexpr int RP = RB * 16;
  constexpr int KT = 64;
  constexpr int LK = KT + 8;  // padded LDS row (144 bytes): the 16 rows of an operand read on distinct banks
  constexpr int NX = (KT * RP / 4 + 255) / 256;  // float4s of the basis tile per thread
  __shared__ __attribute__((aligned(16))) unsigned short Gs[2][2][64][LK];  // [buffer][hi, lo][p][q]
  __shared__ __attribute__((aligned(16))) unsigned short Xs[2][2][RP][LK];  // [buffer][hi, lo][j][q]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = int64_t(blockIdx.x) * 64;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk;
  const int64_t k1 = min(P, k0 + kchunk);
  float4_t acc[2][RB];  // one set per k-step of a tile: independent MFMA chains
#pragma unroll
  for (int b = 0; b < RB; ++b) acc[0][b] = acc[1][b] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int gp = tid >> 2, gg = tid & 3;
  const float *grow = G + min(c0 + gp, P - 1) * P;
  // a tile's raw values in registers: g = this thread's two 8-node runs of
  // its Gamma row, x = its float4s of the basis
  static_assert(KT * RP / 4 == NX * 256, "every thread loads NX float4s of the basis tile");
  // whole tiles (the same test in every lane): plain vector loads, so no lane
  // writes the registers of a load still in flight; the ragged last tile of a
  // chunk: scalar loads with the nodes past k1 read as 0
  auto load = [&](int64_t kb, float (&g)[2][8], float (&x)[NX][4]) {
    if (VEC && kb + KT <= k1) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t q = kb + 32 * h + 8 * gg;
        const float4 a = *reinterpret_cast<const float4 *>(grow + q);
        const float4 b = *reinterpret_cast<const float4 *>(grow + q + 4);
        g[h][0] = a.x, g[h][1] = a.y, g[h][2] = a.z, g[h][3] = a.w;
        g[h][4] = b.x, g[h][5] = b.y, g[h][6] = b.z, g[h][7] = b.w;
      }
#pragma unroll
      for (int u = 0; u < NX; ++u) {
        const int o = tid + 256 * u;
        const float4 v = *reinterpret_cast<const float4 *>(X + (kb + o / (RP / 4)) * RP + (o % (RP / 4)) * 4);
        x[u][0] = v.x, x[u][1] = v.y, x[u][2] = v.z, x[u][3] = v.w;
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t q = kb + 32 * h + 8 * gg;
#pragma unroll
        for (int e = 0; e < 8; ++e) g[h][e] = q + e < k1 ? grow[q + e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < NX; ++u) {
        const int o = tid + 256 * u;
        const int64_t qq = kb + o / (RP / 4);
        const int j4 = (o % (RP / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[u][e] = qq < k1 ? X[qq * RP + j4 + e] : 0.f;
      }
    }
  };
  auto store = [&](int buf, const float (&g)[2][8], const float (&x)[NX][4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u16x8 hv, lv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const unsigned short hb = bf16_rne(g[h][e]);
        hv[e] = hb;
        lv[e] = bf16_rne(g[h][e] - bf16_to_f32(hb));
      }
      *reinterpret_cast<u16x8 *>(&Gs[buf][0][gp][32 * h + 8 * gg]) = hv;
      *reinterpret_cast<u16x8 *>(&Gs[buf][1][gp][32 * h + 8 * gg]) = lv;
    }
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int o = tid + 256 * u;
      const int ql = o / (RP / 4), j4 = (o % (RP / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const unsigned short hb = bf16_rne(x[u][e]);
        Xs[buf][0][j4 + e][ql] = hb;
        Xs[buf][1][j4 + e][ql] = bf16_rne(x[u][e] - bf16_to_f32(hb));
      }
    }
  };
  auto rd = [](const unsigned short *p) { return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p)); };
  // lane l: node offset 8 (l / 16) of the k-step; B: node p = 16 wave + l % 16, A: basis column j = 16 mb + l % 16
  auto mma = [&](int buf) {
    bf16x8 bh[2], bl[2], ah[2][RB], al[2][RB];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int kq = 32 * s + 8 * (lane >> 4);
      bh[s] = rd(&Gs[buf][0][wave * 16 + (lane & 15)][kq]);
      bl[s] = rd(&Gs[buf][1][wave * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int mb = 0; mb < RB; ++mb) {
        ah[s][mb] = rd(&Xs[buf][0][mb * 16 + (lane & 15)][kq]);
        al[s][mb] = rd(&Xs[buf][1][mb * 16 + (lane & 15)][kq]);
      }
    }
    // the three products of a block are 2 RB MFMAs apart
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int mb = 0; mb < RB; ++mb)
        acc[s][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s][mb], bh[s], acc[s][mb], 0, 0, 0);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int mb = 0; mb < RB; ++mb)
        acc[s][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s][mb], bl[s], acc[s][mb], 0, 0, 0);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int mb = 0; mb < RB; ++mb)
        acc[s][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s][mb], bh[s], acc[s][mb], 0, 0, 0);
  };
  // Two register sets, two tiles ahead: while tile kb is multiplied from LDS
  // buffer 0, tile kb + KT waits in set B and tile kb + 2 KT is loading into
  // set A (then the same with the buffers and sets exchanged), so each
  // workgroup keeps two tiles of Gamma in flight.
  float ga[2][8], xa[NX][4], gb[2][8], xb[NX][4];
  if (k0 < k1) {
    load(k0, ga, xa);
    if (k0 + KT < k1) load(k0 + KT, gb, xb);
    store(0, ga, xa);
  }
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += 2 * KT) {
    if (kb + 2 * KT < k1) load(kb + 2 * KT, ga, xa);
    mma(0);
    if (kb + KT >= k1) break;
    store(1, gb, xb);
    __syncthreads();  // buffer 1 written; every wavefront is past buffer 0's products
    if (kb + 3 * KT < k1) load(kb + 3 * KT, gb, xb);
    mma(1);
    if (kb + 2 * KT < k1) store(0, ga, xa);
    __syncthreads();  // buffer 0 written; every wavefront is past buffer 1's products
  }
  // D[j][p]: row j = mb*16 + 4*(lane/16) + v, column p = c0 + wave*16 + lane%16.
  const int64_t p = c0 + wave * 16 + (lane & 15);
  if (p < P) {
    float *dst = part + (int64_t(blockIdx.y) * P + p) * RP;
#pragma unroll
    for (int mb = 0; mb < RB; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[mb * 16 + 4 * (lane >> 4) + v] = acc[0][mb][v] + acc[1][mb][v];
  }
}

// FP64 product for FP64 storage (small grids): thread per (p, j); the Gamma
// row stays in cache across the rp threads that share p.
__global__ void k_panel_f64(int64_t P, int rp, const double *__restrict__ G, const double *__restrict__ X,
                            double *__restrict__ Yraw) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= P * rp) return;
  const int64_t p = e / rp;
  const int j = int(e % rp);
  double s = 0.0;
  for (int64_t q = 0; q < P; ++q) s += G[p * P + q] * X[q * rp + j];
  Yraw[e] = s;
}

constexpr int ROWS = 16;  // rows per workgroup of the row kernels
constexpr int RT = 256;   // threads of the row kernels
constexpr int SG = 16;    // threads per entry in the partial-Gram sum

// out = A^T B over the ROWS rows of a workgroup (A, B: [ROWS][RP + 1] in LDS).
template <int RP>
__device__ inline void rows_gram(const double *A, const double *B, double *__restrict__ out, int tid) {
  constexpr int LD = RP + 1;
  for (int e = tid; e < RP * RP; e += RT) {
    const int a = e / RP, b = e % RP;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int rr = 0; rr < ROWS; rr += 2) {
      s0 = fma(A[rr * LD + a], B[rr * LD + b], s0);
      s1 = fma(A[(rr + 1) * LD + a], B[(rr + 1) * LD + b], s1);
    }
    out[e] = s0 + s1;
  }
}

// Finishes a product, ROWS rows per workgroup: Y[p, j] = sqrt(w_p) * (sum of
// the K-split partials in split order, or Yraw for FP64 storage), then the
// rows' partial Gram matrix:
//   MODE 1: part = Y_c^T Y_c;  MODE 2: part = Q_c^T Y_c  (Rayleigh-Ritz).
// A thread loads sixteen splits of all its entries at once.
template <int MODE, int RP>
__global__ __launch_bounds__(RT) void k_rows_gram(int64_t P, int nsplit, const float *__restrict__ part32,
                                                   const double *__restrict__ Yraw, const double *__restrict__ sw,
                                                   const double *__restrict__ Q, double *__restrict__ Y,
                                                   double *__restrict__ gpart) {
  constexpr int LD = RP + 1;
  constexpr int NE = ROWS * RP / RT;
  static_assert(NE * RT == ROWS * RP, "whole entries per thread");
  __shared__ double Ys[ROWS * LD];
  __shared__ double Qs[MODE == 2 ? ROWS * LD : 1];
  const int tid = threadIdx.x;
  const int64_t p0 = int64_t(blockIdx.x) * ROWS;
  const int64_t base = p0 * RP, lim = P * RP;
  double acc[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) acc[u] = 0.0;
  if (part32) {
    for (int c = 0; c < nsplit; c += 16) {
      float v[16][NE];
#pragma unroll
      for (int s = 0; s < 16; ++s)
#pragma unroll
        for (int u = 0; u < NE; ++u) {
          const int64_t o = base + tid + RT * u;
          v[s][u] = (c + s < nsplit && o < lim) ? part32[int64_t(c + s) * lim + o] : 0.f;
        }
#pragma unroll
      for (int s = 0; s < 16; ++s)
#pragma unroll
        for (int u = 0; u < NE; ++u) acc[u] += double(v[s][u]);
    }
  } else {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int64_t o = base + tid + RT * u;
      acc[u] = o < lim ? Yraw[o] : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + RT * u;
    const int rr = e / RP, j = e % RP;
    const int64_t p = p0 + rr;
    double v = 0.0, qv = 0.0;
    if (p < P) {
      v = acc[u] * sw[p];
      Y[p * RP + j] = v;
      if (MODE == 2) qv = Q[p * RP + j];
    }
    Ys[rr * LD + j] = v;
    if (MODE == 2) Qs[rr * LD + j] = qv;
  }
  __syncthreads();
  rows_gram<RP>(MODE == 2 ? Qs : Ys, Ys, gpart + int64_t(blockIdx.x) * RP * RP, tid);
}

// G = sum of the nparts partial RP x RP matrices in a fixed order: thread g
// of an entry adds partials g, g + SG, g + 2 SG, ... (sixteen loads in
// flight), then the SG sums are combined pairwise.
template <int RP>
__global__ __launch_bounds__(256) void k_sum_gram(int nparts, const double *__restrict__ part,
                                                  double *__restrict__ G) {
  constexpr int EPB = 256 / SG;  // entries per workgroup
  __shared__ double red[SG][EPB];
  const int tid = threadIdx.x;
  const int el = tid % EPB, g = tid / EPB;
  const int e = blockIdx.x * EPB + el;
  double s = 0.0;
  if (e < RP * RP) {
    for (int c = g; c < nparts; c += SG * 16) {
      double v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int pc = c + SG * k;
        v[k] = pc < nparts ? part[int64_t(pc) * RP * RP + e] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) s += v[k];
    }
  }
  red[g][el] = s;
  __syncthreads();
#pragma unroll
  for (int w = SG / 2; w > 0; w >>= 1) {
    if (g < w) red[g][el] += red[g + w][el];
    __syncthreads();
  }
  if (g == 0 && e < RP * RP) G[e] = red[0][el];
}

constexpr int CT = 1024;  // threads of the factorization kernel

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}

// 1/x for finite x != 0: the hardware estimate refined by two Newton steps.
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  return y * fma(-x, y, 2.0);
}

// G = L L^T and L^{-1} in one workgroup by elimination on [G | I]: step j
// (pivot p_j = the current M[j][j]) subtracts (M[r][j] / p_j) times row j from
// every row r > j, over columns j+1.. of the G part and 0..j of the I part.
// Afterwards row r holds p_r on its diagonal and the unit lower triangular
// inverse in its I part, so L^{-1}[r][c] = M[r][RP + c] / sqrt(p_r). A step
// whose pivot is <= 1e-12 of the original diagonal entry (or that entry is
// <= 0) eliminates nothing: its column is dropped. Steps j and j + 1 share one
// barrier: each thread forms row j + 1 after step j, its pivot and its
// multipliers from the values before step j (every thread the same bits);
// row j + 1's final pivot and I part go to Dodd / Lodd, since other threads
// still read its old values. Rinv[c][r] = L^{-1}[r][c] (R = L^T) with the
// columns of dropped vectors zeroed; act[j] = 1 for kept columns.
template <int RP>
__global__ __launch_bounds__(CT) void k_chol(const double *__restrict__ G, double *__restrict__ Rinv,
                                             int *__restrict__ act) {
  static_assert(RP % 2 == 0, "steps go in pairs");
  constexpr int LD = 2 * RP + 1;
  __shared__ double M[RP * LD];
  __shared__ double Lodd[RP / 2][RP];  // I part of rows 1, 3, 5, ...
  __shared__ double Dodd[RP / 2];      // pivots of rows 1, 3, 5, ...
  __shared__ double diag[RP];
  __shared__ int keep[RP];
  const int tid = threadIdx.x;
  for (int e = tid; e < RP * RP; e += CT) {
    const int r = e / RP, c = e % RP;
    M[r * LD + c] = G[e];
    M[r * LD + RP + c] = (r == c) ? 1.0 : 0.0;
  }
  for (int e = tid; e < (RP / 2) * RP; e += CT) Lodd[e / RP][e % RP] = 0.0;  // upper triangle stays 0
  if (tid < RP) diag[tid] = G[tid * RP + tid];
  __syncthreads();
  for (int j = 0; j < RP; j += 2) {
    const int j1 = j + 1;
    const double pj = M[j * LD + j];
    const bool okj = diag[j] > 0.0 && pj > 1e-12 * diag[j];
    const double rpj = okj ? rcp_nr(pj) : 0.0;
    const double mj1 = M[j1 * LD + j] * rpj;  // row j + 1's multiplier at step j
    const double p1 = fma(-mj1, M[j * LD + j1], M[j1 * LD + j1]);
    const bool ok1 = diag[j1] > 0.0 && p1 > 1e-12 * diag[j1];
    const double rp1 = ok1 ? rcp_nr(p1) : 0.0;
    // row rr = 0 is j + 1 (step j only), rows rr > 0 are j + 1 + rr (both
    // steps); columns: G part j+1 .. RP-1 (nb of them), then I part 0 .. j+1
    const int nb = RP - 1 - j;
    for (int e = tid; e < (RP - 1 - j) * (RP + 1); e += CT) {
      const int rr = e / (RP + 1), cc = e % (RP + 1);
      const int r = j1 + rr;
      const int col = cc < nb ? j1 + cc : RP + cc - nb;
      const double mrj = M[r * LD + j] * rpj;
      const double vj = M[j * LD + col];
      const double v = fma(-mrj, vj, M[r * LD + col]);  // after step j
      if (rr == 0) {
        if (col == j1) Dodd[j1 / 2] = v;
        if (col >= RP) Lodd[j1 / 2][col - RP] = v;
      } else if (col != j1) {  // column j + 1 below the diagonal is not read again
        const double v1 = fma(-mj1, vj, M[j1 * LD + col]);                     // row j + 1 after step j
        const double m1 = fma(-mrj, M[j * LD + j1], M[r * LD + j1]) * rp1;  // multiplier at step j + 1
        M[r * LD + col] = fma(-m1, v1, v);
      }
    }
    if (tid == 0) {
      keep[j] = okj ? 1 : 0;
      keep[j1] = ok1 ? 1 : 0;
    }
    __syncthreads();
  }
  for (int e = tid; e < RP * RP; e += CT) {
    const int c = e / RP, r = e % RP;
    const double pr = (r & 1) ? Dodd[r / 2] : M[r * LD + r];
    const double lv = (r & 1) ? Lodd[r / 2][c] : M[r * LD + RP + c];
    Rinv[e] = keep[r] ? lv * rsqrt_nr(pr) : 0.0;
  }
  if (tid < RP) act[tid] = keep[tid];
}

// Q = Y Rinv in FP64 for ROWS rows per workgroup. With GRAM the rows' partial
// Gram of Q is written (first pass of CholeskyQR2); otherwise the next basis
// X = W^1/2 Q in storage type T.
template <typename T, bool GRAM, int RP>
__global__ __launch_bounds__(RT) void k_rows_apply(int64_t P, const double *__restrict__ Y,
                                                    const double *__restrict__ Rinv, const double *__restrict__ sw,
                                                    double *__restrict__ Q, T *__restrict__ X,
                                                    double *__restrict__ gpart) {
  constexpr int LD = RP + 1;
  constexpr int NE = ROWS * RP / RT;
  __shared__ double Ys[ROWS * LD];
  __shared__ double Ri[RP * LD];
  const int tid = threadIdx.x;
  const int64_t p0 = int64_t(blockIdx.x) * ROWS;
  const int64_t base = p0 * RP, lim = P * RP;
  for (int e = tid; e < RP * RP; e += RT) Ri[(e / RP) * LD + e % RP] = Rinv[e];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + RT * u;
    Ys[(e / RP) * LD + e % RP] = base + e < lim ? Y[base + e] : 0.0;
  }
  __syncthreads();
  double qv[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) qv[u] = 0.0;
#pragma unroll 8
  for (int i = 0; i < RP; ++i) {
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + RT * u;
      qv[u] = fma(Ys[(e / RP) * LD + i], Ri[i * LD + e % RP], qv[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + RT * u;
    const int64_t p = p0 + e / RP;
    if (p < P) {
      Q[base + e] = qv[u];
      if (!GRAM) X[base + e] = T(sw[p] * qv[u]);
    }
  }
  if (!GRAM) return;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + RT * u;
    Ys[(e / RP) * LD + e % RP] = (p0 + e / RP < P) ? qv[u] : 0.0;
  }
  __syncthreads();
  rows_gram<RP>(Ys, Ys, gpart + int64_t(blockIdx.x) * RP * RP, tid);
}

// Jacobi rotation of the pair (p, q) from b_pp, b_qq, b_pq, without branches:
// tau = (b_qq - b_pp) / (2 b_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2))
// (t = 1 / (2 tau) for |tau| > 1e18), c = 1 / sqrt(1 + t^2), s = t c. The
// angle only needs to be close (a rotation then leaves b_pq times the angle's
// relative error, which the next sweep removes), so t is formed in FP32 from
// the FP64 difference b_qq - b_pp; c and s are FP64 functions of that t, so
// c^2 + s^2 = 1 to FP64 rounding. The entries are scaled to magnitudes below
// 1 by the caller; b_pq below FP32 range gives the identity.
__device__ inline void jacobi_rot_bf(double app, double aqq, double apq, double *c, double *s) {
  const float a = float(apq), d = float(aqq - app);
  const bool nz = a != 0.0f;
  const float tau = d * (0.5f * __builtin_amdgcn_rcpf(nz ? a : 1.0f));
  const float at = fminf(fabsf(tau), 1e18f);
  const float den = at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.0f));  // |tau| + sqrt(1 + tau^2)
  float t = fabsf(tau) > 1e18f ? 0.5f * __builtin_amdgcn_rcpf(fabsf(tau)) : __builtin_amdgcn_rcpf(den);
  t = tau >= 0.0f ? t : -t;
  const double td = double(t);
  const double w = fma(td, td, 1.0);
  const double h = 0.5 * w;
  double y = __builtin_amdgcn_rsq(w);  // two Newton steps for 1 / sqrt(w)
  y = fma(y, fma(-h * y, y, 0.5), y);
  y = fma(y, fma(-h * y, y, 0.5), y);
  *c = nz ? y : 1.0;
  *s = nz ? td * y : 0.0;
}

// Round-robin pairing of ne (even) indices at a step: pair 0 = (ne-1, step),
// pair m > 0 = ((step + m) mod (ne-1), (step - m) mod (ne-1)).
__device__ inline void rr_pair(int ne, int step, int m, int *a, int *b) {
  if (m == 0) {
    *a = ne - 1;
    *b = step;
  } else {
    *a = (step + m) % (ne - 1);
    *b = (step - m + ne - 1) % (ne - 1);
  }
}

// One workgroup: B = Q^T A Q on the active columns (symmetrized, placed first,
// zero rows and columns for the rest), cyclic Jacobi with round-robin ordering
// of the n active indices (rounded up to even; the inactive ones form fixed
// pairs of zero rows and rotate by the identity). Thread (m1, m2) of the
// (RP/2)^2 threads owns
// the 2x2 block (pair m1) x (pair m2) of B and the entries of V in rows m1 and
// m1 + RP/2, pair m2: it computes rotation m2 from the current B and takes
// rotation m1 from the lane of its wave that computed it (or computes it too
// when RP/2 does not divide 64; every copy of a rotation has the same bits),
// writes B' = J1^T X J2 into the other buffer and V' = V J in place, so a step
// takes one barrier. Eigenvalues sorted descending (stable); outputs the top k,
// their eigenvectors in the RP basis, and FVE.
template <int RP>
__global__ __launch_bounds__((RP / 2) * (RP / 2)) void k_jacobi(const double *__restrict__ G,
                                                                 const int *__restrict__ act, int k,
                                                                 double *__restrict__ evals,
                                                                 double *__restrict__ fve, double *__restrict__ Uk) {
  constexpr int H = RP / 2;
  constexpr int NT = H * H;
  constexpr int NW = (NT + 63) / 64;
  constexpr int LD = RP + 1;
  __shared__ double Bb[2][RP * LD];
  __shared__ double Vb[RP * LD];
  __shared__ int idx[RP];
  __shared__ int n_s;
  __shared__ double red_off[2][NW], red_tot[2][NW];
  const int tid = threadIdx.x;
  if (tid == 0) {
    int n = 0;
    for (int j = 0; j < RP; ++j)
      if (act[j]) idx[n++] = j;
    n_s = n;
  }
  __syncthreads();
  const int n = n_s;
  double mx = 0.0;
  for (int e = tid; e < RP * RP; e += NT) {
    const int a = e / RP, b = e % RP;
    const double v = (a < n && b < n) ? 0.5 * (G[idx[a] * RP + idx[b]] + G[idx[b] * RP + idx[a]]) : 0.0;
    Bb[0][a * LD + b] = v;
    Vb[a * LD + b] = (a == b) ? 1.0 : 0.0;
    mx = fmax(mx, fabs(v));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((tid & 63) == 0) red_off[1][tid >> 6] = mx;
  __syncthreads();
  // exact power-of-two scaling to max |B| in [0.5, 1); undone on the eigenvalues
  mx = 0.0;
  for (int wv = 0; wv < NW; ++wv) mx = fmax(mx, red_off[1][wv]);
  int ex = 0;
  if (mx > 0.0) frexp(mx, &ex);
  for (int e = tid; e < RP * RP; e += NT) Bb[0][(e / RP) * LD + e % RP] = ldexp(Bb[0][(e / RP) * LD + e % RP], -ex);
  __syncthreads();
  const int m1 = tid / H, m2 = tid % H;
  // Round robin over the ne = n + (n & 1) leading indices (pairs m < ne/2):
  // step 0 pairs, then every step moves each index of a pair on by one
  // (mod ne - 1), except index ne - 1 of pair 0. Pairs m >= ne/2 are the
  // fixed inactive pairs (2m, 2m + 1) and rotate by the identity.
  const int ne = n + (n & 1);
  auto first_pair = [&](int m, int *a, int *b) {
    if (m >= ne / 2) {
      *a = 2 * m;
      *b = 2 * m + 1;
    } else {
      rr_pair(ne, 0, m, a, b);
    }
  };
  int a1, b1, a2, b2;
  first_pair(m1, &a1, &b1);
  first_pair(m2, &a2, &b2);
  auto next_pair = [&](int m, int *a, int *b) {
    if (m >= ne / 2) return;
    if (m != 0) *a = *a + 1 == ne - 1 ? 0 : *a + 1;
    *b = *b + 1 == ne - 1 ? 0 : *b + 1;
  };
  int cur = 0;
  for (int sweep = 0; sweep < 60 && n >= 2; ++sweep) {
    // convergence: sum of squares off the diagonal against the total
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < RP * RP; e += NT) {
      const int a = e / RP, b = e % RP;
      const double v = Bb[cur][a * LD + b] * Bb[cur][a * LD + b];
      tot += v;
      if (a != b) off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      tot += __shfl_xor(tot, o);
    }
    if ((tid & 63) == 0) {
      red_off[sweep & 1][tid >> 6] = off;
      red_tot[sweep & 1][tid >> 6] = tot;
    }
    __syncthreads();
    double so = 0.0, st = 0.0;
    for (int wv = 0; wv < NW; ++wv) {
      so += red_off[sweep & 1][wv];
      st += red_tot[sweep & 1][wv];
    }
    if (!(so > 1e-28 * st)) break;  // uniform: every thread summed the same partials
    for (int step = 0; step < ne - 1; ++step) {
      const double *B = Bb[cur];
      double *Bn = Bb[cur ^ 1];
      // every LDS read of the step is issued before the rotation is formed
      const double x00 = B[a1 * LD + a2], x01 = B[a1 * LD + b2];
      const double x10 = B[b1 * LD + a2], x11 = B[b1 * LD + b2];
      double va[2], vb[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        va[h] = Vb[(m1 + h * H) * LD + a2];
        vb[h] = Vb[(m1 + h * H) * LD + b2];
      }
      const double p22 = B[a2 * LD + a2], q22 = B[b2 * LD + b2], o22 = B[a2 * LD + b2];
      asm volatile("" ::"v"(x00), "v"(x01), "v"(x10), "v"(x11), "v"(va[0]), "v"(vb[0]), "v"(va[1]), "v"(vb[1]));
      double c1, s1, c2, s2;
      jacobi_rot_bf(p22, q22, o22, &c2, &s2);
      if constexpr (64 % H == 0) {
        // rotation m1 is rotation m2 of lane (group of H lanes) + m1 of this wave
        const int src = (threadIdx.x & 63 & ~(H - 1)) + m1;
        c1 = __shfl(c2, src);
        s1 = __shfl(s2, src);
      } else {
        jacobi_rot_bf(B[a1 * LD + a1], B[b1 * LD + b1], B[a1 * LD + b1], &c1, &s1);
      }
      const double y00 = c1 * x00 - s1 * x10, y01 = c1 * x01 - s1 * x11;
      const double y10 = s1 * x00 + c1 * x10, y11 = s1 * x01 + c1 * x11;
      Bn[a1 * LD + a2] = c2 * y00 - s2 * y01;
      Bn[a1 * LD + b2] = s2 * y00 + c2 * y01;
      Bn[b1 * LD + a2] = c2 * y10 - s2 * y11;
      Bn[b1 * LD + b2] = s2 * y10 + c2 * y11;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int row = m1 + h * H;
        Vb[row * LD + a2] = c2 * va[h] - s2 * vb[h];
        Vb[row * LD + b2] = s2 * va[h] + c2 * vb[h];
      }
      next_pair(m1, &a1, &b1);
      next_pair(m2, &a2, &b2);
      __syncthreads();
      cur ^= 1;
    }
  }
  const double *Bf = Bb[cur];
  __shared__ int order[RP];
  __shared__ double possum;
  if (tid < n) {
    const double v = Bf[tid * LD + tid];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = Bf[j * LD + j];
      if (u > v || (u == v && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
      if (Bf[j * LD + j] > 0.0) s += Bf[j * LD + j];
    possum = s;
  }
  __syncthreads();
  if (tid == 0) {
    double cum = 0.0;
    for (int l = 0; l < k; ++l) {
      const double v = l < n ? Bf[order[l] * LD + order[l]] : 0.0;
      cum += v;
      evals[l] = ldexp(v, ex);
      fve[l] = possum > 0.0 ? cum / possum : 0.0;
    }
  }
  for (int e = tid; e < RP * k; e += NT) Uk[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < n * k; e += NT) {
    const int a = e / k, l = e % k;
    if (l < n) Uk[int64_t(idx[a]) * k + l] = Vb[a * LD + order[l]];
  }
}

// phi[l][p] = (Q U)[p][l] / sqrt(w_p) (0 where w_p = 0), with per-workgroup
// partial sums of w phi, w |phi| and max |phi| for the sign rule.
template <int RP>
__global__ __launch_bounds__(256) void k_phi(int64_t P, int k, const double *__restrict__ Q,
                                              const double *__restrict__ Uk, const double *__restrict__ w,
                                              double *__restrict__ phi, double *__restrict__ red) {
  __shared__ double r1[4], r2[4], r3[4];
  const int l = blockIdx.y, tid = threadIdx.x;
  const int64_t p = int64_t(blockIdx.x) * 256 + tid;
  double f = 0.0, wp = 0.0;
  if (p < P) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < RP; ++i) v += Q[p * RP + i] * Uk[int64_t(i) * k + l];  // the row's loads all in flight
    wp = w[p];
    f = wp > 0.0 ? v / sqrt(wp) : 0.0;
    phi[int64_t(l) * P + p] = f;
  }
  double s1 = wp * f, s2 = wp * fabs(f), mx = fabs(f);
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  if ((tid & 63) == 0) {
    r1[tid >> 6] = s1;
    r2[tid >> 6] = s2;
    r3[tid >> 6] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    const int64_t o = (int64_t(l) * gridDim.x + blockIdx.x) * 3;
    red[o] = r1[0] + r1[1] + r1[2] + r1[3];
    red[o + 1] = r2[0] + r2[1] + r2[2] + r2[3];
    red[o + 2] = fmax(fmax(r3[0], r3[1]), fmax(r3[2], r3[3]));
  }
}

// One workgroup per eigenvector: sign rule from the partial sums (the
// lowest-index tie-break scans phi only when sum w phi is negligible), then the
// signed eigenfunction is written in storage type T.
template <typename T>
__global__ __launch_bounds__(256) void k_sign_write(int64_t P, int nblk, const double *__restrict__ phi,
                                                     const double *__restrict__ red, T *__restrict__ efuns) {
  __shared__ double S1, S2, MX;
  __shared__ long long first[256];
  const int l = blockIdx.x, tid = threadIdx.x;
  {
    // the workgroups' partials: thread t adds t, t + 256, ...; then a fixed tree
    __shared__ double ra[256], rb[256], rm[256];
    double a = 0.0, b = 0.0, m = 0.0;
    for (int i = tid; i < nblk; i += 256) {
      const int64_t o = (int64_t(l) * nblk + i) * 3;
      a += red[o];
      b += red[o + 1];
      m = fmax(m, red[o + 2]);
    }
    ra[tid] = a;
    rb[tid] = b;
    rm[tid] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) {
        ra[tid] += ra[tid + st];
        rb[tid] += rb[tid + st];
        rm[tid] = fmax(rm[tid], rm[tid + st]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      S1 = ra[0];
      S2 = rb[0];
      MX = rm[0];
    }
    __syncthreads();
  }
  const double *f = phi + int64_t(l) * P;
  bool neg;
  if (fabs(S1) >= 1e-8 * S2) {
    neg = S1 < 0.0;
  } else {
    long long fi = P;
    for (int64_t p = tid; p < P; p += 256)
      if (fabs(f[p]) >= (1.0 - 1e-6) * MX) {
        fi = p;
        break;
      }
    first[tid] = fi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) first[tid] = min(first[tid], first[tid + s]);
      __syncthreads();
    }
    neg = first[0] < P && f[first[0]] < 0.0;
  }
  const double sg = neg ? -1.0 : 1.0;
#pragma unroll 8
  for (int64_t p = tid; p < P; p += 256) efuns[int64_t(l) * P + p] = T(sg * f[p]);
}

inline unsigned nb(int64_t n) { return unsigned((n + 255) / 256); }

template <typename T, int RP>
int eig_run(fpca_context *ctx, const fpca_grid *grid, int64_t P, const T *gamma, const double *quad_w, int k, int r,
            int power_iters, uint64_t seed, double *evals_h, T *efuns, double *fve_h, fpca_covop_s *op, int prec) {
  const bool f32 = sizeof(T) == 4;
  // K split of the panel product: about two workgroups per compute unit
  // (fewer splits read fewer partials back; at P = 4096, 8 splits measured
  // 29 us per product and Gram against 31 us with 16 and 37 us with 4)
  const int64_t colblocks = (P + 63) / 64;
  int64_t nsplit = (2 * int64_t(ctx->num_cus) + colblocks - 1) / colblocks;
  if (nsplit < 1) nsplit = 1;
  int64_t kchunk = ((P + nsplit - 1) / nsplit + 31) / 32 * 32;
  nsplit = (P + kchunk - 1) / kchunk;
  const int64_t ngram = (P + ROWS - 1) / ROWS;
  const int64_t nphi = (P + 255) / 256;
  size_t need = 2 * carve_bytes(P, 8) + carve_bytes(P * RP, sizeof(T)) + 3 * carve_bytes(P * RP, 8) +
                carve_bytes(ngram * RP * RP, 8) + 2 * carve_bytes(RP * RP, 8) + carve_bytes(RP, 4) +
                carve_bytes(RP * k, 8) +
                carve_bytes(2 * k, 8) + carve_bytes(P * k, 8) + carve_bytes(nphi * k * 3, 8);
  need += f32 ? carve_bytes(nsplit * P * RP, 4) : carve_bytes(P * RP, 8);
  if (int rc = ws_reserve(ctx, need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  double *w = cv.take<double>(P);
  double *sw = cv.take<double>(P);
  T *X = cv.take<T>(P * RP);
  double *Y = cv.take<double>(P * RP);
  double *Q = cv.take<double>(P * RP);
  double *Z = cv.take<double>(P * RP);
  double *gpart = cv.take<double>(ngram * RP * RP);
  double *G = cv.take<double>(RP * RP);
  double *Rinv = cv.take<double>(RP * RP);
  int *act = cv.take<int>(RP);
  double *Uk = cv.take<double>(RP * k);
  double *ev_d = cv.take<double>(2 * k);  // eigenvalues, then FVE: one copy to the host
  double *fve_d = ev_d + k;
  double *phi = cv.take<double>(P * k);
  double *red = cv.take<double>(nphi * k * 3);
  float *part = f32 ? cv.take<float>(nsplit * P * RP) : nullptr;
  double *Yraw = f32 ? nullptr : cv.take<double>(P * RP);

  {
    double wv = 1.0;
    for (int q = 0; q < grid->d; ++q) wv /= double(grid->M[q] - 1);
    hipLaunchKernelGGL(k_setup<T>, dim3(nb(P * RP)), dim3(256), 0, ctx->stream, seed, P, r, RP, quad_w, wv,
                       grid->mask, w, sw, X);
    FPCA_LAUNCH_CHECK("setup");
  }

  // Y (or Z) = W^1/2 Gamma X, then the partial Gram into gA (MODE 1: of itself, MODE 2: Q^T Y)
  auto product = [&](double *out, int mode) -> int {
    if constexpr (sizeof(T) == 4) {
      dim3 grd((unsigned)colblocks, (unsigned)nsplit);
      const bool vec = (P % 4 == 0) && ((reinterpret_cast<uintptr_t>(gamma) & 15) == 0);
      constexpr int RB = RP / 16;
      if (prec == FPCA_PREC_BF16X3) {
        if (vec)
          hipLaunchKernelGGL((k_panel_bf16x3<RB, true>), grd, dim3(256), 0, ctx->stream, P, (const float *)gamma,
                             (const float *)X, kchunk, part);
        else
          hipLaunchKernelGGL((k_panel_bf16x3<RB, false>), grd, dim3(256), 0, ctx->stream, P, (const float *)gamma,
                             (const float *)X, kchunk, part);
        FPCA_LAUNCH_CHECK("panel_bf16x3");
      } else {
        if (vec)
          hipLaunchKernelGGL((k_panel_f32<RB, true>), grd, dim3(256), 0, ctx->stream, P, (const float *)gamma,
                             (const float *)X, kchunk, part);
        else
          hipLaunchKernelGGL((k_panel_f32<RB, false>), grd, dim3(256), 0, ctx->stream, P, (const float *)gamma,
                             (const float *)X, kchunk, part);
        FPCA_LAUNCH_CHECK("panel_f32");
      }
    } else {
      if (op) {
        // the covariance operator: Gamma X without Gamma
        if (int rc = covop_apply_internal(op, RP, (const double *)X, Yraw)) return rc;
      } else {
        hipLaunchKernelGGL(k_panel_f64, dim3(nb(P * RP)), dim3(256), 0, ctx->stream, P, RP, (const double *)gamma,
                           (const double *)X, Yraw);
        FPCA_LAUNCH_CHECK("panel_f64");
      }
    }
    if (mode == 2)
      hipLaunchKernelGGL((k_rows_gram<2, RP>), dim3(unsigned(ngram)), dim3(RT), 0, ctx->stream, P, int(nsplit), part,
                         Yraw, sw, Q, out, gpart);
    else
      hipLaunchKernelGGL((k_rows_gram<1, RP>), dim3(unsigned(ngram)), dim3(RT), 0, ctx->stream, P, int(nsplit), part,
                         Yraw, sw, Q, out, gpart);
    FPCA_LAUNCH_CHECK("rows_gram");
    return FPCA_OK;
  };
  // G = sum of the partial Gram matrices; Cholesky factor and R^-1 of G
  auto factor = [&]() -> int {
    hipLaunchKernelGGL(k_sum_gram<RP>, dim3(unsigned((RP * RP + 256 / SG - 1) / (256 / SG))), dim3(256), 0,
                       ctx->stream, int(ngram), gpart, G);
    FPCA_LAUNCH_CHECK("sum_gram");
    hipLaunchKernelGGL(k_chol<RP>, dim3(1), dim3(CT), 0, ctx->stream, G, Rinv, act);
    FPCA_LAUNCH_CHECK("chol");
    return FPCA_OK;
  };
  // CholeskyQR2 of Y (whose partial Gram is in gpart): Y -> Z -> Q, X.
  // CholeskyQR of Y (one pass; the basis of an intermediate power step only
  // has to span the subspace, its loss of orthogonality is about cond(Y)^2 u
  // and the next product and QR remove it): Y -> Q, X.
  auto cholqr1 = [&]() -> int {
    if (int rc = factor()) return rc;
    hipLaunchKernelGGL((k_rows_apply<T, false, RP>), dim3(unsigned(ngram)), dim3(RT), 0, ctx->stream, P, Y, Rinv,
                       sw, Q, X, (double *)nullptr);
    FPCA_LAUNCH_CHECK("rows_apply");
    return FPCA_OK;
  };
  auto cholqr2 = [&]() -> int {
    if (int rc = factor()) return rc;
    hipLaunchKernelGGL((k_rows_apply<T, true, RP>), dim3(unsigned(ngram)), dim3(RT), 0, ctx->stream, P, Y, Rinv, sw,
                       Z, (T *)nullptr, gpart);
    FPCA_LAUNCH_CHECK("rows_apply");
    if (int rc = factor()) return rc;
    hipLaunchKernelGGL((k_rows_apply<T, false, RP>), dim3(unsigned(ngram)), dim3(RT), 0, ctx->stream, P, Z, Rinv,
                       sw, Q, X, (double *)nullptr);
    FPCA_LAUNCH_CHECK("rows_apply");
    return FPCA_OK;
  };

  // orthonormalizations: single CholeskyQR between products, CholeskyQR2 for
  // the basis of the Rayleigh-Ritz step
  const int nprod = 1 + 2 * power_iters;
  for (int it = 0; it < nprod; ++it) {
    if (int rc = product(Y, 1)) return rc;
    if (int rc = (it + 1 < nprod) ? cholqr1() : cholqr2()) return rc;
  }
  if (int rc = product(Z, 2)) return rc;  // Z = A Q and the partials of Q^T Z
  hipLaunchKernelGGL(k_sum_gram<RP>, dim3(unsigned((RP * RP + 256 / SG - 1) / (256 / SG))), dim3(256), 0, ctx->stream,
                     int(ngram), gpart, G);
  FPCA_LAUNCH_CHECK("sum_gram");
  hipLaunchKernelGGL(k_jacobi<RP>, dim3(1), dim3((RP / 2) * (RP / 2)), 0, ctx->stream, G, act, k, ev_d, fve_d, Uk);
  FPCA_LAUNCH_CHECK("jacobi");
  hipLaunchKernelGGL(k_phi<RP>, dim3(unsigned(nphi), unsigned(k)), dim3(256), 0, ctx->stream, P, k, Q, Uk, w, phi,
                     red);
  FPCA_LAUNCH_CHECK("phi");
  hipLaunchKernelGGL(k_sign_write<T>, dim3(unsigned(k)), dim3(256), 0, ctx->stream, P, int(nphi), phi, red, efuns);
  FPCA_LAUNCH_CHECK("sign_write");
  static_assert(fpca_context::kStageBytes >= 2 * 64 * sizeof(double), "staging holds 2k doubles for k <= 64");
  double *hb = ctx->h_stage;
  FPCA_HIP(hipMemcpyAsync(hb, ev_d, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  for (int l = 0; l < k; ++l) {
    evals_h[l] = hb[l];
    if (fve_h) fve_h[l] = hb[k + l];
  }
  return FPCA_OK;
}

template <typename T>
int eig_impl(fpca_context *ctx, const fpca_grid *grid, int64_t P, const T *gamma, const double *quad_w, int k,
             int oversample, int power_iters, uint64_t seed, double *evals_h, T *efuns, double *fve_h,
             fpca_covop_s *op = nullptr, int prec = FPCA_PREC_F64) {
  const int r = k + oversample;
  switch ((r + 15) / 16) {
    case 1:
      return eig_run<T, 16>(ctx, grid, P, gamma, quad_w, k, r, power_iters, seed, evals_h, efuns, fve_h, op, prec);
    case 2:
      return eig_run<T, 32>(ctx, grid, P, gamma, quad_w, k, r, power_iters, seed, evals_h, efuns, fve_h, op, prec);
    case 3:
      return eig_run<T, 48>(ctx, grid, P, gamma, quad_w, k, r, power_iters, seed, evals_h, efuns, fve_h, op, prec);
    default:
      return eig_run<T, 64>(ctx, grid, P, gamma, quad_w, k, r, power_iters, seed, evals_h, efuns, fve_h, op, prec);
  }
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
  if (dtype == FPCA_F32 && prec != FPCA_PREC_F32 && prec != FPCA_PREC_BF16X3)
    return set_error(FPCA_ERR_UNSUPPORTED, "dtype F32 needs prec F32 or BF16X3");
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype");
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return eig_impl<double>(ctx, grid, P, static_cast<const double *>(gamma), quad_w, k, oversample, power_iters, seed,
                            evals, static_cast<double *>(efuns), fve);
  return eig_impl<float>(ctx, grid, P, static_cast<const float *>(gamma), quad_w, k, oversample, power_iters, seed,
                         evals, static_cast<float *>(efuns), fve, nullptr, prec);
}

extern "C" int fpca_eig_covop(fpca_covop op, const double *quad_w, int k, int oversample, int power_iters,
                              uint64_t seed, double *evals, double *efuns, double *fve) {
  if (!op) return set_error(FPCA_ERR_INVALID_ARG, "null operator");
  fpca_context *ctx = op->ctx;
  if (int rc = check_handle(ctx)) return rc;
  if (!evals || !efuns) return set_error(FPCA_ERR_INVALID_ARG, "evals and efuns are required");
  if (k < 1 || oversample < 0 || power_iters < 0)
    return set_error(FPCA_ERR_INVALID_ARG, "need k >= 1, oversample >= 0, power_iters >= 0");
  if (k + oversample > 64 || k + oversample > op->P)
    return set_error(FPCA_ERR_INVALID_ARG, "k + oversample = %d must be <= min(64, P)", k + oversample);
  if (int rc = set_device(ctx)) return rc;
  fpca_grid g{};
  g.d = op->d;
  for (int q = 0; q < 3; ++q) g.M[q] = q < op->d ? op->M[q] : 1;
  g.mask = nullptr;
  return eig_impl<double>(ctx, &g, op->P, nullptr, quad_w, k, oversample, power_iters, seed, evals, efuns, fve, op);
}

// Symmetric Gram products C = alpha * A^T A for the covariance binning
// (the Gram form of the pair sums of eq. 2.4): A is K x N row-major (one row
// per curve), C is N x N. Only tiles on or above the diagonal are computed;
// each is also written transposed below the diagonal.
#include "common.hpp"

namespace fpca {

namespace {

constexpr int TB = 128;  // output tile edge per workgroup
constexpr int TK = 16;   // K rows staged per LDS step
constexpr int LDP = TB + 16;  // padded LDS row (bank spread for the 4 K-rows of an MFMA operand)

typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int XCDS = 8;  // workgroups are dispatched round-robin over the XCDs
constexpr int BAND = 8;  // tile columns per band of the schedule

// Tile (bi, bj), bi <= bj, of workgroup `id`; false for a padding workgroup.
// Workgroup id runs on XCD id % 8, and each XCD takes a contiguous run of
// `per` tiles in band order (bands of 8 tile columns; within a band, rows top
// to bottom with the band's columns of a row together, then the band's
// diagonal triangle), so the tiles sharing one L2 cover a compact block of
// rows and columns and reuse each other's operand slabs.
__device__ inline bool tile_of(int id, int nb, int per, int *bi, int *bj) {
  int t = (id % XCDS) * per + id / XCDS;
  for (int J0 = 0; J0 < nb; J0 += BAND) {
    const int w = min(BAND, nb - J0);
    const int full = J0 * w;  // rows 0 .. J0-1, w columns each
    const int cnt = full + w * (w + 1) / 2;
    if (t < cnt) {
      if (t < full) {
        *bi = t / w;
        *bj = J0 + t % w;
      } else {
        int r = t - full, ii = 0;
        while (r >= w - ii) {
          r -= w - ii;
          ++ii;
        }
        *bi = J0 + ii;
        *bj = J0 + ii + r;
      }
      return true;
    }
    t -= cnt;
  }
  return false;
}

// bf16 split of an FP32 value: hi = round-to-nearest-even bf16(x), lo = bf16(x - hi).
__device__ inline unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// FP32 operands on v_mfma_f32_16x16x4_f32.
template <bool VEC4>
__global__ __launch_bounds__(256) void k_syrk_f32(const float *__restrict__ A, int64_t K, int64_t N,
                                                   float *__restrict__ C, int64_t ldc, float alpha,
                                                   int zero_diag, int nb, int per) {
  __shared__ float As[TK][LDP];
  __shared__ float Bs[TK][LDP];
  int bi, bj;
  if (!tile_of(blockIdx.x, nb, per, &bi, &bj)) return;  // uniform per workgroup
  const bool diag_tile = (bi == bj);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = int64_t(bi) * TB, n0 = int64_t(bj) * TB;

  float4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

  const int lr = tid >> 4;        // staged K row 0..15
  const int lc = (tid & 15) * 4;  // column group within a 64-wide half

  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    const int64_t kr = k0 + lr;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int c = half * 64 + lc;
      float va[4], vb[4];
      if (VEC4) {
        if (kr < K && m0 + c + 3 < N) {
          float4 v = *reinterpret_cast<const float4 *>(A + kr * N + m0 + c);
          va[0] = v.x; va[1] = v.y; va[2] = v.z; va[3] = v.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) va[e] = (kr < K && m0 + c + e < N) ? A[kr * N + m0 + c + e] : 0.f;
        }
        if (!diag_tile) {
          if (kr < K && n0 + c + 3 < N) {
            float4 v = *reinterpret_cast<const float4 *>(A + kr * N + n0 + c);
            vb[0] = v.x; vb[1] = v.y; vb[2] = v.z; vb[3] = v.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) vb[e] = (kr < K && n0 + c + e < N) ? A[kr * N + n0 + c + e] : 0.f;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          va[e] = (kr < K && m0 + c + e < N) ? A[kr * N + m0 + c + e] : 0.f;
          if (!diag_tile) vb[e] = (kr < K && n0 + c + e < N) ? A[kr * N + n0 + c + e] : 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        As[lr][c + e] = va[e];
        if (!diag_tile) Bs[lr][c + e] = vb[e];
      }
    }
    __syncthreads();
    const float(*Bsrc)[LDP] = diag_tile ? As : Bs;
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      float a[4], b[4];
      const int krow = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[krow][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bsrc[krow][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // D layout of a 16x16 MFMA tile: lane l, element v -> row 4*(l/16)+v, column l%16.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int64_t c = n0 + wn * 64 + j * 16 + (lane & 15);
        if (r < N && c < N) {
          float val = alpha * acc[i][j][v];
          if (zero_diag && r == c) val = 0.f;
          C[r * ldc + c] = val;
          if (!diag_tile) C[c * ldc + r] = val;
        }
      }
}

// Precision split for the BF16x3 product: A (K x N row-major FP32) ->
// Th = bf16(A^T), Tl = bf16(A^T - Th), both N x Kp with K contiguous and the
// rows padded with zeros to Kp (a multiple of 32). 64x64 tiles through LDS.
__global__ __launch_bounds__(256) void k_split_t(const float *__restrict__ A, int64_t K, int64_t N, int64_t Kp,
                                                  unsigned short *__restrict__ Th, unsigned short *__restrict__ Tl) {
  __shared__ float tile[64][65];
  const int64_t n0 = int64_t(blockIdx.x) * 64, k0 = int64_t(blockIdx.y) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int64_t k = k0 + r, n = n0 + tx;
    tile[r][tx] = (k < K && n < N) ? A[k * N + n] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t n = n0 + r, k = k0 + tx;
    if (n < N && k < Kp) {
      const float x = tile[tx][r];
      const unsigned short h = bf16_rne(x);
      Th[n * Kp + k] = h;
      Tl[n * Kp + k] = bf16_rne(x - bf16_to_f32(h));
    }
  }
}

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// C = alpha * A^T A from the split operands, 128x128 tile per workgroup (tiles on
// or above the diagonal, mirrored), 4 wavefronts of 64x64, K step 32, double-
// buffered LDS. Per 16x16 block and K step: lo*hi + hi*lo + hi*hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the lo*lo term, below
// 2^-16 of the product, is dropped).
__global__ __launch_bounds__(256) void k_syrk_bf16x3(const unsigned short *__restrict__ Th,
                                                      const unsigned short *__restrict__ Tl, int64_t Kp, int64_t N,
                                                      float *__restrict__ C, int64_t ldc, float alpha, int zero_diag,
                                                      int nb, int per) {
  constexpr int BK = 32;
  constexpr int LR = BK + 8;  // padded LDS row in bf16 elements (80 bytes)
  __shared__ __attribute__((aligned(16))) unsigned short S[2][4][TB][LR];  // [buf][Ah Al Bh Bl][row][k]
  int bi, bj;
  if (!tile_of(blockIdx.x, nb, per, &bi, &bj)) return;  // uniform per workgroup
  const bool diag_tile = (bi == bj);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = int64_t(bi) * TB, n0 = int64_t(bj) * TB;
  const int narr = diag_tile ? 2 : 4;
  float4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  // staging: 128 rows x 4 chunks of 16 bytes per array; 2 chunks per thread
  u16x8 st[4][2];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a >= narr) break;
      const unsigned short *src = (a & 1) ? Tl : Th;
      const int64_t r0 = (a < 2) ? m0 : n0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = tid + 256 * h;
        const int row = c >> 2, part = c & 3;
        const int64_t gr = r0 + row;
        if (gr < N)
          st[a][h] = *reinterpret_cast<const u16x8 *>(src + gr * Kp + kb + part * 8);
        else
          st[a][h] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a >= narr) break;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = tid + 256 * h;
        *reinterpret_cast<u16x8 *>(&S[buf][a][c >> 2][(c & 3) * 8]) = st[a][h];
      }
    }
  };
  int buf = 0;
  load(0);
  store(0);
  __syncthreads();
  const int bh = diag_tile ? 0 : 2, bl = diag_tile ? 1 : 3;
  const int kq = (lane >> 4) * 8;
  for (int64_t kb = 0; kb < Kp; kb += BK) {
    const bool more = kb + BK < Kp;
    if (more) load(kb + BK);
    bf16x8 ah[4], al[4], bhv[4], blv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + (lane & 15);
      ah[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&S[buf][0][r][kq]));
      al[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&S[buf][1][r][kq]));
      const int c = wn * 64 + i * 16 + (lane & 15);
      bhv[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&S[buf][bh][c][kq]));
      blv[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&S[buf][bl][c][kq]));
    }
    // the three products of a block are 16 MFMAs apart (independent
    // accumulators in between), so no MFMA waits on its predecessor
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bhv[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], blv[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bhv[j], acc[i][j], 0, 0, 0);
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int64_t c = n0 + wn * 64 + j * 16 + (lane & 15);
        if (r < N && c < N) {
          float val = alpha * acc[i][j][v];
          if (zero_diag && r == c) val = 0.f;
          C[r * ldc + c] = val;
          if (!diag_tile) C[c * ldc + r] = val;
        }
      }
}

// Plain VALU Gram product for FP64 values and exact integer counts:
// 64x64 output tile, 256 threads with 4x4 outputs each, all tiles computed.
template <typename Tin, typename Tacc, typename Tout>
__global__ __launch_bounds__(256) void k_gram_valu(const Tin *__restrict__ A, int64_t K, int64_t N,
                                                    Tout *__restrict__ C, int64_t ldc, Tacc alpha,
                                                    int zero_diag) {
  __shared__ Tin As[16][64];
  __shared__ Tin Bs[16][64];
  const int tid = threadIdx.x;
  const int64_t m0 = int64_t(blockIdx.y) * 64, n0 = int64_t(blockIdx.x) * 64;
  const int tr = (tid >> 4) * 4, tc = (tid & 15) * 4;
  Tacc acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = Tacc(0);
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      int r = e / 64, c = e % 64;
      int64_t kr = k0 + r;
      As[r][c] = (kr < K && m0 + c < N) ? A[kr * N + m0 + c] : Tin(0);
      Bs[r][c] = (kr < K && n0 + c < N) ? A[kr * N + n0 + c] : Tin(0);
    }
    __syncthreads();
    for (int kk = 0; kk < 16; ++kk) {
      Tacc a[4], b[4];
      for (int i = 0; i < 4; ++i) a[i] = Tacc(As[kk][tr + i]);
      for (int j = 0; j < 4; ++j) b[j] = Tacc(Bs[kk][tc + j]);
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      int64_t r = m0 + tr + i, c = n0 + tc + j;
      if (r < N && c < N) {
        Tacc v = alpha * acc[i][j];
        if (zero_diag && r == c) v = Tacc(0);
        C[r * ldc + c] = Tout(v);
      }
    }
}

}  // namespace

int syrk_f32(fpca_context *ctx, const float *A, int64_t K, int64_t N, float *C, int64_t ldc, float alpha,
             bool zero_diag, int prec) {
  if (N <= 0) return FPCA_OK;
  const int nb = int((N + TB - 1) / TB);
  const int tiles = nb * (nb + 1) / 2;
  const int per = (tiles + XCDS - 1) / XCDS;  // tiles per XCD
  const unsigned grid = unsigned(per) * XCDS;
  bool vec = (N % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (prec == FPCA_PREC_BF16X3) {
    const int64_t Kp = ((K + 31) / 32) * 32;
    const size_t half = carve_bytes(size_t(N) * size_t(Kp), 2);
    if (int rc = ws2_reserve(ctx, 2 * half)) return rc;
    unsigned short *Th = static_cast<unsigned short *>(ctx->ws2);
    unsigned short *Tl = reinterpret_cast<unsigned short *>(static_cast<char *>(ctx->ws2) + half);
    if (Kp > 0) {
      dim3 gs((unsigned)((N + 63) / 64), (unsigned)((Kp + 63) / 64));
      hipLaunchKernelGGL(k_split_t, gs, dim3(256), 0, ctx->stream, A, K, N, Kp, Th, Tl);
      FPCA_LAUNCH_CHECK("split_t");
    }
    hipLaunchKernelGGL(k_syrk_bf16x3, dim3(grid), dim3(256), 0, ctx->stream, Th, Tl, Kp, N, C, ldc, alpha,
                       int(zero_diag), nb, per);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_syrk_f32<true>), dim3(grid), dim3(256), 0, ctx->stream, A, K, N, C, ldc, alpha,
                         int(zero_diag), nb, per);
    else
      hipLaunchKernelGGL((k_syrk_f32<false>), dim3(grid), dim3(256), 0, ctx->stream, A, K, N, C, ldc, alpha,
                         int(zero_diag), nb, per);
  }
  FPCA_LAUNCH_CHECK("syrk_f32");
  return FPCA_OK;
}

int syrk_f64(fpca_context *ctx, const double *A, int64_t K, int64_t N, double *C, int64_t ldc, double alpha,
             bool zero_diag) {
  if (N <= 0) return FPCA_OK;
  dim3 grid(unsigned((N + 63) / 64), unsigned((N + 63) / 64));
  hipLaunchKernelGGL((k_gram_valu<double, double, double>), grid, dim3(256), 0, ctx->stream, A, K, N, C, ldc,
                     alpha, int(zero_diag));
  FPCA_LAUNCH_CHECK("syrk_f64");
  return FPCA_OK;
}

// Exact integer Gram product of per-curve count rows (int32) into int64.
int gram_i32(fpca_context *ctx, const int32_t *A, int64_t K, int64_t N, int64_t *C) {
  if (N <= 0) return FPCA_OK;
  dim3 grid(unsigned((N + 63) / 64), unsigned((N + 63) / 64));
  hipLaunchKernelGGL((k_gram_valu<int32_t, int64_t, int64_t>), grid, dim3(256), 0, ctx->stream, A, K, N, C, N,
                     int64_t(1), 0);
  FPCA_LAUNCH_CHECK("gram_i32");
  return FPCA_OK;
}

}  // namespace fpca

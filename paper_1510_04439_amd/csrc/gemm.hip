// Symmetric Gram products C = alpha * A^T A for the covariance binning
// (the Gram form of the pair sums of eq. 2.4): A is K x N row-major (one row
// per curve), C is N x N. Only tiles on or above the diagonal are computed;
// each is also written transposed below the diagonal, and a diagonal tile
// keeps its upper triangle and mirrors it, so C is exactly symmetric.
#include <algorithm>

#include "common.hpp"

namespace fpca {

namespace {

constexpr int TB = 128;  // output tile edge per workgroup
constexpr int TK = 16;   // K rows staged per LDS step
constexpr int LDP = TB + 16;  // padded LDS row (bank spread for the 4 K-rows of an MFMA operand)

typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int XCDS = 8;  // workgroups are dispatched round-robin over the XCDs
constexpr int BAND = 8;  // tile columns per band of the schedule

// Tile number t (0 <= t < nb(nb+1)/2) in band order -> (bi, bj), bi <= bj:
// bands of 8 tile columns; within a band, rows top to bottom with the band's
// columns of a row together, then the band's diagonal triangle. A run of
// consecutive tiles covers a compact block of rows and columns.
__device__ inline bool band_tile(int t, int nb, int *bi, int *bj) {
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

// Tile of workgroup `id` (false for a padding workgroup): workgroup id runs on
// XCD id % 8, and each XCD takes a contiguous run of `per` tiles in band
// order, so the tiles sharing one L2 reuse each other's operand slabs.
__device__ inline bool tile_of(int id, int nb, int per, int *bi, int *bj) {
  return band_tile((id % XCDS) * per + id / XCDS, nb, bi, bj);
}


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
          // upper triangle and its mirror: C is exactly symmetric
          if (!diag_tile || r <= c) {
            float val = alpha * acc[i][j][v];
            if (zero_diag && r == c) val = 0.f;
            C[r * ldc + c] = val;
            if (r != c) C[c * ldc + r] = val;
          }
        }
      }
}

// Precision split for the BF16x3 product: A (K x N row-major FP32) ->
// Th = bf16(A^T), Tl = bf16(A^T - Th), both N x Kp with K contiguous and the
// rows padded with zeros to Kp (a multiple of 64). 64x64 tiles through LDS.
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

//
// With cs1 (and cs2) given, the same pass also leaves the column sums (and
// sums of squares) of its 64 rows in FP64 at cs1[blockIdx.y][n]: four
// groups of 16 consecutive rows, each added in row order, then combined as
// (g0 + g1) + (g2 + g3) -- the chunk sums of the mean's column-sum kernel,
// bit for bit.
__global__ __launch_bounds__(256) void k_split_t(const float *__restrict__ A, int64_t K, int64_t N, int64_t Kp,
                                                  unsigned short *__restrict__ Th, unsigned short *__restrict__ Tl,
                                                  double *__restrict__ cs1, double *__restrict__ cs2) {
  __shared__ float tile[64][65];
  __shared__ double red[2][4][64];
  const int64_t n0 = int64_t(blockIdx.x) * 64, k0 = int64_t(blockIdx.y) * 64;
  // 16 threads per input row, four consecutive n each (16-byte loads where aligned)
  const int q4 = (threadIdx.x & 15) * 4, ty = threadIdx.x >> 4;
  const bool vec = (N % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  for (int r = ty; r < 64; r += 16) {
    const int64_t k = k0 + r, n = n0 + q4;
    if (vec && k < K && n + 3 < N) {
      const float4 v = *reinterpret_cast<const float4 *>(A + k * N + n);
      tile[r][q4] = v.x;
      tile[r][q4 + 1] = v.y;
      tile[r][q4 + 2] = v.z;
      tile[r][q4 + 3] = v.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) tile[r][q4 + e] = (k < K && n + e < N) ? A[k * N + n + e] : 0.f;
    }
  }
  __syncthreads();
  if (cs1) {
    const int cc = threadIdx.x & 63, g = threadIdx.x >> 6;
    double sm = 0.0, sq = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double x = double(tile[16 * g + u][cc]);
      sm += x;
      sq += x * x;
    }
    red[0][g][cc] = sm;
    red[1][g][cc] = sq;
    __syncthreads();
    if (threadIdx.x < 64 && n0 + threadIdx.x < N) {
      const int64_t o = int64_t(blockIdx.y) * N + n0 + threadIdx.x;
      const int c = threadIdx.x;
      cs1[o] = (red[0][0][c] + red[0][1][c]) + (red[0][2][c] + red[0][3][c]);
      if (cs2) cs2[o] = (red[1][0][c] + red[1][1][c]) + (red[1][2][c] + red[1][3][c]);
    }
  }
  // thread -> output row n0 + tid/4, two runs of eight k (16-byte stores)
  const int rn = threadIdx.x >> 2;
  const int64_t n = n0 + rn;
  if (n >= N) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = (threadIdx.x & 3) * 2 + h;  // run c: k = k0 + 8c .. + 7
    if (k0 + 8 * c >= Kp) continue;           // Kp is a multiple of 64, runs are whole
    u16x8 hv, lv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float x = tile[8 * c + e][rn];
      const unsigned short hb = bf16_rne(x);
      hv[e] = hb;
      lv[e] = bf16_rne(x - bf16_to_f32(hb));
    }
    *reinterpret_cast<u16x8 *>(Th + n * Kp + k0 + 8 * c) = hv;
    *reinterpret_cast<u16x8 *>(Tl + n * Kp + k0 + 8 * c) = lv;
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Work split of the persistent SYRK (all tile numbers in band order, S K
// steps of 64 per tile, G workgroups, tiles = F G + W with 0 <= W < G):
//  - "whole" tiles 0 .. D-1, D = tiles - 2W (or all tiles when W = 0): wave f
//    gives workgroup w the tile f G + slot(w), slot(w) = (w % 8) (G / 8) + w / 8,
//    so the tiles of one XCD are a contiguous run; every whole tile starts at
//    K step 0 on all workgroups together, which keeps the operand slabs that
//    neighbouring tiles share in the XCD's L2;
//  - the last 2W tiles ("split" tiles q = 0 .. 2W-1, R = 2 W S iterations)
//    are cut into contiguous chunks: the W workgroups without a tile in the
//    last wave take cap_hi iterations each, the others cap_lo, in that order
//    (rank u). The piece of chunk u in split tile q leaves its accumulators in
//    partial slot u + q: along the iterations every chunk or tile boundary
//    raises u or q, so the slots of the pieces are distinct and below G + 2W.
struct SkPlan {
  int G, S, F, W, D;     // D: number of whole tiles
  int cap_hi, cap_lo;    // chunk sizes of the split tiles
  int64_t R;             // iterations of the split tiles
};

__device__ inline int sk_slot(const SkPlan &pl, int w) { return (w % XCDS) * (pl.G / XCDS) + w / XCDS; }
// rank of workgroup w in the order of the split-tile chunks
__device__ inline int sk_rank(const SkPlan &pl, int w) {
  const int sl = sk_slot(pl, w);
  return sl >= pl.G - pl.W ? sl - (pl.G - pl.W) : pl.W + sl;
}
__device__ inline int64_t sk_begin(const SkPlan &pl, int u) {
  const int64_t b = u < pl.W ? int64_t(u) * pl.cap_hi : int64_t(pl.W) * pl.cap_hi + int64_t(u - pl.W) * pl.cap_lo;
  return min(b, pl.R);
}
__device__ inline int64_t sk_end(const SkPlan &pl, int u) {
  return min(sk_begin(pl, u) + (u < pl.W ? pl.cap_hi : pl.cap_lo), pl.R);
}

// C = alpha * A^T A from the split operands; tiles of 128x128 on or above the
// diagonal (mirrored), 4 wavefronts of 64x64. K goes through LDS 32 at a time
// (one MFMA k-step) in two buffers: the operands of the next step are copied
// from memory straight into the other buffer (16-byte LDS DMA, no registers)
// while this step's MFMAs run, one barrier per step. An LDS row holds the 32 k
// of one operand row as four 16-byte chunks, chunk c of row r at position
// c ^ swz(r), so that the 16 rows an MFMA operand read touches fall on
// distinct banks. Per 16x16 block and k-step: lo*hi + hi*lo + hi*hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the lo*lo term, below
// 2^-16 of the product, is dropped). Whole tiles are written to C; a piece of
// a split tile leaves its accumulators in its partial slot for k_syrk_fixup.
// Rows past N are loaded from row N - 1: they only reach outputs past N,
// which are not written.
__device__ inline int syrk_swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

__global__ __launch_bounds__(256, 2) void k_syrk_bf16x3(const unsigned short *__restrict__ Th,
                                                         const unsigned short *__restrict__ Tl, int64_t Kp, int64_t N,
                                                         float *__restrict__ C, int64_t ldc, float alpha,
                                                         int zero_diag, int nb, SkPlan pl,
                                                         float *__restrict__ part, int vec4) {
  constexpr int BK = 32;  // K per LDS buffer: one MFMA k-step
  constexpr int SBYTES = 2 * 4 * TB * BK * 2;        // [buf][Ah Al Bh Bl][row][k] in bf16
  constexpr int TBYTES = TB * (TB + 1) * 4;          // the epilogue's float tile
  __shared__ __attribute__((aligned(16))) unsigned char lds[SBYTES > TBYTES ? SBYTES : TBYTES];
  auto S = reinterpret_cast<unsigned short(*)[4][TB][BK]>(lds);
  const int w = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int u = sk_rank(pl, w);
  const int64_t j0 = sk_begin(pl, u), j1 = sk_end(pl, u);
  const int nwhole = pl.F;  // waves of whole tiles
  // segment g: whole tile of wave g (g < nwhole), then chunks of split tiles
  int64_t j = j0;
#pragma unroll 1
  for (int g = 0;; ++g) {
    int t, k0, k1, slot = -1;  // slot >= 0: a piece of a split tile
    if (g < nwhole) {
      t = g * pl.G + sk_slot(pl, w);
      if (t >= pl.D) continue;
      k0 = 0;
      k1 = pl.S;
    } else {
      if (j >= j1) break;
      const int q = int(j / pl.S);
      t = pl.D + q;
      k0 = int(j % pl.S);
      k1 = int(min(int64_t(pl.S), k0 + (j1 - j)));
      slot = u + q;
      j += k1 - k0;
    }
    int bi, bj;
    band_tile(t, nb, &bi, &bj);
    const bool diag_tile = (bi == bj);
    const int64_t m0 = int64_t(bi) * TB, n0 = int64_t(bj) * TB;
    const int narr = diag_tile ? 2 : 4;
    float4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) acc[i][jj] = float4_t{0.f, 0.f, 0.f, 0.f};
    // one buffer: per array 128 rows x 4 chunks = 8 wave copies of 64 chunks;
    // wavefront v takes copies v and v + 4 of every array. Lane L of copy cp
    // fills position L % 4 of row 16 cp + L / 4, i.e. chunk (L % 4) ^ swz(row).
    auto dma = [&](int64_t kb, int buf) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a >= narr) break;
        const unsigned short *src = (a & 1) ? Tl : Th;
        const int64_t r0 = (a < 2) ? m0 : n0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cp = wave + 4 * h;
          const int row = 16 * cp + (lane >> 2);
          const int ch = (lane & 3) ^ syrk_swz(row);
          const int64_t gr = min(r0 + row, N - 1);
          __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + gr * Kp + kb + ch * 8),
                                           (__attribute__((address_space(3))) void *)(&S[buf][a][16 * cp][0]), 16,
                                           0, 0);
        }
      }
    };
    const int bh = diag_tile ? 0 : 2, bl = diag_tile ? 1 : 3;
    // lane l reads chunk l / 16 of rows l % 16 (+ 16 i) of its wavefront's 64
    const int kc = lane >> 4;
    auto rd = [&](int buf, int a, int r) {
      return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&S[buf][a][r][8 * (kc ^ syrk_swz(r))]));
    };
    // the three products of a block are 16 MFMAs apart (independent
    // accumulators in between), so no MFMA waits on its predecessor
    auto step = [&](int buf) {
      bf16x8 ah[4], al[4], bhv[4], blv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wm * 64 + i * 16 + (lane & 15);
        const int c = wn * 64 + i * 16 + (lane & 15);
        ah[i] = rd(buf, 0, r);
        al[i] = rd(buf, 1, r);
        bhv[i] = rd(buf, bh, c);
        blv[i] = rd(buf, bl, c);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bhv[jj], acc[i][jj], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], blv[jj], acc[i][jj], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bhv[jj], acc[i][jj], 0, 0, 0);
    };
    // the plan counts K in steps of 64: two LDS buffers' worth each
    const int64_t kb0 = int64_t(k0) * 64, kb1 = int64_t(k1) * 64;
    dma(kb0, 0);
    int buf = 0;
    for (int64_t kb = kb0; kb < kb1; kb += BK) {
      // this wavefront's copies have landed; after the barrier every
      // wavefront's have, and every wavefront is done with the other buffer
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (kb + BK < kb1) dma(kb + BK, buf ^ 1);
      step(buf);
      buf ^= 1;
    }
    __syncthreads();  // the epilogue and the next segment reuse the buffers
    // D layout of a 16x16 MFMA block: lane l, element e -> row 4*(l/16)+e, column l%16
    if (slot < 0) {
      // through LDS (free after the last step's barrier): rows of the tile and
      // rows of its mirror leave as whole 512-byte rows
      constexpr int LDT = TB + 1;
      static_assert(TBYTES >= sizeof(float) * TB * LDT, "the epilogue tile fits in the LDS array");
      float *T = reinterpret_cast<float *>(lds);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            T[(wm * 64 + i * 16 + 4 * (lane >> 4) + e) * LDT + wn * 64 + jj * 16 + (lane & 15)] =
                alpha * acc[i][jj][e];
      __syncthreads();
      for (int q = tid; q < TB * (TB / 4); q += 256) {
        const int a = q / (TB / 4), b4 = (q % (TB / 4)) * 4;
        // direct: row m0 + a, columns n0 + b4 .. + 3 (upper triangle of a diagonal tile)
        {
          const int64_t r = m0 + a, c = n0 + b4;
          float v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = (zero_diag && r == c + k) ? 0.f : T[a * LDT + b4 + k];
          if (vec4 && !diag_tile && r < N && c + 3 < N) {
            *reinterpret_cast<float4_t *>(C + r * ldc + c) = float4_t{v[0], v[1], v[2], v[3]};
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (r < N && c + k < N && (!diag_tile || a <= b4 + k)) C[r * ldc + c + k] = v[k];
          }
        }
        // mirror: row n0 + a, columns m0 + b4 .. + 3 (entries below a diagonal tile's diagonal)
        {
          const int64_t r = n0 + a, c = m0 + b4;
          float v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = T[(b4 + k) * LDT + a];
          if (vec4 && !diag_tile && r < N && c + 3 < N) {
            *reinterpret_cast<float4_t *>(C + r * ldc + c) = float4_t{v[0], v[1], v[2], v[3]};
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (r < N && c + k < N && (!diag_tile || b4 + k < a)) C[r * ldc + c + k] = v[k];
          }
        }
      }
      __syncthreads();  // the next segment stages into the same LDS
    } else {
      float *dst = part + int64_t(slot) * (TB * TB) + (wm * 64 + 4 * (lane >> 4)) * TB + wn * 64 +
                   (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float *row = dst + (i * 16 + e) * TB;
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) row[jj * 16] = acc[i][jj][e];
        }
    }
  }
}

// Split tiles of k_syrk_bf16x3: workgroup (q, slab) adds, in chunk order, the
// pieces of split tile q for 8 rows of the tile (one float4 per thread, the
// pieces' loads issued together) and writes them, and their mirror through an
// LDS transpose, to C.
constexpr int FX_ROWS = 8;
__global__ __launch_bounds__(256) void k_syrk_fixup(const float *__restrict__ part, SkPlan pl, int nb, int64_t N,
                                                     float *__restrict__ C, int64_t ldc, float alpha, int zero_diag) {
  __shared__ float T[FX_ROWS][TB + 1];
  __shared__ const float *src[64];  // the host keeps the pieces of a tile below 64
  __shared__ int nsrc;
  const int q = blockIdx.x / (TB / FX_ROWS), rb = (blockIdx.x % (TB / FX_ROWS)) * FX_ROWS;
  int bi, bj;
  band_tile(pl.D + q, nb, &bi, &bj);
  const int64_t m0 = int64_t(bi) * TB, n0 = int64_t(bj) * TB;
  const int tid = threadIdx.x;
  if (tid < 64) {  // wave 0: chunks u0 .. u0 + 63 that overlap iterations [q S, (q+1) S)
    const int64_t a = int64_t(q) * pl.S, b = a + pl.S;
    const int64_t hi_end = int64_t(pl.W) * pl.cap_hi;  // first chunk ending after a
    const int u0 = a < hi_end ? int(a / pl.cap_hi) : pl.W + int((a - hi_end) / pl.cap_lo);
    const int u = u0 + tid;
    bool ov = false;
    if (u < pl.G) {
      const int64_t j0 = sk_begin(pl, u), j1 = sk_end(pl, u);
      ov = j0 < b && j1 > a;
    }
    if (ov) src[tid] = part + int64_t(u + q) * (TB * TB) + int64_t(rb) * TB;
    const uint64_t m = __ballot(ov);  // the overlapping chunks are consecutive from u0
    if (tid == 0) nsrc = __popcll(m);
  }
  __syncthreads();
  const int ns = nsrc;
  const int rr = tid >> 5, c4 = (tid & 31) * 4;
  const int off = rr * TB + c4;
  float4_t sum = float4_t{0.f, 0.f, 0.f, 0.f};
  int k = 0;
  for (; k + 4 <= ns; k += 4) {
    const float4_t v0 = *reinterpret_cast<const float4_t *>(src[k] + off);
    const float4_t v1 = *reinterpret_cast<const float4_t *>(src[k + 1] + off);
    const float4_t v2 = *reinterpret_cast<const float4_t *>(src[k + 2] + off);
    const float4_t v3 = *reinterpret_cast<const float4_t *>(src[k + 3] + off);
    sum += v0;
    sum += v1;
    sum += v2;
    sum += v3;
  }
  for (; k < ns; ++k) sum += *reinterpret_cast<const float4_t *>(src[k] + off);
  const int64_t r = m0 + rb + rr;
  const bool diag_tile = (bi == bj);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t cc = n0 + c4 + i;
    float val = alpha * sum[i];
    if (zero_diag && r == cc) val = 0.f;
    T[rr][c4 + i] = val;
    if (r < N && cc < N && (!diag_tile || r <= cc)) {  // a diagonal tile: upper triangle and its mirror
      C[r * ldc + cc] = val;
      if (diag_tile && r != cc) C[cc * ldc + r] = val;
    }
  }
  __syncthreads();
  if (!diag_tile) {  // mirror: row n0 + c, columns m0 + rb .. m0 + rb + 7
    const int c = tid >> 1, r4 = (tid & 1) * 4;
    const int64_t mr = n0 + c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t cc = m0 + rb + r4 + i;
      if (mr < N && cc < N) C[mr * ldc + cc] = T[r4 + i][c];
    }
  }
}

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
             bool zero_diag, int prec, double *colsum, double *colsq) {
  if (N <= 0) return FPCA_OK;
  const int nb = int((N + TB - 1) / TB);
  const int tiles = nb * (nb + 1) / 2;
  const int per = (tiles + XCDS - 1) / XCDS;  // tiles per XCD
  const unsigned grid = unsigned(per) * XCDS;
  bool vec = (N % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (prec == FPCA_PREC_BF16X3) {
    const int64_t Kp = ((K + 63) / 64) * 64;
    const int64_t nsteps = Kp / 64;
    // persistent workgroups: two per CU, a multiple of the XCD count
    int G = 2 * ctx->num_cus;
    G = (G / XCDS) * XCDS;
    if (G < XCDS) G = XCDS;
    SkPlan pl{};
    pl.G = G;
    pl.S = int(nsteps);
    pl.F = tiles / G;
    pl.W = tiles % G;
    if (pl.F == 0) {  // a single partial wave: whole tiles only
      pl.F = 1;
      pl.W = 0;
    }
    pl.D = tiles - 2 * pl.W;
    pl.R = int64_t(2) * pl.W * nsteps;
    // chunks of the split tiles: each workgroup ends near ceil(tiles S / G)
    // steps; at most 60 chunks per split tile
    const int64_t c = pl.W > 0 ? std::max<int64_t>((int64_t(pl.W) * nsteps + G - 1) / G, (nsteps + 59) / 60) : 0;
    pl.cap_lo = int(c);
    pl.cap_hi = int(nsteps + c);
    const size_t half = carve_bytes(size_t(N) * size_t(Kp), 2);
    const size_t pbytes = carve_bytes(size_t(G + 2 * pl.W) * TB * TB, 4);
    if (int rc = ws2_reserve(ctx, 2 * half + pbytes)) return rc;
    unsigned short *Th = static_cast<unsigned short *>(ctx->ws2);
    unsigned short *Tl = reinterpret_cast<unsigned short *>(static_cast<char *>(ctx->ws2) + half);
    float *part = reinterpret_cast<float *>(static_cast<char *>(ctx->ws2) + 2 * half);
    if (nsteps == 0) {  // K = 0: the product is zero
      if (ldc == N) return fill_f32(ctx, C, 0.f, N * N);
      for (int64_t r = 0; r < N; ++r)
        if (int rc = fill_f32(ctx, C + r * ldc, 0.f, N)) return rc;
      return FPCA_OK;
    }
    dim3 gs((unsigned)((N + 63) / 64), (unsigned)((Kp + 63) / 64));
    hipLaunchKernelGGL(k_split_t, gs, dim3(256), 0, ctx->stream, A, K, N, Kp, Th, Tl, colsum, colsq);
    FPCA_LAUNCH_CHECK("split_t");
    const int vec4 = (ldc % 4 == 0) && ((reinterpret_cast<uintptr_t>(C) & 15) == 0);
    hipLaunchKernelGGL(k_syrk_bf16x3, dim3(unsigned(G)), dim3(256), 0, ctx->stream, Th, Tl, Kp, N, C, ldc, alpha,
                       int(zero_diag), nb, pl, part, vec4);
    FPCA_LAUNCH_CHECK("syrk_bf16x3");
    if (pl.W > 0) {
      hipLaunchKernelGGL(k_syrk_fixup, dim3(unsigned(2 * pl.W * (TB / FX_ROWS))), dim3(256), 0, ctx->stream, part, pl, nb, N,
                         C, ldc,
                         alpha, int(zero_diag));
      FPCA_LAUNCH_CHECK("syrk_fixup");
    }
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

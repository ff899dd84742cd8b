// Binned local-linear smoothers of the mean (eq. 2.3) and of the raw
// covariance on the 2d-dimensional grid (eq. 2.4).
//
// The moments of the weighted least-squares fit at a node x,
//   S0 = sum w K, S1_k = sum w K u_k, S2_kl = sum w K u_k u_l,
//   T0 = sum g K, T1_k = sum g K u_k,   K = prod_k (1 - u_k^2)_+, u = (y - x)/h,
// factor over the coordinates because the kernel is a product: along each
// coordinate in turn, every partial moment array is correlated with the 1-D
// taps (1-u^2)u^j, j = 0..(remaining degree). This file holds the general
// pass-per-coordinate engine for D <= 6 (partial moments in FP64 for either
// storage type) and the per-node FP64 solve.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "tiled.hpp"
#include "wls.hpp"

namespace fpca {

int smooth_cov_fused_d2(fpca_context *ctx, const fpca_grid *grid, double c0, const float *G, const double *bw,
                        const float *mu, float *gamma, int8_t *status);
bool smooth_cov_fused_d2_supported(const fpca_grid *grid, const double *bw);

namespace {

constexpr int MAXD = 6;
constexpr int MAXMOM = 1 + MAXD + MAXD * (MAXD + 1) / 2 + 1 + MAXD;  // 35

struct MomArray {
  int fam;  // 0: weights (S moments, degree <= 2); 1: sums (T moments, degree <= 1)
  int e[MAXD];
  int deg() const {
    int s = 0;
    for (int k = 0; k < MAXD; ++k) s += e[k];
    return s;
  }
};

// One coordinate pass over a batch of arrays (blockIdx.y = array a):
// o_j[e] = sum_m taps_j[m] src_a[e + m stride]. The source is the FP32 or
// FP64 input on the first pass and an FP64 partial moment after it; the
// partial moments and taps are FP64 so that the normal equations of nearly
// degenerate windows (sparse bins, data on one side of the node) keep their
// singular structure to FP64 rounding.
constexpr int MAXB = MAXMOM + 1;  // arrays in one pass
template <typename TS>
struct PassBatch {
  const TS *src[MAXB];
  double *out[MAXB][3];
  int nj[MAXB];
};

template <typename TS>
__global__ __launch_bounds__(256) void k_pass(int64_t total, int64_t stride, int Mk, PassBatch<TS> pb,
                                               const double *__restrict__ taps, int R) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int a = blockIdx.y;
  const TS *__restrict__ src = pb.src[a];
  const int nj = pb.nj[a];
  const int xk = int((e / stride) % Mk);
  const int lo = -min(R, xk), hi = min(R, Mk - 1 - xk);
  const int W = 2 * R + 1;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  // four taps' loads in flight at a time; the sums run in tap order
  int m = lo;
  for (; m + 3 <= hi; m += 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = double(src[e + int64_t(m + u) * stride]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a0 = fma(taps[m + u + R], v[u], a0);
      if (nj > 1) a1 = fma(taps[W + m + u + R], v[u], a1);
      if (nj > 2) a2 = fma(taps[2 * W + m + u + R], v[u], a2);
    }
  }
  for (; m <= hi; ++m) {
    const double v = double(src[e + int64_t(m) * stride]);
    a0 = fma(taps[m + R], v, a0);
    if (nj > 1) a1 = fma(taps[W + m + R], v, a1);
    if (nj > 2) a2 = fma(taps[2 * W + m + R], v, a2);
  }
  pb.out[a][0][e] = a0;
  if (nj > 1) pb.out[a][1][e] = a1;
  if (nj > 2) pb.out[a][2][e] = a2;
}

struct MomPtrs {
  const double *p[MAXMOM];
};

// ---------------------------------------------------------------- FFT passes
// The same pass by the convolution theorem, for long windows: along a line of
// M values, out_j(o) = sum_m taps_j[m] in(o + m) is the cross-correlation of
// the zero-padded line with the taps, i.e. the inverse FFT of
// FFT(line) * conj(FFT(taps placed circularly)) with L >= M + R (a power of two,
// so the wrap-around never reaches the kept outputs). FP64 complex radix-2 FFTs
// in LDS (one workgroup per line and array); the tap spectra and twiddles are
// formed once per pass. Values below 1e-12 x (max |line| x sum |taps_j|) are
// flushed to zero: they are rounding residue of sums that are exactly zero in
// the direct pass (an empty window keeps S0 = 0 and its EMPTY status).
constexpr int FFT_LMAX = 4096;
constexpr int FFT_T = 256;

__device__ inline int bitrev(int x, int logL) { return int(__brev(unsigned(x)) >> (32 - logL)); }

// In-place radix-2 transforms of nl lines of length L stored one after the
// other in buf (input in bit-reversed order, output in natural order);
// tw[k] = exp(-2 pi i k / L), conjugated for the inverse.
__device__ void fft_lds(double2 *buf, int L, int logL, int nl, const double2 *tw, bool inverse) {
  const int nb = nl * (L / 2);
  for (int s = 1; s <= logL; ++s) {
    const int half = 1 << (s - 1);
    const int tstep = L >> s;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int l = b >> (logL - 1), bb = b & (L / 2 - 1);
      const int grp = bb >> (s - 1), j = bb & (half - 1);
      const int i0 = l * L + grp * (half << 1) + j, i1 = i0 + half;
      double2 w = tw[j * tstep];
      if (inverse) w.y = -w.y;
      const double2 u = buf[i0], v0 = buf[i1];
      const double2 v = make_double2(v0.x * w.x - v0.y * w.y, v0.x * w.y + v0.y * w.x);
      buf[i0] = make_double2(u.x + v.x, u.y + v.y);
      buf[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
  }
}

// Per pass: twiddles (block 0) and, per tap family e (block e), conj(FFT(taps_e
// placed at m mod L)) and sum |taps_e|.
__global__ __launch_bounds__(FFT_T) void k_fft_setup(int L, int logL, int R, const double *__restrict__ taps,
                                                   double2 *__restrict__ tw, double2 *__restrict__ spec,
                                                   double *__restrict__ tapsum) {
  extern __shared__ double2 sm[];
  double2 *buf = sm;      // [L]
  double2 *twl = sm + L;  // [L/2]
  const int e = blockIdx.x, W = 2 * R + 1;
  for (int k = threadIdx.x; k < L / 2; k += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * double(k) / double(L), &sn, &cs);
    twl[k] = make_double2(cs, sn);
    if (e == 0) tw[k] = twl[k];
  }
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    const int m = i <= R ? i : i - L;  // circular position of offset m
    const double v = (m >= -R && m <= R) ? taps[e * W + m + R] : 0.0;
    buf[bitrev(i, logL)] = make_double2(v, 0.0);
  }
  __syncthreads();
  fft_lds(buf, L, logL, 1, twl, false);
  for (int k = threadIdx.x; k < L; k += blockDim.x) spec[e * L + k] = make_double2(buf[k].x, -buf[k].y);
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int m = 0; m < W; ++m) s += fabs(taps[e * W + m]);
    tapsum[e] = s;
  }
}

// Two real lines share one complex transform: line 2i is the real part and
// line 2i+1 the imaginary part. Correlating with real taps is a real-linear
// map, so the inverse transform of (spectrum x tap spectrum) returns line
// 2i's correlation in its real part and line 2i+1's in its imaginary part.
// One workgroup takes npair = FFT_BATCH / L such pairs (L >= 16). Element
// (line l, position x) maps to thread slots so that neighbouring threads
// touch neighbouring addresses: x fastest along the contiguous coordinate
// (stride 1), the line fastest along the others (neighbouring lines are
// neighbours in memory there).
constexpr int FFT_BATCH = 2048;
constexpr int FFT_LMIN = 16;

template <typename TS>
__global__ __launch_bounds__(FFT_T) void k_pass_fft(int64_t stride, int Mk, int64_t nlines, int L, int logL,
                                                  int npair, PassBatch<TS> pb, const double2 *__restrict__ tw,
                                                  const double2 *__restrict__ spec,
                                                  const double *__restrict__ tapsum) {
  extern __shared__ double2 sm[];
  double2 *A = sm;              // [npair][L]: transform of each pair of lines
  double2 *Bf = sm + npair * L;  // [npair][L]: one family's product, then its correlation
  __shared__ unsigned long long amax_l[2 * FFT_BATCH / FFT_LMIN];
  const int a = blockIdx.y;
  const int nl = 2 * npair;
  const int64_t line0 = int64_t(blockIdx.x) * nl;
  const TS *__restrict__ src = pb.src[a];
  const int nj = pb.nj[a];
  const int E = nl * L;
  const bool xfast = stride == 1;
  for (int l = threadIdx.x; l < nl; l += blockDim.x) amax_l[l] = 0ull;
  __syncthreads();
  for (int i = threadIdx.x; i < E; i += blockDim.x) {
    const int l = xfast ? i >> logL : i % nl;
    const int x = xfast ? i & (L - 1) : i / nl;
    const int64_t line = line0 + l;
    double v = 0.0;
    if (x < Mk && line < nlines) {
      const int64_t base = (line / stride) * (stride * Mk) + line % stride;
      v = double(src[base + int64_t(x) * stride]);
    }
    // non-negative doubles order as their bit patterns
    if (v != 0.0) atomicMax(&amax_l[l], static_cast<unsigned long long>(__double_as_longlong(fabs(v))));
    double *slot = reinterpret_cast<double *>(&A[(l >> 1) * L + bitrev(x, logL)]);
    slot[l & 1] = v;
  }
  __syncthreads();
  fft_lds(A, L, logL, npair, tw, false);
  const double inv = 1.0 / double(L);
  const int Ep = npair * L;
  for (int j = 0; j < nj; ++j) {
    for (int i = threadIdx.x; i < Ep; i += blockDim.x) {
      const int k = i & (L - 1);
      const double2 x = A[i], y = spec[j * L + k];
      Bf[(i & ~(L - 1)) + bitrev(k, logL)] = make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
    }
    __syncthreads();
    fft_lds(Bf, L, logL, npair, tw, true);
    const double ts = 1e-12 * tapsum[j];
    double *__restrict__ out = pb.out[a][j];
    for (int i = threadIdx.x; i < E; i += blockDim.x) {
      const int l = xfast ? i >> logL : i % nl;
      const int x = xfast ? i & (L - 1) : i / nl;
      const int64_t line = line0 + l;
      if (x < Mk && line < nlines) {
        const int64_t base = (line / stride) * (stride * Mk) + line % stride;
        const double2 c = Bf[(l >> 1) * L + x];
        const double v = ((l & 1) ? c.y : c.x) * inv;
        const double thr = ts * __longlong_as_double(static_cast<long long>(amax_l[l]));
        out[base + int64_t(x) * stride] = fabs(v) <= thr ? 0.0 : v;
      }
    }
    __syncthreads();
  }
}

}  // namespace

namespace {

template <typename T, int D>
__global__ __launch_bounds__(256) void k_wls(int64_t total, MomPtrs mp, T *__restrict__ out,
                                              int8_t *__restrict__ status) {
  constexpr int NM = 1 + D + D * (D + 1) / 2 + 1 + D;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double m[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) m[i] = mp.p[i][e];
  int8_t st;
  const double b0 = wls_b0<D>(m, &st);
  out[e] = T(b0);
  if (status) status[e] = st;
}

// In-place covariance assembly on 32x32 tile pairs (I <= J):
//   out(p,q) = (b(p,q) + b(q,p))/2 - mu_p mu_q, zero outside the mask.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(int64_t P, T *__restrict__ A, const T *__restrict__ mu,
                                                   const uint8_t *__restrict__ mask, int nb) {
  __shared__ T ta[32][33];
  __shared__ T tb[32][33];
  int id = blockIdx.x, bi = 0;
  while (id >= nb - bi) {
    id -= nb - bi;
    ++bi;
  }
  const int bj = bi + id;
  const int64_t r0 = int64_t(bi) * 32, c0 = int64_t(bj) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int rr = ty; rr < 32; rr += 8) {
    const int64_t r = r0 + rr, c = c0 + tx;
    ta[rr][tx] = (r < P && c < P) ? A[r * P + c] : T(0);
    const int64_t r2 = c0 + rr, c2 = r0 + tx;
    tb[rr][tx] = (r2 < P && c2 < P) ? A[r2 * P + c2] : T(0);
  }
  __syncthreads();
  for (int rr = ty; rr < 32; rr += 8) {
    const int64_t r = r0 + rr, c = c0 + tx;
    if (r < P && c < P) {
      T v = T(0.5) * (ta[rr][tx] + tb[tx][rr]);
      if (mu) v -= mu[r] * mu[c];
      if (mask && (!mask[r] || !mask[c])) v = T(0);
      A[r * P + c] = v;
    }
    const int64_t r2 = c0 + rr, c2 = r0 + tx;
    if (bi != bj && r2 < P && c2 < P) {
      T v = T(0.5) * (tb[rr][tx] + ta[tx][rr]);
      if (mu) v -= mu[r2] * mu[c2];
      if (mask && (!mask[r2] || !mask[c2])) v = T(0);
      A[r2 * P + c2] = v;
    }
  }
}

template <typename T>
__global__ void k_offdiag_fill(T *A, int64_t P, T v) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t step = int64_t(gridDim.x) * blockDim.x;
  for (; e < P * P; e += step) A[e] = (e / P == e % P) ? T(0) : v;
}

inline unsigned nblk(int64_t n) { return unsigned((n + 255) / 256); }

// taps of coordinate k (blockIdx.y) at ts.off[k]: [j][m + R] = (1 - u^2) u^j,
// u = m / (h (M-1)), 0 for |u| >= 1 (j = 0, 1, 2).
struct TapSpec {
  double h[MAXD];
  int M[MAXD], R[MAXD];
  int64_t off[MAXD];
};
__global__ void k_taps(TapSpec ts, double *taps) {
  const int k = blockIdx.y;
  const int R = ts.R[k], W = 2 * R + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * W) return;
  const int j = e / W, m = e % W - R;
  const double u = double(m) / (ts.h[k] * double(ts.M[k] - 1));
  const double K = fabs(u) < 1.0 ? 1.0 - u * u : 0.0;
  taps[ts.off[k] + e] = K * (j == 0 ? 1.0 : (j == 1 ? u : u * u));
}

// 1-D taps (1 - u^2) u^j at offsets m = -R..R, u = m / (h (M-1)), zero for |u| >= 1.
int tap_radius(double h, int M) { return int(std::floor(h * double(M - 1))); }

template <typename T>
int smooth_generic(fpca_context *ctx, int D, const int *dims, const double *h, const T *w, const T *g, T *out,
                   int8_t *status) {
  int64_t total = 1;
  int64_t stride[MAXD];
  for (int k = 0; k < D; ++k) total *= dims[k];
  stride[D - 1] = 1;
  for (int k = D - 2; k >= 0; --k) stride[k] = stride[k + 1] * dims[k + 1];
  int R[MAXD];
  size_t tap_count = 0;
  for (int k = 0; k < D; ++k) {
    R[k] = tap_radius(h[k], dims[k]);
    if (R[k] > 4096) return set_error(FPCA_ERR_UNSUPPORTED, "bandwidth spans too many grid steps");
    tap_count += 3 * size_t(2 * R[k] + 1);
  }
  std::vector<size_t> tap_off(D);
  {
    size_t o = 0;
    for (int k = 0; k < D; ++k) {
      tap_off[k] = o;
      o += 3 * size_t(2 * R[k] + 1);
    }
  }
  // Plan the passes: coordinates from the last (contiguous) to the first.
  std::vector<std::vector<MomArray>> lists(D + 1);
  lists[0].push_back(MomArray{0, {0}});
  lists[0].push_back(MomArray{1, {0}});
  size_t maxA = 0, maxB = 0;
  for (int s = 0; s < D; ++s) {
    const int k = D - 1 - s;
    for (const MomArray &a : lists[s]) {
      const int maxdeg = a.fam == 0 ? 2 : 1;
      for (int j = 0; j <= maxdeg - a.deg(); ++j) {
        MomArray b = a;
        b.e[k] += j;
        lists[s + 1].push_back(b);
      }
    }
    if (s % 2 == 0)
      maxA = std::max(maxA, lists[s + 1].size());
    else
      maxB = std::max(maxB, lists[s + 1].size());
  }
  const size_t bytesA = carve_bytes(maxA * size_t(total), sizeof(double));
  const size_t bytesB = carve_bytes(maxB * size_t(total), sizeof(double));
  const size_t bytesT = carve_bytes(tap_count, sizeof(double));
  const size_t bytesF = carve_bytes(FFT_LMAX / 2 + 3 * FFT_LMAX, sizeof(double2)) + carve_bytes(3, sizeof(double));
  if (int rc = ws_reserve(ctx, bytesA + bytesB + bytesT + bytesF)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  double *bufA = cv.take<double>(maxA * size_t(total));
  double *bufB = cv.take<double>(maxB * size_t(total));
  double *taps = cv.take<double>(tap_count);
  double2 *f_tw = cv.take<double2>(FFT_LMAX / 2);
  double2 *f_spec = cv.take<double2>(3 * FFT_LMAX);
  double *f_sum = cv.take<double>(3);
  // tap tables are computed on the device (no host buffer in the stream: the
  // sequence can be captured into a graph)
  {
    TapSpec ts{};
    int wmax = 1;
    for (int k = 0; k < D; ++k) {
      ts.h[k] = h[k];
      ts.M[k] = dims[k];
      ts.R[k] = R[k];
      ts.off[k] = int64_t(tap_off[k]);
      wmax = std::max(wmax, 2 * R[k] + 1);
    }
    hipLaunchKernelGGL(k_taps, dim3(unsigned((3 * wmax + 255) / 256), unsigned(D)), dim3(256), 0, ctx->stream, ts,
                       taps);
    FPCA_LAUNCH_CHECK("taps");
  }

  std::vector<const double *> cur;
  for (int s = 0; s < D; ++s) {
    const int k = D - 1 - s;
    double *dst = (s % 2 == 0) ? bufA : bufB;
    std::vector<const double *> next;
    PassBatch<T> b0{};      // first pass: the inputs, in their storage type
    PassBatch<double> b1{};  // later passes: FP64 partial moments
    const int na = int(lists[s].size());
    if (na > MAXB) return set_error(FPCA_ERR_UNSUPPORTED, "too many moment arrays in one pass");
    size_t o = 0;
    for (int a = 0; a < na; ++a) {
      const MomArray &m = lists[s][a];
      const int nj = (m.fam == 0 ? 2 : 1) - m.deg() + 1;
      for (int j = 0; j < 3; ++j) {
        double *oj = j < nj ? dst + (o + j) * size_t(total) : nullptr;
        if (j < nj) next.push_back(oj);
        b0.out[a][j] = b1.out[a][j] = oj;
      }
      b0.nj[a] = b1.nj[a] = nj;
      if (s == 0)
        b0.src[a] = a == 0 ? w : g;
      else
        b1.src[a] = cur[a];
      o += nj;
    }
    // direct or FFT pass (the handle's convolution mode; AUTO times both the
    // first time a pass shape is met and keeps the faster)
    int L = FFT_LMIN, logL = 4;
    while (L < dims[k] + R[k]) {
      L <<= 1;
      ++logL;
    }
    const bool fft_ok = L <= FFT_LMAX && total / dims[k] <= 0x7fffffffLL;
    auto run_direct = [&]() -> int {
      if (s == 0)
        hipLaunchKernelGGL(k_pass<T>, dim3(nblk(total), unsigned(na)), dim3(256), 0, ctx->stream, total, stride[k],
                           dims[k], b0, taps + tap_off[k], R[k]);
      else
        hipLaunchKernelGGL(k_pass<double>, dim3(nblk(total), unsigned(na)), dim3(256), 0, ctx->stream, total,
                           stride[k], dims[k], b1, taps + tap_off[k], R[k]);
      FPCA_LAUNCH_CHECK("moment pass");
      return FPCA_OK;
    };
    auto run_fft = [&]() -> int {
      // up to 96 KB (setup) and 128 KB (pass) of dynamic LDS at L = 4096
      FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_setup),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, FFT_LMAX * 24));
      FPCA_HIP(hipFuncSetAttribute(s == 0 ? reinterpret_cast<const void *>(&k_pass_fft<T>)
                                          : reinterpret_cast<const void *>(&k_pass_fft<double>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, FFT_LMAX * 32));
      hipLaunchKernelGGL(k_fft_setup, dim3(3), dim3(FFT_T), size_t(L) * 24, ctx->stream, L, logL, R[k],
                         taps + tap_off[k], f_tw, f_spec, f_sum);
      FPCA_LAUNCH_CHECK("fft setup");
      const int64_t nlines = total / dims[k];
      const int npair = std::max(1, FFT_BATCH / L);
      const dim3 grid(unsigned((nlines + 2 * npair - 1) / (2 * npair)), unsigned(na));
      const size_t lds = size_t(npair) * L * 32;
      if (s == 0)
        hipLaunchKernelGGL(k_pass_fft<T>, grid, dim3(FFT_T), lds, ctx->stream, stride[k], dims[k], nlines, L, logL,
                           npair, b0, f_tw, f_spec, f_sum);
      else
        hipLaunchKernelGGL(k_pass_fft<double>, grid, dim3(FFT_T), lds, ctx->stream, stride[k], dims[k], nlines, L,
                           logL, npair, b1, f_tw, f_spec, f_sum);
      FPCA_LAUNCH_CHECK("fft pass");
      return FPCA_OK;
    };
    int method = 0;  // 0 direct, 1 FFT
    if (fft_ok && ctx->conv_mode == FPCA_CONV_FFT) method = 1;
    if (fft_ok && ctx->conv_mode == FPCA_CONV_AUTO) {
      const std::vector<int64_t> key = {int64_t(s == 0 ? sizeof(T) : 8), total, stride[k], dims[k], R[k], na};
      int found = -1;
      for (const auto &e : ctx->conv_cache)
        if (e.first == key) found = e.second;
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      (void)hipStreamIsCapturing(ctx->stream, &cs);
      if (found < 0 && cs == hipStreamCaptureStatusNone) {
        hipEvent_t e0, e1, e2;
        FPCA_HIP(hipEventCreate(&e0));
        FPCA_HIP(hipEventCreate(&e1));
        FPCA_HIP(hipEventCreate(&e2));
        FPCA_HIP(hipEventRecord(e0, ctx->stream));
        if (int rc = run_fft()) return rc;
        FPCA_HIP(hipEventRecord(e1, ctx->stream));
        if (int rc = run_direct()) return rc;
        FPCA_HIP(hipEventRecord(e2, ctx->stream));
        FPCA_HIP(hipEventSynchronize(e2));
        float t_fft = 0.f, t_dir = 0.f;
        FPCA_HIP(hipEventElapsedTime(&t_fft, e0, e1));
        FPCA_HIP(hipEventElapsedTime(&t_dir, e1, e2));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        found = t_fft < t_dir ? 1 : 0;
        ctx->conv_cache.push_back({key, found});
      }
      method = found > 0 ? 1 : 0;
    }
    if (int rc = method == 1 ? run_fft() : run_direct()) return rc;
    cur.swap(next);
  }
  // Gather the final arrays in moment order.
  MomPtrs mp{};
  const std::vector<MomArray> &fin = lists[D];
  auto find = [&](int fam, const int *e) -> const double * {
    for (size_t i = 0; i < fin.size(); ++i) {
      if (fin[i].fam != fam) continue;
      bool eq = true;
      for (int k = 0; k < D; ++k) eq &= fin[i].e[k] == e[k];
      if (eq) return cur[i];
    }
    return nullptr;
  };
  int q = 0;
  int e[MAXD] = {0};
  mp.p[q++] = find(0, e);
  for (int k = 0; k < D; ++k) {
    int ek[MAXD] = {0};
    ek[k] = 1;
    mp.p[q++] = find(0, ek);
  }
  for (int k = 0; k < D; ++k)
    for (int l = k; l < D; ++l) {
      int ek[MAXD] = {0};
      ek[k] += 1;
      ek[l] += 1;
      mp.p[q++] = find(0, ek);
    }
  mp.p[q++] = find(1, e);
  for (int k = 0; k < D; ++k) {
    int ek[MAXD] = {0};
    ek[k] = 1;
    mp.p[q++] = find(1, ek);
  }
  for (int i = 0; i < q; ++i)
    if (!mp.p[i]) return set_error(FPCA_ERR_DEVICE, "internal: moment %d missing", i);
  switch (D) {
#define WLS_CASE(DD)                                                                                        \
  case DD:                                                                                                  \
    hipLaunchKernelGGL((k_wls<T, DD>), dim3(nblk(total)), dim3(256), 0, ctx->stream, total, mp, out, status); \
    break;
    WLS_CASE(1)
    WLS_CASE(2)
    WLS_CASE(3)
    WLS_CASE(4)
    WLS_CASE(5)
    WLS_CASE(6)
#undef WLS_CASE
    default:
      return set_error(FPCA_ERR_UNSUPPORTED, "D=%d", D);
  }
  FPCA_LAUNCH_CHECK("wls");
  return FPCA_OK;
}

int check_bw(const double *bw, int d) {
  if (!bw) return set_error(FPCA_ERR_INVALID_ARG, "bandwidth is required");
  for (int k = 0; k < d; ++k)
    if (!(bw[k] > 0.0) || !std::isfinite(bw[k]))
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidth[%d] must be positive and finite", k);
  return FPCA_OK;
}

template <typename T>
int assemble(fpca_context *ctx, int64_t P, T *A, const T *mu, const uint8_t *mask) {
  const int nb = int((P + 31) / 32);
  hipLaunchKernelGGL(k_assemble<T>, dim3(unsigned(nb * (nb + 1) / 2)), dim3(256), 0, ctx->stream, P, A, mu, mask,
                     nb);
  FPCA_LAUNCH_CHECK("assemble");
  return FPCA_OK;
}

template <typename T>
int smooth_cov_impl(fpca_context *ctx, const fpca_grid *grid, const T *C, double c_uniform, const T *G,
                    const T *mu, const double *bw, T *gamma, int8_t *status) {
  const GridDims gd = make_dims(grid);
  const int64_t P = gd.P;
  const int d = grid->d;
  if constexpr (sizeof(T) == 4) {
    if (!C && smooth_cov_fused_d2_supported(grid, bw))
      return smooth_cov_fused_d2(ctx, grid, c_uniform, G, bw, mu, gamma, status);
  }
  if (use_queue_engine(ctx, grid)) {
    // the persistent-queue engine: FP64 moments kept on chip between passes
    std::vector<TiledJob> jobs(1);
    TiledJob &j = jobs[0];
    j = TiledJob{};
    j.grid = grid;
    j.Ca = C;
    j.Ga = G;
    j.c0 = c_uniform;
    j.h = bw;
    j.out = gamma;
    j.status = status;
    TiledConfig cfg;
    size_t lds = tiled_lds(jobs, 16);
    cfg.qb = 16;
    if (!lds || lds > 80 * 1024) {
      cfg.qb = 8;
      lds = tiled_lds(jobs, 8);
    }
    if (lds) {
      cfg.wg_per_cu = int(std::max<size_t>(1, std::min<size_t>(2, (160 * 1024) / (lds + 256))));
      TiledLaunch L;
      if (int rc = tiled_plan<T>(ctx, jobs, false, cfg, &L)) return rc;
      if (int rc = tiled_queue(ctx, L)) return rc;
      return assemble<T>(ctx, P, gamma, mu, grid->mask);
    }
  }
  int dims[MAXD];
  double h[MAXD];
  for (int k = 0; k < d; ++k) {
    dims[k] = dims[k + d] = grid->M[k];
    h[k] = h[k + d] = bw[k];
  }
  if (!C) {
    // complete common grid: the pair weights c_uniform (1 - delta_pq) are
    // materialized for the general engine, in the handle's second arena
    if (int rc = ws2_reserve(ctx, carve_bytes(size_t(P) * P, sizeof(T)))) return rc;
    T *tmp = static_cast<T *>(ctx->ws2);
    hipLaunchKernelGGL(k_offdiag_fill<T>, dim3(nblk(P * P) > 65536 ? 65536 : nblk(P * P)), dim3(256), 0,
                       ctx->stream, tmp, P, T(c_uniform));
    FPCA_LAUNCH_CHECK("offdiag");
    if (int rc = smooth_generic<T>(ctx, 2 * d, dims, h, tmp, G, gamma, status)) return rc;
  } else {
    if (int rc = smooth_generic<T>(ctx, 2 * d, dims, h, C, G, gamma, status)) return rc;
  }
  return assemble<T>(ctx, P, gamma, mu, grid->mask);
}

}  // namespace

bool use_queue_engine(const fpca_context *ctx, const fpca_grid *grid) {
  if (!tiled_supported(grid) || ctx->engine == FPCA_ENGINE_PASSES) return false;
  if (ctx->engine == FPCA_ENGINE_QUEUE) return true;
  int64_t P = 1;
  for (int k = 0; k < grid->d; ++k) P *= grid->M[k];
  const int D = 2 * grid->d;
  const double foot = double(P) * double(P) * 8.0 * double(2 + 2 * D + D * (D + 1) / 2);
  return foot > double(256 << 20);
}

}  // namespace fpca

using namespace fpca;

extern "C" int fpca_smooth_mean(fpca_handle ctx, const fpca_grid *grid, int dtype, const void *weights,
                                const void *sums, int kernel, const double *bandwidth, void *mu, int8_t *status) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (kernel != FPCA_K_EPANECHNIKOV) return set_error(FPCA_ERR_UNSUPPORTED, "kernel %d", kernel);
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (!weights || !sums || !mu) return set_error(FPCA_ERR_INVALID_ARG, "weights, sums and mu are required");
  if (int rc = check_bw(bandwidth, grid->d)) return rc;
  if (int rc = set_device(ctx)) return rc;
  if (dtype == FPCA_F64)
    return smooth_generic<double>(ctx, grid->d, grid->M, bandwidth, static_cast<const double *>(weights),
                                  static_cast<const double *>(sums), static_cast<double *>(mu), status);
  return smooth_generic<float>(ctx, grid->d, grid->M, bandwidth, static_cast<const float *>(weights),
                               static_cast<const float *>(sums), static_cast<float *>(mu), status);
}

extern "C" int fpca_smooth_cov(fpca_handle ctx, const fpca_grid *grid, int dtype, const void *C, double c_uniform,
                               const void *G, const void *mu, int kernel, const double *bandwidth, void *gamma,
                               int8_t *status) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (kernel != FPCA_K_EPANECHNIKOV) return set_error(FPCA_ERR_UNSUPPORTED, "kernel %d", kernel);
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (!G || !gamma) return set_error(FPCA_ERR_INVALID_ARG, "G and gamma are required");
  if (!C && !(c_uniform > 0.0 && std::isfinite(c_uniform)))
    return set_error(FPCA_ERR_INVALID_ARG, "C = NULL needs a positive c_uniform");
  if (P > (int64_t(1) << 15)) return set_error(FPCA_ERR_UNSUPPORTED, "covariance grid too large (P=%lld)", (long long)P);
  if (int rc = check_bw(bandwidth, grid->d)) return rc;
  if (int rc = set_device(ctx)) return rc;
  return smooth_cov_internal(ctx, grid, dtype, C, c_uniform, G, mu, bandwidth, gamma, status);
}

int fpca::smooth_cov_internal(fpca_context *ctx, const fpca_grid *grid, int dtype, const void *C, double c_uniform,
                              const void *G, const void *mu, const double *bandwidth, void *gamma, int8_t *status) {
  if (dtype == FPCA_F64)
    return smooth_cov_impl<double>(ctx, grid, static_cast<const double *>(C), c_uniform,
                                   static_cast<const double *>(G), static_cast<const double *>(mu), bandwidth,
                                   static_cast<double *>(gamma), status);
  return smooth_cov_impl<float>(ctx, grid, static_cast<const float *>(C), c_uniform, static_cast<const float *>(G),
                                static_cast<const float *>(mu), bandwidth, static_cast<float *>(gamma), status);
}

extern "C" int fpca_set_conv(fpca_handle ctx, int mode) {
  if (int rc = check_handle(ctx)) return rc;
  if (mode != FPCA_CONV_DIRECT && mode != FPCA_CONV_FFT && mode != FPCA_CONV_AUTO)
    return set_error(FPCA_ERR_INVALID_ARG, "bad convolution mode %d", mode);
  ctx->conv_mode = mode;
  return FPCA_OK;
}

extern "C" int fpca_set_engine(fpca_handle ctx, int engine) {
  if (int rc = check_handle(ctx)) return rc;
  if (engine != FPCA_ENGINE_AUTO && engine != FPCA_ENGINE_QUEUE && engine != FPCA_ENGINE_PASSES)
    return set_error(FPCA_ERR_INVALID_ARG, "bad engine %d", engine);
  ctx->engine = engine;
  return FPCA_OK;
}

// Covariance smoother for general pair weights (eq. 2.4 on the 2d-dimensional
// grid, any C) and the batched cross-validation built on it (Section 3.3's
// criterion read on folds of curves), as ONE persistent launch that drains a
// queue of tasks.
//
// The moments of the local-linear fit factor over the 2d coordinates
// (product kernel), so they are formed by 1-D passes with the taps
// (1-u^2)u^e, e = 0..2. The passes are grouped into three stages that keep
// their intermediates on chip and write only the arrays the next stage needs,
// in FP64 (windows can be exactly degenerate with sparse or masked data, and
// FP64 keeps such systems singular to rounding, so the status rule holds):
//
//  stage T   one task per s-row p: the whole t-block of that row (P nodes) in
//            LDS; passes t_d .. t_1, depth first, so at most two t-blocks of
//            partial moments are live; emits the t-moment arrays
//            X[x][p][q] (C: t-degree <= 2, G: t-degree <= 1; 14 for d = 3).
//  stage S   one task per (s_1 index, block of QB t-columns): the remaining
//            s-coordinates s_d .. s_2 of those columns in LDS; emits
//            Y[y][p][q] (27 arrays for d = 3). For d = 1 there is nothing to
//            do and Y is X.
//  stage W   one task per (block of s-positions other than s_1, block of QB
//            t-columns): for each position the s_1 pass of every Y array
//            lands in LDS as the final moments of M_1 x QB nodes, then one
//            lane per node solves the (2d+1) x (2d+1) system in FP64
//            (wls_b0) and writes b0 (and the status).
//  score     (cross-validation) tile pairs of b0, masked and scored against
//            the held-out fold: sum Q_f - 2 G_f g + C_f g^2, FP64 partial per
//            task. C and G are symmetric, so a score needs b0 at p <= q only
//            (s_1 <= t_1): in cross-validation stage W solves those nodes and
//            stage S skips the rows no such node reads.
//  finish    the partials of a job summed in a fixed order.
//
// The queue is a list of segments (job, stage, task count) in rounds: round r
// holds stage T of job r, stage S of job r-1, W of r-2, score of r-3 and
// finish of r-4, so the stages of consecutive jobs overlap. A task waits (a
// bounded spin on a completion counter, then an acquire fence) only for tasks
// placed earlier in the queue: its own job's previous stage, and the job that
// last used the same intermediate slot. Tasks are taken in queue order by
// running workgroups, so every awaited task has been taken by a workgroup
// that does not wait on a later one: the queue always drains. Completion is
// published by a release fence in every thread, a barrier and a counter
// increment; intermediates cross XCDs through memory.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "tiled.hpp"
#include "wls.hpp"

namespace fpca {

namespace {

// ------------------------------------------------------------------ sync
__device__ inline bool wait_done(const int *c, int target, long long limit, int *err) {
  long long it = 0;
  while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++it > limit) {
      __hip_atomic_fetch_or(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// ------------------------------------------------------------------ passes
// A block of up to three axes (A, B, C) with sizes n[] and element strides s[].
struct Blk {
  int n[3];
  long long s[3];
};

// Taps live in a small per-launch table in global memory, read through the
// constant address space: their index is the same for every lane, so they are
// scalar loads into SGPRs that feed the FMAs directly.
typedef const __attribute__((address_space(4))) double CDbl;
// LDS pointers keep their address space, so their loads are ds_read.
typedef __attribute__((address_space(3))) double LDbl;

constexpr int TQ_KC = 8;  // window reads issued together
constexpr int TQ_U = 8;   // global reads per thread issued before their LDS stores

// dst[at(e)] = get(e) for e < n (at(e) = e by default): every thread issues
// TQ_U independent reads before storing them, so a workgroup keeps
// TQ_U * TQ_THREADS reads in flight.
template <typename GET, typename DST>
__device__ inline void stage_to_lds(__attribute__((address_space(3))) double *dst, int n, GET get, DST at) {
  for (int b = threadIdx.x; b < n; b += TQ_U * TQ_THREADS) {
    double v[TQ_U];
#pragma unroll
    for (int u = 0; u < TQ_U; ++u) {
      const int e = b + u * TQ_THREADS;
      v[u] = e < n ? get(e) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TQ_U; ++u) {
      const int e = b + u * TQ_THREADS;
      if (e < n) dst[at(e)] = v[u];
    }
  }
}
template <typename GET>
__device__ inline void stage_to_lds(__attribute__((address_space(3))) double *dst, int n, GET get) {
  stage_to_lds(dst, n, get, [](int e) { return e; });
}

// q = x / d and r = x % d for 0 <= x < 2^22 and a small divisor d, from a
// float reciprocal rd = 1/d (one product and one correction step).
__device__ inline void fast_divmod(int x, int d, float rd, int &q, int &r) {
  q = int(float(x) * rd);
  r = x - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
}

// acc[j][q] += sum over |m| <= R of t_j[m + R] * in(x0 + q + m), q < TQ_SEG,
// with in(x) = ld(x) for 0 <= x < n and 0 outside. A register window slides
// over m: each step reads one new value and issues TQ_SEG FMAs per output
// family; the tap index is the same for every lane (scalar loads).
template <typename LD>
__device__ inline void window_acc(LD ld, int x0, int n, int R, CDbl *t0, CDbl *t1, CDbl *t2, int nj,
                                  double (&acc)[3][TQ_SEG]) {
  auto ldz = [&](int x) {
    const int xc = min(max(x, 0), n - 1);
    const double v = ld(xc);
    return x == xc ? v : 0.0;
  };
  double w[TQ_SEG];
#pragma unroll
  for (int q = 0; q < TQ_SEG; ++q) w[q] = ldz(x0 + q - R);
  const int W = 2 * R + 1;
  // steps m = -R + k, k = 0..W-1, in chunks of TQ_KC whose reads are issued
  // together before the chunk's FMAs
  for (int kc = 0; kc < W; kc += TQ_KC) {
    double nx[TQ_KC];
#pragma unroll
    for (int i = 0; i < TQ_KC; ++i) nx[i] = ldz(x0 + TQ_SEG - R + kc + i);
#pragma unroll
    for (int i = 0; i < TQ_KC; ++i) {
      if (kc + i < W) {
        const double a0 = t0[kc + i];
#pragma unroll
        for (int q = 0; q < TQ_SEG; ++q) acc[0][q] = fma(a0, w[q], acc[0][q]);
        if (nj > 1) {
          const double a1 = t1[kc + i];
#pragma unroll
          for (int q = 0; q < TQ_SEG; ++q) acc[1][q] = fma(a1, w[q], acc[1][q]);
        }
        if (nj > 2) {
          const double a2 = t2[kc + i];
#pragma unroll
          for (int q = 0; q < TQ_SEG; ++q) acc[2][q] = fma(a2, w[q], acc[2][q]);
        }
#pragma unroll
        for (int q = 0; q + 1 < TQ_SEG; ++q) w[q] = w[q + 1];
        w[TQ_SEG - 1] = nx[i];
      }
    }
  }
}

// One pass along axis `ax` of block `bk`: for every line (the other two axes)
// and output position o along ax,
//   out_j(o) = sum_{|m| <= R} taps[(e0 + j) * W + m + R] * in(o + m),  j < nj,
// with in(x) = 0 outside 0..n-1. Each lane forms TQ_SEG consecutive outputs;
// lanes take consecutive lines. `ld(i)` reads the source at element offset i,
// `st(j, i, v)` stores output j at offset i (same offsets in the destination).
template <int ax, typename LD, typename STF>
__device__ inline void pass_axis(const Blk &bk, CDbl *taps, int R, int e0, int nj, LD ld, STF st, int lo = 0) {
  // lo > 0 limits the pass to axis-0 indices >= lo: for ax = 0 the outputs
  // from the segment holding lo on (lo a multiple of TQ_SEG), otherwise the
  // lines whose axis-0 index is >= lo
  constexpr int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
  const int n2 = bk.n[o2];
  const int l1lo = ax == 0 ? 0 : lo;
  const int nl = (bk.n[o1] - l1lo) * n2;
  const int n = bk.n[ax];
  const int sglo = ax == 0 ? lo / TQ_SEG : 0;
  const int nseg = (n + TQ_SEG - 1) / TQ_SEG - sglo;
  const int W = 2 * R + 1;
  const long long sx = bk.s[ax];
  const float rnl = 1.0f / float(nl), rn2 = 1.0f / float(n2);
  for (int it = threadIdx.x; it < nl * nseg; it += TQ_THREADS) {
    int sg, line, l1, l2;
    fast_divmod(it, nl, rnl, sg, line);
    fast_divmod(line, n2, rn2, l1, l2);
    l1 += l1lo;
    const long long base = (long long)l1 * bk.s[o1] + (long long)l2 * bk.s[o2];
    const int x0 = (sg + sglo) * TQ_SEG;
    double acc[3][TQ_SEG];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int q = 0; q < TQ_SEG; ++q) acc[j][q] = 0.0;
    window_acc([&](int xc) { return ld(base + xc * sx); }, x0, n, R, taps + e0 * W, taps + (e0 + 1) * W,
               taps + (e0 + 2) * W, nj, acc);
#pragma unroll
    for (int q = 0; q < TQ_SEG; ++q) {
      if (x0 + q < n) {
        const long long i = base + (x0 + q) * sx;
        st(0, i, acc[0][q]);
        if (nj > 1) st(1, i, acc[1][q]);
        if (nj > 2) st(2, i, acc[2][q]);
      }
    }
  }
}

// taps of coordinate k: [e][m + R], e = 0..2, u = m / (h (M-1)) (written by
// the host into the launch's tap table).
__device__ inline CDbl *tap_ptr(const TArgs &a, const TJob &jb, int k) {
  const int off = k == 0 ? jb.tap_off[0] : (k == 1 ? jb.tap_off[1] : jb.tap_off[2]);
  return (CDbl *)(a.taps + off);
}

// The job's intermediate slots (selects, not an indexed kernel-argument array,
// which would be copied to scratch memory).
__device__ inline double *slot_x(const TArgs &a, int sl) { return sl == 0 ? a.X[0] : (sl == 1 ? a.X[1] : a.X[2]); }
__device__ inline double *slot_y(const TArgs &a, int sl) { return sl == 0 ? a.Y[0] : (sl == 1 ? a.Y[1] : a.Y[2]); }
__device__ inline void *slot_g(const TArgs &a, int sl) { return sl == 0 ? a.Gh[0] : (sl == 1 ? a.Gh[1] : a.Gh[2]); }

// ------------------------------------------------------------------ stage T
template <typename T, int d>
__device__ void stage_t(const TArgs &a, const TJob &jb, int p, LDbl *lds) {
  LDbl *L0 = lds;  // the input row, FP64 (staged with all loads in flight)
  LDbl *L1 = L0 + jb.P;
  LDbl *L2 = L1 + jb.P;
  const long long P = jb.P;
  double *X = slot_x(a, jb.slot);
  // t-block as axes (A, B, C) = (t1, t2, t3), last coordinate fastest
  Blk bk;
  bk.n[0] = d == 3 ? jb.M[0] : 1;
  bk.n[1] = d == 3 ? jb.M[1] : (d == 2 ? jb.M[0] : 1);
  bk.n[2] = jb.M[d - 1];
  bk.s[2] = 1;
  bk.s[1] = bk.n[2];
  bk.s[0] = (long long)bk.n[1] * bk.n[2];
  // Cross-validation (d = 3): stage S reads row p (s_1 = p / PR) only in
  // column blocks whose last t_1 is >= s_1 - R, i.e. columns with
  // t_1 >= t1_lo (QB divides PR = M_2 M_3 here); the t_1 pass forms those from
  // the segment holding t1_lo on (t1_out) and reads t-slabs t_1 >= t1_in,
  // the only ones the t_3 and t_2 passes need to form.
  int t1_out = 0, t1_in = 0;
  if (d == 3 && a.cv && (P / jb.M[0]) % a.qb == 0) {
    const int t1_lo = max(0, int(p / (P / jb.M[0])) - jb.R[0]);
    t1_out = (t1_lo / TQ_SEG) * TQ_SEG;
    t1_in = max(0, t1_out - jb.R[0]);
  }
  int xi = 0;
  for (int fam = 0; fam < 2; ++fam) {
    const int md = 2 - fam;
    const T *A = (fam == 0 && !jb.Ca) ? nullptr : static_cast<const T *>(fam == 0 ? jb.Ca : jb.Ga) + p * P;
    const T *B = (fam == 0 ? jb.Cb : jb.Gb) ? static_cast<const T *>(fam == 0 ? jb.Cb : jb.Gb) + p * P : nullptr;
    const bool uni = fam == 0 && !jb.Ca;  // complete common grid: C = c0 (1 - delta)
    const double c0 = jb.c0;
    if (fam == 1) __syncthreads();  // the C passes have finished reading L0
    stage_to_lds(L0, jb.P,
                 [&](int i) { return uni ? (i == p ? 0.0 : c0) : (B ? double(A[i]) - double(B[i]) : double(A[i])); });
    __syncthreads();
    auto ldg = [&](long long i) { return L0[i]; };
    const int kc = d - 1;  // coordinate of axis C (t_d)
    if constexpr (d == 1) {
      const int nj = md + 1;
      pass_axis<2>(bk, tap_ptr(a, jb, kc), jb.R[kc], 0, nj, ldg,
                [&](int j, long long i, double v) { X[(long long)(xi + j) * P * P + p * P + i] = v; });
      xi += nj;
    } else {
      for (int ec = 0; ec <= md; ++ec) {
        pass_axis<2>(bk, tap_ptr(a, jb, kc), jb.R[kc], ec, 1, ldg, [&](int, long long i, double v) { L1[i] = v; },
                     t1_in);
        __syncthreads();
        if constexpr (d == 2) {
          const int nj = md - ec + 1;
          pass_axis<1>(bk, tap_ptr(a, jb, 0), jb.R[0], 0, nj, [&](long long i) { return L1[i]; },
              [&](int j, long long i, double v) { X[(long long)(xi + j) * P * P + p * P + i] = v; });
          xi += nj;
          __syncthreads();
        } else {
          for (int eb = 0; eb <= md - ec; ++eb) {
            pass_axis<1>(bk, tap_ptr(a, jb, 1), jb.R[1], eb, 1, [&](long long i) { return L1[i]; },
                [&](int, long long i, double v) { L2[i] = v; }, t1_in);
            __syncthreads();
            const int nj = md - ec - eb + 1;
            pass_axis<0>(bk, tap_ptr(a, jb, 0), jb.R[0], 0, nj, [&](long long i) { return L2[i]; },
                [&](int j, long long i, double v) { X[(long long)(xi + j) * P * P + p * P + i] = v; }, t1_out);
            xi += nj;
            __syncthreads();
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ stage S
// Task (s_1 index a1, column block qb): block (A, B, C) = (s_2, s_3, q) for
// d = 3, (1, s_2, q) for d = 2.
template <int d>
__device__ void stage_s(const TArgs &a, const TJob &jb, int task, LDbl *lds) {
  const int QB = a.qb;
  const long long P = jb.P;
  const int nqb = (jb.P + QB - 1) / QB;
  const int a1 = task / nqb, q0 = (task % nqb) * QB;
  const int qn = min(QB, jb.P - q0);
  const int PR = jb.P / jb.M[0];  // s-positions per s_1 index
  // cross-validation scores only need nodes p <= q (s_1 <= t_1): the s_1 pass
  // of stage W reads this row only for outputs within R of it
  if (a.cv && a1 > (q0 + qn - 1) / PR + jb.R[0]) return;
  LDbl *L0 = lds;
  LDbl *L1 = L0 + (long long)PR * QB;
  const double *X = slot_x(a, jb.slot);
  double *Y = slot_y(a, jb.slot);
  Blk bk;
  bk.n[0] = d == 3 ? jb.M[1] : 1;
  bk.n[1] = jb.M[d - 1];
  bk.n[2] = qn;
  bk.s[2] = 1;
  bk.s[1] = QB;
  bk.s[0] = (long long)bk.n[1] * QB;
  const long long prow = (long long)a1 * PR;  // first s-node of this s_1 index
  const float rqb = 1.0f / float(QB);
  // The block of array x + 1 is read into registers (TQ_SPF per thread, every
  // load issued at clamped addresses, then masked) while the passes of array
  // x run; PR * QB <= TQ_SPF * TQ_THREADS (checked by the planner).
  double pf[TQ_SPF];
  auto fetch = [&](int x) {
    const double *Xx = X + (long long)x * P * P;
#pragma unroll
    for (int u = 0; u < TQ_SPF; ++u) {
      const int e = threadIdx.x + u * TQ_THREADS;
      int r, c;
      fast_divmod(min(e, PR * QB - 1), QB, rqb, r, c);
      const bool ok = e < PR * QB && c < qn;
      const double v = Xx[(prow + r) * P + q0 + min(c, qn - 1)];
      pf[u] = ok ? v : 0.0;
    }
  };
  fetch(0);
  int yi = 0;
  for (int x = 0; x < a.nx; ++x) {
    const int md = (2 - a.tabs->x_fam[x]) - a.tabs->x_deg[x];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TQ_SPF; ++u) {
      const int e = threadIdx.x + u * TQ_THREADS;
      if (e < PR * QB) L0[e] = pf[u];
    }
    __syncthreads();
    if (x + 1 < a.nx) fetch(x + 1);
    // element (r, c) of the block -> Y offset (prow + r) * P + q0 + c
    auto gidx = [&](long long i) { return (prow + i / QB) * P + q0 + (i % QB); };
    if constexpr (d == 2) {
      const int nj = md + 1;
      pass_axis<1>(bk, tap_ptr(a, jb, 1), jb.R[1], 0, nj, [&](long long i) { return L0[i]; },
          [&](int j, long long i, double v) { Y[(long long)(yi + j) * P * P + gidx(i)] = v; });
      yi += nj;
    } else {
      for (int ec = 0; ec <= md; ++ec) {
        pass_axis<1>(bk, tap_ptr(a, jb, 2), jb.R[2], ec, 1, [&](long long i) { return L0[i]; },
            [&](int, long long i, double v) { L1[i] = v; });
        __syncthreads();
        const int nj = md - ec + 1;
        pass_axis<0>(bk, tap_ptr(a, jb, 1), jb.R[1], 0, nj, [&](long long i) { return L1[i]; },
            [&](int j, long long i, double v) { Y[(long long)(yi + j) * P * P + gidx(i)] = v; });
        yi += nj;
        __syncthreads();
      }
    }
  }
}

// ------------------------------------------------------------------ stage W
template <typename T, int d>
__device__ void stage_w(const TArgs &a, const TJob &jb, int task, LDbl *lds) {
  constexpr int D = 2 * d;
  constexpr int NM = 1 + D + D * (D + 1) / 2 + 1 + D;
  const int QB = a.qb;
  const long long P = jb.P;
  const int M1 = jb.M[0];
  const int PR = jb.P / M1;
  const int nqb = (jb.P + QB - 1) / QB;
  const int npb = (PR + jb.pb - 1) / jb.pb;
  const int pbi = task / nqb, q0 = (task % nqb) * QB;
  const int qn = min(QB, jb.P - q0);
  LDbl *F = lds;                           // [NM][M1][QB] final moments
  LDbl *Ys = F + (long long)NM * M1 * QB;  // [ny][M1][QB] the position's pencils
  const double *Y = (d == 1) ? slot_x(a, jb.slot) : slot_y(a, jb.slot);
  const int ny = (d == 1) ? a.nx : a.ny;
  const int W = 2 * jb.R[0] + 1;
  const int R = jb.R[0];
  CDbl *tp = tap_ptr(a, jb, 0);
  const float rqb = 1.0f / float(QB);
  const int r_end = min(PR, (pbi + 1) * jb.pb);
  (void)npb;
  const int pen = M1 * QB;
  // Cross-validation scores only need nodes p <= q, so s_1 <= t_1 <= n_out - 1
  // (the last t_1 of the column block): the s_1 pass forms outputs below
  // n_out from input rows below n_in (beyond them the line is read as zero,
  // which those outputs never reach); smoothing needs every node.
  const int n_out = a.cv ? min(M1, (q0 + qn - 1) / PR + 1) : M1;
  const int n_in = min(M1, n_out + R);
  const int pen_in = n_in * QB;
  const float rpen_in = 1.0f / float(pen_in);
  const int nseg_out = (n_out + TQ_SEG - 1) / TQ_SEG;
  const int per_out = QB * nseg_out;
  const float rper_out = 1.0f / float(per_out);
  for (int r = pbi * jb.pb; r < r_end; ++r) {
    __syncthreads();
    // stage the pencils (input rows below n_in) of every Y array at
    // s-position (., r), all loads in flight
    stage_to_lds(Ys, ny * pen_in, [&](int e) {
      int y, rem, a1, c;
      fast_divmod(e, pen_in, rpen_in, y, rem);
      fast_divmod(rem, QB, rqb, a1, c);
      return c < qn ? Y[(long long)y * P * P + ((long long)a1 * PR + r) * P + q0 + c] : 0.0;
    }, [&](int e) {
      int y, rem;
      fast_divmod(e, pen_in, rpen_in, y, rem);
      return y * pen + rem;
    });
    __syncthreads();
    // s_1 pass of every Y array at s-position (., r), columns q0..q0+qn
    for (int it = threadIdx.x; it < ny * per_out; it += TQ_THREADS) {
      int y, rem, sg, c;
      fast_divmod(it, per_out, rper_out, y, rem);
      fast_divmod(rem, QB, rqb, sg, c);
      const int fam = (d == 1) ? a.tabs->x_fam[y] : a.tabs->y_fam[y];
      const int deg = (d == 1) ? a.tabs->x_deg[y] : a.tabs->y_deg[y];
      const int nj = (2 - fam) - deg + 1;
      const LDbl *src = Ys + (long long)y * pen + c;
      const int sx = QB;
      const int x0 = sg * TQ_SEG;
      double acc[3][TQ_SEG];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < TQ_SEG; ++q) acc[j][q] = 0.0;
      window_acc([&](int xc) { return src[xc * sx]; }, x0, n_in, R, tp, tp + W, tp + 2 * W, nj, acc);
#pragma unroll
      for (int q = 0; q < TQ_SEG; ++q) {
        const int xo = x0 + q;
        if (xo < n_out) {
#pragma unroll
          for (int j = 0; j < 3; ++j)
            if (j < nj) F[((long long)a.tabs->y_mom[y][j] * M1 + xo) * QB + c] = acc[j][q];
        }
      }
    }
    __syncthreads();
    // one lane per node (a1, c): the FP64 solve
    for (int e = threadIdx.x; e < n_out * QB; e += TQ_THREADS) {
      const int a1 = e / QB, c = e % QB;
      if (c >= qn) continue;
      double m[NM];
#pragma unroll
      for (int i = 0; i < NM; ++i) m[i] = F[((long long)i * M1 + a1) * QB + c];
      int8_t st;
      const long long o = ((long long)a1 * PR + r) * P + q0 + c;
      if (jb.loo) {
        // the node's own bin: u = 0 there, so it enters S0 and T0 only
        const T *Ca = static_cast<const T *>(jb.Ca), *Cb = static_cast<const T *>(jb.Cb);
        const T *Ga = static_cast<const T *>(jb.Ga), *Gb = static_cast<const T *>(jb.Gb);
        const double cw = Ca ? double(Ca[o]) - (Cb ? double(Cb[o]) : 0.0)
                             : (a1 * PR + r == q0 + c ? 0.0 : jb.c0);
        const double gw = double(Ga[o]) - (Gb ? double(Gb[o]) : 0.0);
        m[0] -= cw;
        m[1 + D + D * (D + 1) / 2] -= gw;
      }
      const double b0 = wls_b0<D>(m, &st);
      if (a.cv) {
        static_cast<T *>(slot_g(a, jb.slot))[o] = T(b0);
      } else {
        static_cast<T *>(jb.out)[o] = T(b0);
        if (jb.status) jb.status[o] = st;
      }
    }
  }
}

// ------------------------------------------------------------------ score
// Tile pairs (I, J), I <= J, of the P x P grid in TQ_TILE x TQ_TILE tiles.
// Stage W solved the nodes p <= q only (C and G are symmetric, so the fit at
// (q, p) is the fit at (p, q) up to rounding): g(p, q) = b0(min, max), read
// from tile (I, J) alone (for leave-one-out jobs too: the node's own bin is
// the same at both), 0 outside the mask and where b0 is NaN (an empty window).
template <typename T>
__device__ void stage_score(const TArgs &a, const TJob &jb, int job, int task, LDbl *lds) {
  const int P = jb.P;
  const int nt = (P + TQ_TILE - 1) / TQ_TILE;
  LDbl *A = lds;                            // [TQ_TILE][TQ_TILE+1]: b0 of tile (I, J)
  LDbl *red = A + TQ_TILE * (TQ_TILE + 1);  // [TQ_THREADS / 64] wave sums
  const T *Gh = static_cast<const T *>(slot_g(a, jb.slot));
  const T *Q = static_cast<const T *>(jb.Qf);
  const T *G = static_cast<const T *>(jb.Gf);
  const T *C = static_cast<const T *>(jb.Cf);
  const uint8_t *mask = jb.mask;
  double s = 0.0;
  const int npairs = nt * (nt + 1) / 2;
  for (int t = task * jb.tpt; t < min(npairs, (task + 1) * jb.tpt); ++t) {
    int id = t, I = 0;
    while (id >= nt - I) {
      id -= nt - I;
      ++I;
    }
    const int J = I + id;
    const int r0 = I * TQ_TILE, c0 = J * TQ_TILE;
    constexpr int EPT = TQ_TILE * TQ_TILE / TQ_THREADS;  // elements of a tile per thread
    static_assert(EPT * TQ_THREADS == TQ_TILE * TQ_TILE, "tile must split evenly over the workgroup");
    // every read of this tile pair is issued before any of them is used
    double va[EPT], q1[EPT], g1[EPT], w1[EPT], q2[EPT], g2[EPT], w2[EPT];
    bool in1[EPT], in2[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * TQ_THREADS;
      const int rr = e / TQ_TILE, cc = e % TQ_TILE;
      const bool ia = r0 + rr < P && c0 + cc < P, ib = c0 + rr < P && r0 + cc < P;
      va[u] = ia ? double(Gh[(long long)(r0 + rr) * P + c0 + cc]) : 0.0;
      // held-out arrays at (p, q) = (r0 + rr, c0 + cc) and at the mirror (c0 + rr, r0 + cc)
      in1[u] = ia;
      const long long o1 = (long long)(r0 + rr) * P + c0 + cc;
      q1[u] = ia ? double(Q[o1]) : 0.0;
      g1[u] = ia ? double(G[o1]) : 0.0;
      w1[u] = ia ? double(C[o1]) : 0.0;
      in2[u] = ib && I != J;
      const long long o2 = (long long)(c0 + rr) * P + r0 + cc;
      q2[u] = in2[u] ? double(Q[o2]) : 0.0;
      g2[u] = in2[u] ? double(G[o2]) : 0.0;
      w2[u] = in2[u] ? double(C[o2]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * TQ_THREADS;
      A[(e / TQ_TILE) * (TQ_TILE + 1) + e % TQ_TILE] = va[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = threadIdx.x + u * TQ_THREADS;
      const int rr = e / TQ_TILE, cc = e % TQ_TILE;
      // (p, q) in tile (I, J): p < q off the diagonal tile; on it the smaller
      // index's row holds the solved node
      if (in1[u]) {
        const int p = r0 + rr, q = c0 + cc;
        double g = (I != J || rr <= cc) ? A[rr * (TQ_TILE + 1) + cc] : A[cc * (TQ_TILE + 1) + rr];
        if (mask && (!mask[p] || !mask[q])) g = 0.0;
        if (g != g) g = 0.0;
        s += q1[u] - 2.0 * g1[u] * g + w1[u] * g * g;
      }
      // (q, p) = (c0 + rr, r0 + cc) in tile (J, I), I < J: the node (r0 + cc, c0 + rr) of tile (I, J)
      if (in2[u]) {
        const int q = c0 + rr, p = r0 + cc;
        double g = A[cc * (TQ_TILE + 1) + rr];
        if (mask && (!mask[p] || !mask[q])) g = 0.0;
        if (g != g) g = 0.0;
        s += q2[u] - 2.0 * g2[u] * g + w2[u] * g * g;
      }
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < TQ_THREADS / 64; ++w) tot += red[w];
    a.part[(long long)job * a.part_stride + task] = tot;
  }
}

// ------------------------------------------------------------------ kernel
template <typename T, int d>
__global__ __launch_bounds__(TQ_THREADS) void k_tiled(TArgs a) {
  extern __shared__ double lds_raw[];
  LDbl *lds = (LDbl *)lds_raw;
  __shared__ long long s_task;
  __shared__ int s_ok;
  int cur = 0;
  // Tasks are taken a.chunk at a time (one atomic on the queue counter) and
  // run in order; completions of consecutive tasks of one segment are
  // published together, before the workgroup moves to another segment or
  // takes a new chunk. Nothing waits on a task of its own segment, so the
  // earliest unpublished task always gets published: its workgroup has
  // finished every earlier task of its chunk, and that task's dependencies
  // lie earlier in the queue.
  long long g = 0, gend = 0;
  int pend = 0, pend_job = 0, pend_stage = 0;  // completions not yet counted
  auto publish = [&]() {
    if (pend == 0) return;
    // every lane's stores are released before the count moves
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(a.done + pend_job * TQ_NSTAGE + pend_stage, pend, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    pend = 0;
  };
  for (;;) {
    if (g >= gend) {
      publish();
      if (threadIdx.x == 0)
        s_task = __hip_atomic_fetch_add(a.qctr, a.chunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      // the task index, and all that follows from it, is uniform: keep it in SGPRs
      g = ((long long)__builtin_amdgcn_readfirstlane(int(s_task >> 32)) << 32) |
          (unsigned int)__builtin_amdgcn_readfirstlane(int(s_task & 0xffffffff));
      gend = g + a.chunk;
      __syncthreads();
    }
    if (g >= a.total) break;
    while (cur + 1 < a.nseg && a.segs[cur + 1].start <= g) ++cur;
    const TSeg sg = a.segs[cur];
    const int job = sg.job, stage = sg.stage;
    const int task = int(g - sg.start);
    if (pend > 0 && (job != pend_job || stage != pend_stage)) publish();
    const TJob jb = a.jobs[job];
    // dependencies: earlier tasks of the queue only
    if (threadIdx.x == 0) {
      bool ok = true;
      const int pv = jb.prev;
      const int *dn = a.done;
      if (stage == TQ_T) {
        if (pv >= 0) ok = wait_done(dn + pv * TQ_NSTAGE + (d == 1 ? TQ_W : TQ_S), a.jobs[pv].ntask[d == 1 ? TQ_W : TQ_S],
                                    a.spin_limit, a.err);
      } else if (stage == TQ_S) {
        ok = wait_done(dn + job * TQ_NSTAGE + TQ_T, a.jobs[job].ntask[TQ_T], a.spin_limit, a.err);
        if (ok && pv >= 0) ok = wait_done(dn + pv * TQ_NSTAGE + TQ_W, a.jobs[pv].ntask[TQ_W], a.spin_limit, a.err);
      } else if (stage == TQ_W) {
        const int prev_stage = d == 1 ? TQ_T : TQ_S;
        ok = wait_done(dn + job * TQ_NSTAGE + prev_stage, a.jobs[job].ntask[prev_stage], a.spin_limit, a.err);
        if (ok && a.cv && pv >= 0) ok = wait_done(dn + pv * TQ_NSTAGE + TQ_SC, a.jobs[pv].ntask[TQ_SC], a.spin_limit, a.err);
      } else if (stage == TQ_SC) {
        ok = wait_done(dn + job * TQ_NSTAGE + TQ_W, a.jobs[job].ntask[TQ_W], a.spin_limit, a.err);
      } else {
        ok = wait_done(dn + job * TQ_NSTAGE + TQ_SC, a.jobs[job].ntask[TQ_SC], a.spin_limit, a.err);
      }
      s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    if (s_ok) {
      if (stage == TQ_T) {
        stage_t<T, d>(a, jb, task, lds);
      } else if (stage == TQ_S) {
        if constexpr (d > 1) stage_s<d>(a, jb, task, lds);
      } else if (stage == TQ_W) {
        stage_w<T, d>(a, jb, task, lds);
      } else if (stage == TQ_SC) {
        stage_score<T>(a, jb, job, task, lds);
      } else {
        // fixed order: thread t sums partials t, t + TQ_THREADS, ...; then a fixed tree
        LDbl *fin = lds;  // TQ_THREADS partial sums
        double s = 0.0;
        const int ns = a.jobs[job].ntask[TQ_SC];
        for (int i = threadIdx.x; i < ns; i += TQ_THREADS) s += a.part[(long long)job * a.part_stride + i];
        fin[threadIdx.x] = s;
        __syncthreads();
        for (int w = TQ_THREADS / 2; w > 0; w >>= 1) {
          if (threadIdx.x < w) fin[threadIdx.x] += fin[threadIdx.x + w];
          __syncthreads();
        }
        if (threadIdx.x == 0) a.scores[job] = fin[0];
      }
    }
    pend_job = job;
    pend_stage = stage;
    ++pend;
    ++g;
    __syncthreads();  // the task's LDS and s_ok are free for the next one
  }
  publish();
}

// ------------------------------------------------------------------ host
struct Tables {
  int d = 0, nx = 0, ny = 0;
  signed char x_fam[TQ_MAXX], x_deg[TQ_MAXX];
  signed char y_fam[TQ_MAXY], y_deg[TQ_MAXY];
  signed char y_mom[TQ_MAXY][3];
};

// Moment index in the order S0, S1[D], S2 (upper triangle by rows), T0, T1[D]
// of the exponent vector e over the D = 2d coordinates (s_1..s_d, t_1..t_d).
int moment_index(int D, int fam, const int *e) {
  int deg = 0, c1 = -1, c2 = -1;
  for (int k = 0; k < D; ++k)
    for (int r = 0; r < e[k]; ++r) {
      if (c1 < 0)
        c1 = k;
      else
        c2 = k;
      ++deg;
    }
  const int NC = 1 + D + D * (D + 1) / 2;
  if (fam == 1) return deg == 0 ? NC : NC + 1 + c1;
  if (deg == 0) return 0;
  if (deg == 1) return 1 + c1;
  int idx = 1 + D;
  for (int r = 0; r < c1; ++r) idx += D - r;
  return idx + (c2 - c1);
}

Tables make_tables(int d) {
  Tables tb;
  tb.d = d;
  const int D = 2 * d;
  // X: fam, then t-exponents from the last coordinate (outermost) to the first
  struct XE {
    int fam, et[3];
  };
  std::vector<XE> xs;
  for (int fam = 0; fam < 2; ++fam) {
    const int md = 2 - fam;
    if (d == 1) {
      for (int e1 = 0; e1 <= md; ++e1) xs.push_back({fam, {e1, 0, 0}});
    } else if (d == 2) {
      for (int e2 = 0; e2 <= md; ++e2)
        for (int e1 = 0; e1 <= md - e2; ++e1) xs.push_back({fam, {e1, e2, 0}});
    } else {
      for (int e3 = 0; e3 <= md; ++e3)
        for (int e2 = 0; e2 <= md - e3; ++e2)
          for (int e1 = 0; e1 <= md - e3 - e2; ++e1) xs.push_back({fam, {e1, e2, e3}});
    }
  }
  tb.nx = int(xs.size());
  for (int i = 0; i < tb.nx; ++i) {
    tb.x_fam[i] = (signed char)xs[i].fam;
    tb.x_deg[i] = (signed char)(xs[i].et[0] + xs[i].et[1] + xs[i].et[2]);
  }
  // Y: for each X, s-exponents from s_d (outermost) down to s_2
  struct YE {
    int fam, es[3], et[3];
  };
  std::vector<YE> ys;
  for (const XE &x : xs) {
    const int md = (2 - x.fam) - (x.et[0] + x.et[1] + x.et[2]);
    if (d == 1) {
      ys.push_back({x.fam, {0, 0, 0}, {x.et[0], x.et[1], x.et[2]}});
    } else if (d == 2) {
      for (int a2 = 0; a2 <= md; ++a2) ys.push_back({x.fam, {0, a2, 0}, {x.et[0], x.et[1], x.et[2]}});
    } else {
      for (int a3 = 0; a3 <= md; ++a3)
        for (int a2 = 0; a2 <= md - a3; ++a2) ys.push_back({x.fam, {0, a2, a3}, {x.et[0], x.et[1], x.et[2]}});
    }
  }
  tb.ny = int(ys.size());
  for (int i = 0; i < tb.ny; ++i) {
    const YE &y = ys[i];
    const int deg = y.es[1] + y.es[2] + y.et[0] + y.et[1] + y.et[2];
    tb.y_fam[i] = (signed char)y.fam;
    tb.y_deg[i] = (signed char)deg;
    for (int a1 = 0; a1 < 3; ++a1) {
      if (a1 > (2 - y.fam) - deg) {
        tb.y_mom[i][a1] = -1;
        continue;
      }
      int e[6] = {0, 0, 0, 0, 0, 0};
      e[0] = a1;
      for (int k = 1; k < d; ++k) e[k] = y.es[k];
      for (int k = 0; k < d; ++k) e[d + k] = y.et[k];
      tb.y_mom[i][a1] = (signed char)moment_index(D, y.fam, e);
    }
  }
  return tb;
}

}  // namespace

bool tiled_supported(const fpca_grid *g) {
  const int d = g->d;
  int64_t P = 1;
  for (int k = 0; k < d; ++k) P *= g->M[k];
  if (P > 4096) return false;
  if (d == 1) return g->M[0] <= 64;
  if (d == 2) return g->M[0] <= 32 && g->M[1] <= 64;
  return g->M[0] <= 16 && g->M[1] <= 16 && g->M[2] <= 16;
}

namespace {

int tap_radius_t(double h, int M) {
  int R = int(std::floor(h * double(M - 1)));
  return std::min(R, M - 1);
}

size_t lds_bytes(int d, int Pmax, int M1max, int PRmax, int qb) {
  const int D = 2 * d;
  const int NM = 1 + D + D * (D + 1) / 2 + 1 + D;
  const int NY = d == 3 ? 27 : (d == 2 ? 14 : 5);
  size_t t = size_t(d + 0) * size_t(Pmax);  // L0 (+ L1, L2)
  size_t s = (d == 3 ? 2 : (d == 2 ? 1 : 0)) * size_t(PRmax) * qb;
  size_t w = size_t(NM + NY) * M1max * qb;
  size_t sc = TQ_TILE * (TQ_TILE + 1) + TQ_THREADS;
  return 8 * std::max(std::max(t, s), std::max(w, sc));
}

template <typename T, int d>
int launch_tiled(fpca_context *ctx, const TArgs &args, size_t lds, int grid) {
  static bool attr = false;  // set once, outside any stream capture
  if (!attr) {
    FPCA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tiled<T, d>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, int(TQ_LDS_MAX)));
    attr = true;
  }
  hipLaunchKernelGGL((k_tiled<T, d>), dim3(grid), dim3(TQ_THREADS), lds, ctx->stream, args);
  FPCA_LAUNCH_CHECK("tiled");
  return FPCA_OK;
}

__global__ void k_zero_i32(int *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace

// Plans one persistent launch over `jobs` (same d; grids may differ in
// size): carves the intermediate slots from the handle's arena (ws) and the
// queue tables from ws3, and uploads the job and segment tables on the
// handle's stream. tiled_queue then zeroes the counters and launches; the
// two are split so that a caller can capture the launch into a graph while
// the tables (which hold the callers' pointers) are uploaded outside it.
template <typename T>
int tiled_plan(fpca_context *ctx, const std::vector<TiledJob> &jobs, bool cv, const TiledConfig &cfg,
               TiledLaunch *L) {
  const int d = jobs[0].grid->d;
  const int J = int(jobs.size());
  const Tables tb = make_tables(d);
  const int NS = std::min(J, TQ_MAXSLOT);
  const int qb = cfg.qb;
  int Pmax = 0, M1max = 0, PRmax = 0, Mmax[3] = {1, 1, 1};
  std::vector<TJob> hj(J);
  for (int j = 0; j < J; ++j) {
    const fpca_grid *g = jobs[j].grid;
    if (g->d != d) return set_error(FPCA_ERR_INVALID_ARG, "every dataset needs the same d");
    TJob &t = hj[j];
    std::memset(&t, 0, sizeof(t));
    t.Ca = jobs[j].Ca;
    t.Cb = jobs[j].Cb;
    t.Ga = jobs[j].Ga;
    t.Gb = jobs[j].Gb;
    t.Qf = jobs[j].Qf;
    t.Gf = jobs[j].Gf;
    t.Cf = jobs[j].Cf;
    t.mask = g->mask;
    t.c0 = jobs[j].c0;
    t.loo = jobs[j].loo;
    t.out = jobs[j].out;
    t.status = jobs[j].status;
    int P = 1;
    for (int k = 0; k < 3; ++k) {
      t.M[k] = k < d ? g->M[k] : 1;
      t.h[k] = k < d ? jobs[j].h[k] : 1.0;
      t.R[k] = k < d ? tap_radius_t(jobs[j].h[k], g->M[k]) : 0;
      P *= t.M[k];
      Mmax[k] = std::max(Mmax[k], t.M[k]);
    }
    t.P = P;
    t.slot = j % NS;
    t.prev = j >= NS ? j - NS : -1;
    const int PR = P / t.M[0];
    if (int64_t(PR) * qb > int64_t(TQ_SPF) * TQ_THREADS)
      return set_error(FPCA_ERR_UNSUPPORTED, "tiled smoother: %d s-positions x %d columns per stage-S block", PR, qb);
    const int nqb = (P + qb - 1) / qb;
    t.pb = std::max(1, (2048 + t.M[0] * qb - 1) / (t.M[0] * qb));
    t.pb = std::min(t.pb, PR);
    const int nt = (P + TQ_TILE - 1) / TQ_TILE;
    const int npairs = nt * (nt + 1) / 2;
    t.tpt = std::max(1, npairs / 1024);
    t.ntask[TQ_T] = P;
    t.ntask[TQ_S] = d == 1 ? 0 : t.M[0] * nqb;
    t.ntask[TQ_W] = ((PR + t.pb - 1) / t.pb) * nqb;
    t.ntask[TQ_SC] = cv ? (npairs + t.tpt - 1) / t.tpt : 0;
    t.ntask[TQ_FIN] = cv ? 1 : 0;
    Pmax = std::max(Pmax, P);
    M1max = std::max(M1max, t.M[0]);
    PRmax = std::max(PRmax, PR);
  }
  // tap table: per job and coordinate k, (1-u^2) u^e at m = -R..R, u = m / (h (M-1))
  std::vector<double> tapv;
  for (int j = 0; j < J; ++j)
    for (int k = 0; k < d; ++k) {
      TJob &t = hj[j];
      t.tap_off[k] = int(tapv.size());
      const int R = t.R[k];
      for (int e = 0; e < 3; ++e)
        for (int m = -R; m <= R; ++m) {
          const double u = double(m) / (t.h[k] * double(t.M[k] - 1));
          const double K = std::fabs(u) < 1.0 ? 1.0 - u * u : 0.0;
          tapv.push_back(K * (e == 0 ? 1.0 : (e == 1 ? u : u * u)));
        }
    }
  const size_t lds = lds_bytes(d, Pmax, M1max, PRmax, qb);
  if (lds > TQ_LDS_MAX) return set_error(FPCA_ERR_UNSUPPORTED, "tiled smoother: %zu bytes of LDS", lds);
  // queue: round r holds stage s of job r - s
  std::vector<TSeg> segs;
  long long total = 0;
  for (int r = 0; r < J + TQ_NSTAGE - 1; ++r)
    for (int s = 0; s < TQ_NSTAGE; ++s) {
      const int j = r - s;
      if (j < 0 || j >= J || hj[j].ntask[s] == 0) continue;
      segs.push_back(TSeg{total, j, s});
      total += hj[j].ntask[s];
    }
  const int nx = tb.nx, ny = d == 1 ? tb.nx : tb.ny;
  const size_t PPmax = size_t(Pmax) * Pmax;
  int part_stride = 1;
  for (int j = 0; j < J; ++j) part_stride = std::max(part_stride, hj[j].ntask[TQ_SC]);
  const size_t bx = carve_bytes(size_t(nx) * PPmax, 8);
  const size_t by = d == 1 ? 0 : carve_bytes(size_t(ny) * PPmax, 8);
  const size_t bg = cv ? carve_bytes(PPmax, sizeof(T)) : 0;
  if (int rc = ws_reserve(ctx, NS * (bx + by + bg))) return rc;
  const size_t nzero = size_t(J) * TQ_NSTAGE + 1;
  const size_t small = carve_bytes(J, sizeof(TJob)) + carve_bytes(segs.size(), sizeof(TSeg)) +
                       carve_bytes(tapv.size(), sizeof(double)) + carve_bytes(1, sizeof(TTables)) +
                       carve_bytes(nzero, 4) + carve_bytes(size_t(J) * part_stride, 8) + carve_bytes(J, 8);
  if (int rc = ws3_reserve(ctx, small)) return rc;
  Carver cw{static_cast<char *>(ctx->ws), 0, ctx->ws_size};
  Carver c3{static_cast<char *>(ctx->ws3), 0, ctx->ws3_size};
  TArgs &a = L->args;
  std::memset(&a, 0, sizeof(a));
  for (int s = 0; s < NS; ++s) {
    a.X[s] = cw.take<double>(size_t(nx) * PPmax);
    a.Y[s] = d == 1 ? nullptr : cw.take<double>(size_t(ny) * PPmax);
    a.Gh[s] = cv ? static_cast<void *>(cw.take<T>(PPmax)) : nullptr;
  }
  TJob *d_jobs = c3.take<TJob>(J);
  TSeg *d_segs = c3.take<TSeg>(segs.size());
  double *d_taps = c3.take<double>(tapv.size());
  TTables *d_tabs = c3.take<TTables>(1);
  int *zero = c3.take<int>(nzero);
  a.part = c3.take<double>(size_t(J) * part_stride);
  a.scores = c3.take<double>(J);
  a.jobs = d_jobs;
  a.segs = d_segs;
  a.nseg = int(segs.size());
  a.total = total;
  a.done = zero;
  a.qctr = zero + size_t(J) * TQ_NSTAGE;
  a.err = ctx->d_flags;
  a.part_stride = part_stride;
  a.cv = cv ? 1 : 0;
  a.qb = qb;
  a.taps = d_taps;
  a.spin_limit = 1LL << 20;
  a.nx = tb.nx;
  a.ny = tb.ny;
  TTables tt;
  std::memcpy(tt.x_fam, tb.x_fam, sizeof(tt.x_fam));
  std::memcpy(tt.x_deg, tb.x_deg, sizeof(tt.x_deg));
  std::memcpy(tt.y_fam, tb.y_fam, sizeof(tt.y_fam));
  std::memcpy(tt.y_deg, tb.y_deg, sizeof(tt.y_deg));
  std::memcpy(tt.y_mom, tb.y_mom, sizeof(tt.y_mom));
  if (d == 1)
    for (int i = 0; i < tb.nx; ++i) {  // stage W reads X directly
      tt.y_fam[i] = tb.x_fam[i];
      tt.y_deg[i] = tb.x_deg[i];
    }
  a.tabs = d_tabs;
  const size_t b1 = sizeof(TJob) * J, b2 = sizeof(TSeg) * segs.size(), b3 = sizeof(double) * tapv.size(),
               b4 = sizeof(TTables);
  char *hs = nullptr;
  if (int rc = tables_stage(ctx, b1 + b2 + b3 + b4, &hs)) return rc;
  std::memcpy(hs, hj.data(), b1);
  std::memcpy(hs + b1, segs.data(), b2);
  std::memcpy(hs + b1 + b2, tapv.data(), b3);
  std::memcpy(hs + b1 + b2 + b3, &tt, b4);
  FPCA_HIP(hipMemcpyAsync(d_jobs, hs, b1, hipMemcpyHostToDevice, ctx->stream));
  FPCA_HIP(hipMemcpyAsync(d_segs, hs + b1, b2, hipMemcpyHostToDevice, ctx->stream));
  FPCA_HIP(hipMemcpyAsync(d_taps, hs + b1 + b2, b3, hipMemcpyHostToDevice, ctx->stream));
  FPCA_HIP(hipMemcpyAsync(d_tabs, hs + b1 + b2 + b3, b4, hipMemcpyHostToDevice, ctx->stream));
  FPCA_HIP(hipEventRecord(ctx->ev_tables, ctx->stream));
  L->lds = lds;
  L->grid = std::max(1, ctx->num_cus * cfg.wg_per_cu);
  // tasks per queue atomic: about a segment's share per workgroup, at most
  // TQ_CHUNK_MAX (d = 3, 16^6 nodes, 80 jobs: 628 / 552 / 520 / 508 ms at
  // 2 / 4 / 8 / 16)
  a.chunk = int(std::max<long long>(1, std::min<long long>(TQ_CHUNK_MAX, total / (int64_t(segs.size()) * L->grid))));
  L->d = d;
  L->f64 = sizeof(T) == 8;
  L->zero = zero;
  L->nzero = int(nzero);
  L->njobs = J;
  return FPCA_OK;
}

int tiled_queue(fpca_context *ctx, const TiledLaunch &L) {
  hipLaunchKernelGGL(k_zero_i32, dim3(unsigned((L.nzero + 255) / 256)), dim3(256), 0, ctx->stream, L.zero, L.nzero);
  FPCA_LAUNCH_CHECK("zero counters");
  if (L.f64) {
    switch (L.d) {
      case 1: return launch_tiled<double, 1>(ctx, L.args, L.lds, L.grid);
      case 2: return launch_tiled<double, 2>(ctx, L.args, L.lds, L.grid);
      case 3: return launch_tiled<double, 3>(ctx, L.args, L.lds, L.grid);
    }
  } else {
    switch (L.d) {
      case 1: return launch_tiled<float, 1>(ctx, L.args, L.lds, L.grid);
      case 2: return launch_tiled<float, 2>(ctx, L.args, L.lds, L.grid);
      case 3: return launch_tiled<float, 3>(ctx, L.args, L.lds, L.grid);
    }
  }
  return set_error(FPCA_ERR_UNSUPPORTED, "d=%d", L.d);
}

// LDS a configuration needs for these grids (0 if it does not fit).
size_t tiled_lds(const std::vector<TiledJob> &jobs, int qb) {
  const int d = jobs[0].grid->d;
  int Pmax = 0, M1max = 0, PRmax = 0, Mmax[3] = {1, 1, 1};
  for (const TiledJob &j : jobs) {
    int P = 1;
    for (int k = 0; k < d; ++k) {
      P *= j.grid->M[k];
      Mmax[k] = std::max(Mmax[k], j.grid->M[k]);
    }
    Pmax = std::max(Pmax, P);
    M1max = std::max(M1max, j.grid->M[0]);
    PRmax = std::max(PRmax, P / j.grid->M[0]);
  }
  const size_t lds = lds_bytes(d, Pmax, M1max, PRmax, qb);
  return lds > TQ_LDS_MAX ? 0 : lds;
}

const void *tiled_scores(const TiledLaunch &L) { return L.args.scores; }

template int tiled_plan<float>(fpca_context *, const std::vector<TiledJob> &, bool, const TiledConfig &,
                               TiledLaunch *);
template int tiled_plan<double>(fpca_context *, const std::vector<TiledJob> &, bool, const TiledConfig &,
                                TiledLaunch *);

}  // namespace fpca

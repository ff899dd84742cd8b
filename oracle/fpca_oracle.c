/*
 * FP64 CPU oracle for the binned local-linear FPCA hot path
 * (Chen & Jiang, "Multi-dimensional Functional Principal Component Analysis").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * HIP library is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or constant with the GPU library.
 *
 * Conventions
 *  - Grid: M_k nodes per coordinate at m/(M_k-1); flat index with the last
 *    coordinate fastest. A covariance array is the 2d-dimensional array with
 *    dims (M_1..M_d, M_1..M_d): flat index p*P + q, p the s-node, q the t-node.
 *  - Everything is IEEE binary64, compiled without FP contraction.
 *
 * Parity pins (checked by the CPU test suite, not by re-typing formulas):
 *  mass / first-moment preservation of linear binning, the pair-loop versus
 *  Gram-identity agreement, exact reproduction of linear surfaces, brute-force
 *  least squares on raw observations, symmetry, closed-form eigenpairs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_DOMAIN (-2)

#define ST_OK 0
#define ST_FALLBACK 1
#define ST_EMPTY 2

#define MAXD 3
#define MAXDD 6

/* Linear binning of one coordinate (the binning strategy of Section 3.2):
 * u = x*(M-1) as one FP64 multiply, lower node k = min(floor(u), M-2),
 * fraction rho = u - k; weights 1-rho on node k and rho on node k+1. */
static int bin_coord(double x, int M, int *k, double *rho) {
  if (!(x >= 0.0 && x <= 1.0)) return ORC_ERR_DOMAIN;
  double u = x * (double)(M - 1);
  int kk = (int)floor(u);
  if (kk > M - 2) kk = M - 2;
  *k = kk;
  *rho = u - (double)kk;
  return ORC_OK;
}

/* The 2^d nodes that observation point x spreads onto, with their weights,
 * and the flat index of the lower corner. */
static int corners(int d, const int *M, const double *x, int64_t *node, double *wt,
                   int64_t *lower) {
  int k[MAXD];
  double rho[MAXD];
  for (int c = 0; c < d; ++c) {
    int rc = bin_coord(x[c], M[c], &k[c], &rho[c]);
    if (rc) return rc;
  }
  int64_t lo = 0;
  for (int c = 0; c < d; ++c) lo = lo * M[c] + k[c];
  *lower = lo;
  for (int b = 0; b < (1 << d); ++b) {
    int64_t p = 0;
    double w = 1.0;
    for (int c = 0; c < d; ++c) {
      int bit = (b >> (d - 1 - c)) & 1;
      p = p * M[c] + (k[c] + bit);
      w *= bit ? rho[c] : (1.0 - rho[c]);
    }
    node[b] = p;
    wt[b] = w;
  }
  return ORC_OK;
}

static int64_t grid_size(int d, const int *M) {
  int64_t P = 1;
  for (int c = 0; c < d; ++c) P *= M[c];
  return P;
}

static int check_grid(int d, const int *M) {
  if (d < 1 || d > MAXD) return ORC_ERR_ARG;
  for (int c = 0; c < d; ++c)
    if (M[c] < 2) return ORC_ERR_ARG;
  return ORC_OK;
}

/* Corner indices and weights of every observation: node[N*2^d], wt[N*2^d], lower[N]. */
int orc_bin_corners(int d, const int *M, int64_t N, const double *t, int64_t *node,
                    double *wt, int64_t *lower) {
  if (check_grid(d, M)) return ORC_ERR_ARG;
  int nc = 1 << d;
  for (int64_t j = 0; j < N; ++j) {
    int rc = corners(d, M, t + j * d, node + j * nc, wt + j * nc, lower + j);
    if (rc) return rc;
  }
  return ORC_OK;
}

/* Mean binning (eq. 2.3 with weights 1/N_i, binned as in Section 3.2):
 *   c[p] = sum_i (1/N_i) sum_j W_p(t_ij),  s[p] = sum_i (1/N_i) sum_j W_p(t_ij) Y_ij,
 *   idx[j] = flat lower corner of t_ij,    cnt[p] = #observations with lower corner p. */
int orc_bin_mean(int d, const int *M, int64_t n, const int64_t *offsets, const double *t,
                 const double *y, double *c, double *s, int32_t *idx, int64_t *cnt) {
  if (check_grid(d, M) || n < 0) return ORC_ERR_ARG;
  int64_t P = grid_size(d, M);
  memset(c, 0, sizeof(double) * P);
  memset(s, 0, sizeof(double) * P);
  if (cnt) memset(cnt, 0, sizeof(int64_t) * P);
  int64_t node[1 << MAXD];
  double wt[1 << MAXD];
  for (int64_t i = 0; i < n; ++i) {
    int64_t a = offsets[i], b = offsets[i + 1];
    if (b <= a) continue;
    double w = 1.0 / (double)(b - a);
    for (int64_t j = a; j < b; ++j) {
      int64_t lo;
      int rc = corners(d, M, t + j * d, node, wt, &lo);
      if (rc) return rc;
      for (int q = 0; q < (1 << d); ++q) {
        c[node[q]] += w * wt[q];
        s[node[q]] += w * wt[q] * y[j];
      }
      if (idx) idx[j] = (int32_t)lo;
      if (cnt) cnt[lo] += 1;
    }
  }
  return ORC_OK;
}

/* Covariance binning by explicit ordered pairs j != l (eq. 2.4, weights
 * 1/(N_i(N_i-1)); curves with N_i < 2 contribute nothing):
 *   C[p,q] += w W_p(t_ij) W_q(t_il),  G[p,q] += w W_p W_q Y_ij Y_il,
 *   Q[p,q] += w W_p W_q (Y_ij Y_il)^2 (the squared raw products used by CV),
 *   cnt2[lower_j, lower_l] += 1.
 * If fold != NULL and fold_sel >= 0, only curves with fold[i] == fold_sel count.
 * Any output pointer may be NULL. */
int orc_bin_cov_pairs(int d, const int *M, int64_t n, const int64_t *offsets, const double *t,
                      const double *y, const int32_t *fold, int fold_sel, double *C, double *G,
                      double *Q, int64_t *cnt2) {
  if (check_grid(d, M) || n < 0) return ORC_ERR_ARG;
  int64_t P = grid_size(d, M);
  int nc = 1 << d;
  if (C) memset(C, 0, sizeof(double) * P * P);
  if (G) memset(G, 0, sizeof(double) * P * P);
  if (Q) memset(Q, 0, sizeof(double) * P * P);
  if (cnt2) memset(cnt2, 0, sizeof(int64_t) * P * P);
  for (int64_t i = 0; i < n; ++i) {
    if (fold && fold_sel >= 0 && fold[i] != fold_sel) continue;
    int64_t a = offsets[i], b = offsets[i + 1];
    int64_t Ni = b - a;
    if (Ni < 2) continue;
    double w = 1.0 / ((double)Ni * (double)(Ni - 1));
    int64_t *node = (int64_t *)malloc(sizeof(int64_t) * Ni * nc);
    double *wt = (double *)malloc(sizeof(double) * Ni * nc);
    int64_t *lo = (int64_t *)malloc(sizeof(int64_t) * Ni);
    for (int64_t j = 0; j < Ni; ++j) {
      int rc = corners(d, M, t + (a + j) * d, node + j * nc, wt + j * nc, lo + j);
      if (rc) {
        free(node); free(wt); free(lo);
        return rc;
      }
    }
    for (int64_t j = 0; j < Ni; ++j) {
      for (int64_t l = 0; l < Ni; ++l) {
        if (j == l) continue;
        double yy = y[a + j] * y[a + l];
        for (int u = 0; u < nc; ++u) {
          for (int v = 0; v < nc; ++v) {
            int64_t pq = node[j * nc + u] * P + node[l * nc + v];
            double ww = w * wt[j * nc + u] * wt[l * nc + v];
            if (C) C[pq] += ww;
            if (G) G[pq] += ww * yy;
            if (Q) Q[pq] += ww * yy * yy;
          }
        }
        if (cnt2) cnt2[lo[j] * P + lo[l]] += 1;
      }
    }
    free(node); free(wt); free(lo);
  }
  return ORC_OK;
}

/* One-dimensional Epanechnikov profile K(u) = (1-u^2)_+ at the grid offset m
 * along a coordinate with M nodes and bandwidth h: u = m / (h (M-1)).
 * The constants 3/4 and 1/h of K_h are dropped: b0 of the weighted least
 * squares problem does not change when all weights are scaled by one constant. */
static double epan(int m, double h, int M) {
  double u = (double)m / (h * (double)(M - 1));
  return (fabs(u) < 1.0) ? (1.0 - u * u) : 0.0;
}

static double uval(int m, double h, int M) { return (double)m / (h * (double)(M - 1)); }

/* Solve the (D+1)x(D+1) normal equations of the local-linear fit
 *   [[S0, S1^T], [S1, S2]] beta = [T0; T1]
 * and return b0 = beta_0 with a status:
 *   EMPTY    S0 == 0: no data in the window, b0 = NaN;
 *   FALLBACK a zero diagonal entry, a non-positive Cholesky pivot, or a smallest
 *            pivot below 1e-10 of the unit-diagonal (Jacobi-scaled) system:
 *            b0 = T0/S0 (the local-constant fit);
 *   OK       b0 from the Cholesky solve. */
static int8_t wls_solve(int D, const double *A_in, const double *r_in, double *b0, double *minpiv) {
  int n = D + 1;
  double A[(MAXDD + 1) * (MAXDD + 1)], r[MAXDD + 1], sc[MAXDD + 1], L[(MAXDD + 1) * (MAXDD + 1)];
  *minpiv = 0.0;
  if (!(A_in[0] > 0.0)) {
    *b0 = NAN;
    return ST_EMPTY;
  }
  for (int i = 0; i < n; ++i) {
    if (!(A_in[i * n + i] > 0.0)) {
      *b0 = r_in[0] / A_in[0];
      return ST_FALLBACK;
    }
    sc[i] = 1.0 / sqrt(A_in[i * n + i]);
  }
  for (int i = 0; i < n; ++i) {
    r[i] = r_in[i] * sc[i];
    for (int j = 0; j < n; ++j) A[i * n + j] = sc[i] * A_in[i * n + j] * sc[j];
  }
  memset(L, 0, sizeof(L));
  double mp = 1e300;
  for (int j = 0; j < n; ++j) {
    double dj = A[j * n + j];
    for (int k = 0; k < j; ++k) dj -= L[j * n + k] * L[j * n + k];
    if (!(dj > 0.0)) {
      *b0 = r_in[0] / A_in[0];
      return ST_FALLBACK;
    }
    if (dj < mp) mp = dj;
    double ljj = sqrt(dj);
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / ljj;
    }
  }
  *minpiv = mp;
  if (mp < 1e-10) {
    *b0 = r_in[0] / A_in[0];
    return ST_FALLBACK;
  }
  double z[MAXDD + 1], x[MAXDD + 1];
  for (int i = 0; i < n; ++i) {
    double v = r[i];
    for (int k = 0; k < i; ++k) v -= L[i * n + k] * z[k];
    z[i] = v / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = z[i];
    for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
    x[i] = v / L[i * n + i];
  }
  *b0 = x[0] * sc[0];
  return ST_OK;
}

/* Number of moments of a D-dimensional local-linear fit:
 * S0, S1[D], S2 upper triangle [D(D+1)/2], T0, T1[D]. */
int orc_num_moments(int D) { return 1 + D + D * (D + 1) / 2 + 1 + D; }

/* Binned local-linear smoother, evaluated node by node by direct summation
 * over the window (the definition of eqs. 2.3 / 2.4 on binned data):
 * at node x and every bin y with |y_k - x_k| <= h_k in all D coordinates,
 * weight K = prod_k (1-u_k^2)_+, u_k = (y_k - x_k)/h_k, and
 *   S0 = sum w K, S1_k = sum w K u_k, S2_kl = sum w K u_k u_l,
 *   T0 = sum g K, T1_k = sum g K u_k,
 * followed by the weighted least-squares solve for b0.
 *   dims[D], h[D]: array dims and per-dimension bandwidths;
 *   w, g: binned weights and weighted responses (prod dims entries);
 *   nodes: n_nodes flat indices to evaluate, or NULL for every node;
 *   b0, status: outputs per evaluated node; mom (optional): the moments in the
 *   order above; minpiv (optional): smallest pivot of the scaled system. */
int orc_smooth(int D, const int *dims, const double *h, const double *w, const double *g,
               int64_t n_nodes, const int64_t *nodes, double *b0, int8_t *status, double *mom,
               double *minpiv) {
  if (D < 1 || D > MAXDD) return ORC_ERR_ARG;
  int64_t total = 1;
  int R[MAXDD];
  int64_t stride[MAXDD];
  for (int k = 0; k < D; ++k) {
    if (dims[k] < 2 || !(h[k] > 0.0)) return ORC_ERR_ARG;
    total *= dims[k];
    R[k] = (int)floor(h[k] * (double)(dims[k] - 1));
  }
  stride[D - 1] = 1;
  for (int k = D - 2; k >= 0; --k) stride[k] = stride[k + 1] * dims[k + 1];
  if (!nodes) n_nodes = total;
  int nm = orc_num_moments(D);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < n_nodes; ++e) {
    int64_t flat = nodes ? nodes[e] : e;
    int x[MAXDD], lo[MAXDD], hi[MAXDD], y[MAXDD];
    int64_t rem = flat;
    for (int k = 0; k < D; ++k) {
      x[k] = (int)(rem / stride[k]);
      rem -= (int64_t)x[k] * stride[k];
      lo[k] = x[k] - R[k] < 0 ? 0 : x[k] - R[k];
      hi[k] = x[k] + R[k] > dims[k] - 1 ? dims[k] - 1 : x[k] + R[k];
    }
    double S0 = 0, S1[MAXDD] = {0}, S2[MAXDD][MAXDD] = {{0}}, T0 = 0, T1[MAXDD] = {0};
    for (int k = 0; k < D; ++k) y[k] = lo[k];
    for (;;) {
      double K = 1.0, u[MAXDD];
      int64_t yf = 0;
      for (int k = 0; k < D; ++k) {
        K *= epan(y[k] - x[k], h[k], dims[k]);
        u[k] = uval(y[k] - x[k], h[k], dims[k]);
        yf += (int64_t)y[k] * stride[k];
      }
      if (K != 0.0) {
        double wk = w[yf] * K, gk = g[yf] * K;
        S0 += wk;
        T0 += gk;
        for (int k = 0; k < D; ++k) {
          S1[k] += wk * u[k];
          T1[k] += gk * u[k];
          for (int l = k; l < D; ++l) S2[k][l] += wk * u[k] * u[l];
        }
      }
      int k = D - 1;
      while (k >= 0) {
        if (++y[k] <= hi[k]) break;
        y[k] = lo[k];
        --k;
      }
      if (k < 0) break;
    }
    int n = D + 1;
    double A[(MAXDD + 1) * (MAXDD + 1)], r[MAXDD + 1];
    A[0] = S0;
    r[0] = T0;
    for (int k = 0; k < D; ++k) {
      A[0 * n + 1 + k] = A[(1 + k) * n + 0] = S1[k];
      r[1 + k] = T1[k];
      for (int l = k; l < D; ++l) A[(1 + k) * n + 1 + l] = A[(1 + l) * n + 1 + k] = S2[k][l];
    }
    double mp;
    status[e] = wls_solve(D, A, r, &b0[e], &mp);
    if (minpiv) minpiv[e] = mp;
    if (mom) {
      double *o = mom + e * nm;
      int q = 0;
      o[q++] = S0;
      for (int k = 0; k < D; ++k) o[q++] = S1[k];
      for (int k = 0; k < D; ++k)
        for (int l = k; l < D; ++l) o[q++] = S2[k][l];
      o[q++] = T0;
      for (int k = 0; k < D; ++k) o[q++] = T1[k];
    }
  }
  return ORC_OK;
}

/* Weighted least-squares solve on moment vectors supplied by the caller
 * (same ordering as orc_smooth's `mom`), used to pin the solver by itself. */
int orc_wls_from_moments(int D, int64_t n_nodes, const double *mom, double *b0, int8_t *status,
                         double *minpiv) {
  if (D < 1 || D > MAXDD) return ORC_ERR_ARG;
  int nm = orc_num_moments(D), n = D + 1;
  for (int64_t e = 0; e < n_nodes; ++e) {
    const double *o = mom + e * nm;
    double A[(MAXDD + 1) * (MAXDD + 1)], r[MAXDD + 1];
    int q = 0;
    A[0] = o[q++];
    for (int k = 0; k < D; ++k) A[1 + k] = A[(1 + k) * n] = o[q++];
    for (int k = 0; k < D; ++k)
      for (int l = k; l < D; ++l) {
        A[(1 + k) * n + 1 + l] = A[(1 + l) * n + 1 + k] = o[q++];
      }
    r[0] = o[q++];
    for (int k = 0; k < D; ++k) r[1 + k] = o[q++];
    double mp;
    status[e] = wls_solve(D, A, r, &b0[e], &mp);
    if (minpiv) minpiv[e] = mp;
  }
  return ORC_OK;
}

/* splitmix64 (Steele, Lea & Flood, OOPSLA 2014): the n-th output (n = 0,1,...)
 * of the generator started at state `seed` is mix(seed + (n+1)*gamma). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int orc_splitmix64(uint64_t seed, int64_t count, uint64_t *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = splitmix64_at(seed, (uint64_t)i);
  return ORC_OK;
}

/* Standard normal number i of stream `seed` by the Box-Muller transform
 * (Box & Muller 1958), cosine branch: u1 = (a>>11 + 1) 2^-53 in (0,1],
 * u2 = (b>>11) 2^-53 in [0,1), with a, b outputs 2i and 2i+1 of splitmix64.
 * A P x r test matrix uses i = j*P + p for entry (p, j). */
int orc_normals(uint64_t seed, int64_t count, double *out) {
  const double two53 = 1.0 / 9007199254740992.0;
  const double two_pi = 6.283185307179586476925286766559;
  for (int64_t i = 0; i < count; ++i) {
    uint64_t a = splitmix64_at(seed, 2 * (uint64_t)i);
    uint64_t b = splitmix64_at(seed, 2 * (uint64_t)i + 1);
    double u1 = (double)((a >> 11) + 1) * two53;
    double u2 = (double)(b >> 11) * two53;
    out[i] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  }
  return ORC_OK;
}

/* Threads the OpenMP loops of this library use. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

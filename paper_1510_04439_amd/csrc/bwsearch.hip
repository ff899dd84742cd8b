// Bandwidth selection of Section 3.3: leave-one-observation-out
// cross-validation of the covariance smoother, minimized over continuous
// bandwidths by a derivative-free trust-region method whose local model is a
// quadratic regression on the sampled criterion (the paper replaces the
// interpolation of the interpolation-based trust-region method by a
// regression, the empirical criterion being noisy).
//
// Criterion (binned reading): at every node x of the 2d-dimensional grid the
// local-linear fit leaves x's own bin out (its weight and sum leave S0 and T0;
// u = 0 there, so no other moment changes) and the data are scored through
// their bins, sum_x Q - 2 G b_{-x} + C b_{-x}^2 (b = 0 where the reduced
// window is empty or outside the mask). The criteria of a batch of bandwidth
// vectors are one persistent launch of the task-queue smoother
// (smooth_tiled.hip, leave-one-out jobs).
//
// Search: on x = log h over the box [log h_lo, log h_hi]; the initial design
// is the centre, +-r e_k, +-r/2 e_k and the diagonal points centre +
// r/2 (e_k + e_l); the model is fitted by least squares (normal equations
// with a 1e-10 relative ridge) to the points within 2r (max norm) of the
// centre, or to the p + 1 nearest (p = (d+1)(d+2)/2); the step minimizes the
// model in the ball of radius r (Newton point, or the boundary point by 200
// bisection steps on the shift); acceptance 0.1, expansion 0.75 when the step
// reaches 0.9 r, halving otherwise; after a rejected step a geometry point
// centre + r e_k (k cycling) is sampled with the next candidate; stop when
// r < 0.01 or the evaluation budget is spent. The best sampled point wins.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "tiled.hpp"

namespace fpca {
namespace {

typedef std::vector<double> Vec;

// Symmetric eigendecomposition of a d x d matrix (d <= 3) by cyclic Jacobi:
// eigenvalues ascending in lam, eigenvectors as the columns of V.
void sym_eig(int d, const double *A, double *lam, double *V) {
  double a[9], v[9];
  std::memcpy(a, A, sizeof(double) * d * d);
  for (int i = 0; i < d * d; ++i) v[i] = 0.0;
  for (int i = 0; i < d; ++i) v[i * d + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) off += a[p * d + q] * a[p * d + q];
    if (off < 1e-300) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = a[p * d + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * d + q] - a[p * d + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < d; ++k) {
          const double akp = a[k * d + p], akq = a[k * d + q];
          a[k * d + p] = c * akp - s * akq;
          a[k * d + q] = s * akp + c * akq;
        }
        for (int k = 0; k < d; ++k) {
          const double apk = a[p * d + k], aqk = a[q * d + k];
          a[p * d + k] = c * apk - s * aqk;
          a[q * d + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < d; ++k) {
          const double vkp = v[k * d + p], vkq = v[k * d + q];
          v[k * d + p] = c * vkp - s * vkq;
          v[k * d + q] = s * vkp + c * vkq;
        }
      }
  }
  int idx[3] = {0, 1, 2};
  std::sort(idx, idx + d, [&](int x, int y) { return a[x * d + x] < a[y * d + y]; });
  for (int j = 0; j < d; ++j) {
    lam[j] = a[idx[j] * d + idx[j]];
    for (int k = 0; k < d; ++k) V[k * d + j] = v[k * d + idx[j]];
  }
}

// argmin g.z + z.H.z/2 over |z| <= 1.
Vec tr_step(int d, const Vec &g, const Vec &H) {
  double lam[3], V[9];
  sym_eig(d, H.data(), lam, V);
  double gam[3];
  for (int j = 0; j < d; ++j) {
    gam[j] = 0.0;
    for (int k = 0; k < d; ++k) gam[j] += V[k * d + j] * g[k];
  }
  auto back = [&](const double *y) {
    Vec z(d, 0.0);
    for (int k = 0; k < d; ++k)
      for (int j = 0; j < d; ++j) z[k] += V[k * d + j] * y[j];
    return z;
  };
  auto norm = [&](const Vec &z) {
    double s = 0.0;
    for (double v : z) s += v * v;
    return std::sqrt(s);
  };
  if (lam[0] > 0.0) {
    double y[3];
    for (int j = 0; j < d; ++j) y[j] = -gam[j] / lam[j];
    Vec zn = back(y);
    if (norm(zn) <= 1.0) return zn;
  }
  const double mu_lo = std::max(0.0, -lam[0]);
  double amax = 0.0, gn = 0.0, gamn = 0.0;
  for (int j = 0; j < d; ++j) {
    amax = std::max(amax, std::fabs(lam[j]));
    gn += g[j] * g[j];
    gamn += gam[j] * gam[j];
  }
  gn = std::sqrt(gn);
  gamn = std::sqrt(gamn);
  const double tiny = 1e-14 * std::max(1.0, amax);
  if (lam[0] + mu_lo <= tiny && std::fabs(gam[0]) <= 1e-14 * std::max(1.0, gn)) {
    double y[3] = {0.0, 0.0, 0.0}, s = 0.0;
    for (int j = 0; j < d; ++j)
      if (lam[j] + mu_lo > tiny) {
        y[j] = -gam[j] / (lam[j] + mu_lo);
        s += y[j] * y[j];
      }
    y[0] = std::sqrt(std::max(1.0 - s, 0.0));
    return back(y);
  }
  auto phi = [&](double mu) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) s += gam[j] * gam[j] / ((lam[j] + mu) * (lam[j] + mu));
    return s;
  };
  double lo = mu_lo, hi = mu_lo + gamn + 1e-12;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (lam[0] + mid <= 0.0 || phi(mid) > 1.0)
      lo = mid;
    else
      hi = mid;
  }
  double y[3];
  for (int j = 0; j < d; ++j) y[j] = -gam[j] / (lam[j] + hi);
  return back(y);
}

// Least-squares quadratic c0 + g.z + z.H.z/2 through (Z rows, f).
void fit_quadratic(int d, const std::vector<Vec> &Z, const Vec &f, Vec &g, Vec &H) {
  const int nb = 1 + d + d * (d + 1) / 2;
  const int m = int(Z.size());
  std::vector<double> A(size_t(m) * nb);
  for (int i = 0; i < m; ++i) {
    double *r = &A[size_t(i) * nb];
    int c = 0;
    r[c++] = 1.0;
    for (int k = 0; k < d; ++k) r[c++] = Z[i][k];
    for (int k = 0; k < d; ++k)
      for (int l = k; l < d; ++l) r[c++] = Z[i][k] * Z[i][l];
  }
  std::vector<double> N(size_t(nb) * nb, 0.0), rhs(nb, 0.0);
  for (int a = 0; a < nb; ++a) {
    for (int b = 0; b < nb; ++b) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += A[size_t(i) * nb + a] * A[size_t(i) * nb + b];
      N[size_t(a) * nb + b] = s;
    }
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += A[size_t(i) * nb + a] * f[i];
    rhs[a] = s;
  }
  double tr = 0.0;
  for (int a = 0; a < nb; ++a) tr += N[size_t(a) * nb + a];
  for (int a = 0; a < nb; ++a) N[size_t(a) * nb + a] += 1e-10 * tr / nb;
  // Cholesky N = L L^T, then L y = rhs, L^T c = y
  std::vector<double> L(size_t(nb) * nb, 0.0);
  for (int j = 0; j < nb; ++j) {
    double s = N[size_t(j) * nb + j];
    for (int k = 0; k < j; ++k) s -= L[size_t(j) * nb + k] * L[size_t(j) * nb + k];
    const double ljj = std::sqrt(std::max(s, 1e-300));
    L[size_t(j) * nb + j] = ljj;
    for (int i = j + 1; i < nb; ++i) {
      double t = N[size_t(i) * nb + j];
      for (int k = 0; k < j; ++k) t -= L[size_t(i) * nb + k] * L[size_t(j) * nb + k];
      L[size_t(i) * nb + j] = t / ljj;
    }
  }
  Vec y(nb), c(nb);
  for (int i = 0; i < nb; ++i) {
    double s = rhs[i];
    for (int k = 0; k < i; ++k) s -= L[size_t(i) * nb + k] * y[k];
    y[i] = s / L[size_t(i) * nb + i];
  }
  for (int i = nb - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < nb; ++k) s -= L[size_t(k) * nb + i] * c[k];
    c[i] = s / L[size_t(i) * nb + i];
  }
  g.assign(d, 0.0);
  H.assign(size_t(d) * d, 0.0);
  for (int k = 0; k < d; ++k) g[k] = c[1 + k];
  int i = 1 + d;
  for (int k = 0; k < d; ++k)
    for (int l = k; l < d; ++l, ++i) {
      if (k == l)
        H[size_t(k) * d + k] = 2.0 * c[i];
      else
        H[size_t(k) * d + l] = H[size_t(l) * d + k] = c[i];
    }
}

// Leave-one-out criteria of the bandwidth rows hs (n x d) in one launch.
template <typename T>
int loo_batch(fpca_context *ctx, const fpca_grid *grid, const T *C, const T *G, const T *Q, int n,
              const double *hs, double *out) {
  std::vector<TiledJob> jobs(n);
  for (int i = 0; i < n; ++i) {
    TiledJob &j = jobs[i];
    j = TiledJob{};
    j.grid = grid;
    j.Ca = C;
    j.Ga = G;
    j.Qf = Q;
    j.Gf = G;
    j.Cf = C;
    j.h = hs + size_t(i) * grid->d;
    j.loo = 1;
  }
  TiledConfig cfg;
  size_t lds = tiled_lds(jobs, 16);
  cfg.qb = 16;
  if (!lds || lds > 80 * 1024) {
    cfg.qb = 8;
    lds = tiled_lds(jobs, 8);
  }
  if (!lds) return set_error(FPCA_ERR_UNSUPPORTED, "leave-one-out CV: grid too large for the task-queue smoother");
  cfg.wg_per_cu = int(std::max<size_t>(1, std::min<size_t>(2, (160 * 1024) / (lds + 256))));
  TiledLaunch L;
  if (int rc = tiled_plan<T>(ctx, jobs, true, cfg, &L)) return rc;
  if (int rc = tiled_queue(ctx, L)) return rc;
  FPCA_HIP(hipMemcpyAsync(ctx->h_flags, ctx->d_flags, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  FPCA_HIP(hipStreamSynchronize(ctx->stream));
  if (*ctx->h_flags & 2) {
    const int keep = *ctx->h_flags & ~2;
    *ctx->h_flags = 0;
    FPCA_HIP(hipMemcpy(ctx->d_flags, &keep, sizeof(int), hipMemcpyHostToDevice));
    return set_error(FPCA_ERR_DEVICE, "leave-one-out CV: a task waited past its spin limit");
  }
  FPCA_HIP(hipMemcpy(out, L.args.scores, sizeof(double) * n, hipMemcpyDeviceToHost));
  return FPCA_OK;
}

template <typename T>
int search_impl(fpca_context *ctx, const fpca_grid *grid, const T *C, const T *G, const T *Q, const double *h_lo,
                const double *h_hi, const double *h_init, int max_evals, double *h_out, double *cv_out,
                int *n_evals, double *trace) {
  const int d = grid->d;
  Vec lo(d), hi(d), x0(d);
  double wmax = 0.0;
  for (int k = 0; k < d; ++k) {
    lo[k] = std::log(h_lo[k]);
    hi[k] = std::log(h_hi[k]);
    x0[k] = std::min(std::max(std::log(h_init[k]), lo[k]), hi[k]);
    wmax = std::max(wmax, hi[k] - lo[k]);
  }
  double delta = std::min(std::max(0.25 * wmax, 0.05), 1.0);
  const double dmin = 0.01, dmax = 1.0, eta1 = 0.1, eta2 = 0.75;
  const int p = (d + 1) * (d + 2) / 2;
  std::vector<Vec> X;
  Vec F;
  auto clip = [&](Vec x) {
    for (int k = 0; k < d; ++k) x[k] = std::min(std::max(x[k], lo[k]), hi[k]);
    return x;
  };
  auto seen = [&](const Vec &q) {
    for (const Vec &r : X)
      if (r == q) return true;
    return false;
  };
  auto evaluate = [&](std::vector<Vec> pts, Vec &vals) -> int {
    for (Vec &q : pts) q = clip(q);
    std::vector<double> hs(pts.size() * d);
    for (size_t i = 0; i < pts.size(); ++i)
      for (int k = 0; k < d; ++k) hs[i * d + k] = std::exp(pts[i][k]);
    vals.assign(pts.size(), 0.0);
    if (int rc = loo_batch<T>(ctx, grid, C, G, Q, int(pts.size()), hs.data(), vals.data())) return rc;
    for (size_t i = 0; i < pts.size(); ++i) {
      X.push_back(pts[i]);
      F.push_back(vals[i]);
    }
    return FPCA_OK;
  };
  auto e_k = [&](int k, double s) {
    Vec e(d, 0.0);
    e[k] = s;
    return e;
  };
  auto add = [&](const Vec &a, const Vec &b) {
    Vec r(d);
    for (int k = 0; k < d; ++k) r[k] = a[k] + b[k];
    return r;
  };
  // initial design
  std::vector<Vec> design = {x0};
  for (int k = 0; k < d; ++k) {
    design.push_back(add(x0, e_k(k, delta)));
    design.push_back(add(x0, e_k(k, -delta)));
  }
  for (int k = 0; k < d; ++k) {
    design.push_back(add(x0, e_k(k, 0.5 * delta)));
    design.push_back(add(x0, e_k(k, -0.5 * delta)));
  }
  for (int k = 0; k < d; ++k)
    for (int l = k + 1; l < d; ++l) design.push_back(add(x0, add(e_k(k, 0.5 * delta), e_k(l, 0.5 * delta))));
  std::vector<Vec> uniq;
  for (const Vec &q0 : design) {
    const Vec q = clip(q0);
    if (std::find(uniq.begin(), uniq.end(), q) == uniq.end()) uniq.push_back(q);
  }
  Vec vals;
  if (int rc = evaluate(uniq, vals)) return rc;
  int b = int(std::min_element(F.begin(), F.end()) - F.begin());
  Vec xc = X[b];
  double fc = F[b];
  int it = 0;
  bool failed = false;
  while (int(X.size()) < max_evals && delta >= dmin) {
    // regression points
    std::vector<int> sel;
    for (size_t i = 0; i < X.size(); ++i) {
      double dist = 0.0;
      for (int k = 0; k < d; ++k) dist = std::max(dist, std::fabs(X[i][k] - xc[k]));
      if (dist <= 2.0 * delta) sel.push_back(int(i));
    }
    if (int(sel.size()) < p + 1) {
      std::vector<int> ord(X.size());
      for (size_t i = 0; i < X.size(); ++i) ord[i] = int(i);
      std::vector<double> e2(X.size());
      for (size_t i = 0; i < X.size(); ++i) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += (X[i][k] - xc[k]) * (X[i][k] - xc[k]);
        e2[i] = std::sqrt(s);
      }
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return e2[x] < e2[y]; });
      sel.assign(ord.begin(), ord.begin() + std::min<size_t>(ord.size(), size_t(p + 1)));
    }
    std::vector<Vec> Z;
    Vec fz;
    for (int i : sel) {
      Vec z(d);
      for (int k = 0; k < d; ++k) z[k] = (X[i][k] - xc[k]) / delta;
      Z.push_back(z);
      fz.push_back(F[i]);
    }
    Vec g, H;
    fit_quadratic(d, Z, fz, g, H);
    const Vec z = tr_step(d, g, H);
    Vec xp(d);
    for (int k = 0; k < d; ++k) xp[k] = xc[k] + delta * z[k];
    xp = clip(xp);
    double stepn = 0.0;
    for (int k = 0; k < d; ++k) stepn += (xp[k] - xc[k]) * (xp[k] - xc[k]);
    if (std::sqrt(stepn) <= 1e-6) {
      delta *= 0.5;
      ++it;
      failed = true;
      continue;
    }
    std::vector<Vec> batch = {xp};
    if (failed) {
      const int k = it % d;
      Vec xg = clip(add(xc, e_k(k, delta)));
      if (seen(xg)) xg = clip(add(xc, e_k(k, -delta)));
      if (!seen(xg) && xg != xp) batch.push_back(xg);
    }
    const size_t first = X.size();
    if (int rc = evaluate(batch, vals)) return rc;
    const Vec &p0 = X[first];
    Vec zs(d);
    for (int k = 0; k < d; ++k) zs[k] = (p0[k] - xc[k]) / delta;
    double gz = 0.0, zHz = 0.0, zn = 0.0;
    for (int k = 0; k < d; ++k) {
      gz += g[k] * zs[k];
      zn += zs[k] * zs[k];
      for (int l = 0; l < d; ++l) zHz += zs[k] * H[size_t(k) * d + l] * zs[l];
    }
    const double pred = -(gz + 0.5 * zHz);
    const double rho = pred > 0.0 ? (fc - vals[0]) / pred : -1.0;
    if (rho >= eta1 && vals[0] < fc) {
      xc = p0;
      fc = vals[0];
      if (rho >= eta2 && std::sqrt(zn) >= 0.9) delta = std::min(2.0 * delta, dmax);
      failed = false;
    } else {
      delta *= 0.5;
      failed = true;
    }
    if (vals.size() > 1 && vals[1] < fc) {
      xc = X[first + 1];
      fc = vals[1];
    }
    ++it;
  }
  b = int(std::min_element(F.begin(), F.end()) - F.begin());
  for (int k = 0; k < d; ++k) h_out[k] = std::exp(X[b][k]);
  if (cv_out) *cv_out = F[b];
  if (n_evals) *n_evals = int(X.size());
  if (trace)
    for (size_t i = 0; i < X.size() && int(i) < max_evals; ++i) {
      for (int k = 0; k < d; ++k) trace[i * (d + 1) + k] = std::exp(X[i][k]);
      trace[i * (d + 1) + d] = F[i];
    }
  return FPCA_OK;
}

int check_loo_args(fpca_context *ctx, const fpca_grid *grid, int dtype, const void *C, const void *G, const void *Q) {
  if (int rc = check_handle(ctx)) return rc;
  int64_t P;
  if (int rc = check_grid(grid, &P)) return rc;
  if (dtype != FPCA_F64 && dtype != FPCA_F32) return set_error(FPCA_ERR_INVALID_ARG, "bad dtype %d", dtype);
  if (!C || !G || !Q) return set_error(FPCA_ERR_INVALID_ARG, "C, G and Q are required");
  if (!tiled_supported(grid))
    return set_error(FPCA_ERR_UNSUPPORTED, "leave-one-out CV needs P <= 4096 and M_1 <= 64/32/16 for d = 1/2/3");
  return set_device(ctx);
}

}  // namespace
}  // namespace fpca

using namespace fpca;

extern "C" int fpca_cv_loo(fpca_handle ctx, const fpca_grid *grid, int dtype, const void *C, const void *G,
                           const void *Q, int n_h, const double *bandwidths, double *scores) {
  if (int rc = check_loo_args(ctx, grid, dtype, C, G, Q)) return rc;
  if (n_h < 1 || !bandwidths || !scores) return set_error(FPCA_ERR_INVALID_ARG, "need n_h >= 1, bandwidths, scores");
  for (int i = 0; i < n_h * grid->d; ++i)
    if (!(bandwidths[i] > 0.0) || !std::isfinite(bandwidths[i]))
      return set_error(FPCA_ERR_INVALID_ARG, "bandwidths must be positive and finite");
  if (dtype == FPCA_F64)
    return loo_batch<double>(ctx, grid, static_cast<const double *>(C), static_cast<const double *>(G),
                             static_cast<const double *>(Q), n_h, bandwidths, scores);
  return loo_batch<float>(ctx, grid, static_cast<const float *>(C), static_cast<const float *>(G),
                          static_cast<const float *>(Q), n_h, bandwidths, scores);
}

extern "C" int fpca_bw_search(fpca_handle ctx, const fpca_grid *grid, int dtype, const void *C, const void *G,
                              const void *Q, const double *h_lo, const double *h_hi, const double *h_init,
                              int max_evals, double *h_out, double *cv_out, int *n_evals, double *trace) {
  if (int rc = check_loo_args(ctx, grid, dtype, C, G, Q)) return rc;
  if (!h_lo || !h_hi || !h_init || !h_out) return set_error(FPCA_ERR_INVALID_ARG, "h_lo, h_hi, h_init, h_out required");
  const int d = grid->d;
  for (int k = 0; k < d; ++k)
    if (!(h_lo[k] > 0.0) || !(h_hi[k] >= h_lo[k]) || !std::isfinite(h_hi[k]) || !(h_init[k] > 0.0))
      return set_error(FPCA_ERR_INVALID_ARG, "need 0 < h_lo <= h_hi and h_init > 0");
  const int need = 1 + 4 * d + d * (d - 1) / 2;
  if (max_evals < need) return set_error(FPCA_ERR_INVALID_ARG, "max_evals must be at least %d", need);
  if (dtype == FPCA_F64)
    return search_impl<double>(ctx, grid, static_cast<const double *>(C), static_cast<const double *>(G),
                               static_cast<const double *>(Q), h_lo, h_hi, h_init, max_evals, h_out, cv_out,
                               n_evals, trace);
  return search_impl<float>(ctx, grid, static_cast<const float *>(C), static_cast<const float *>(G),
                            static_cast<const float *>(Q), h_lo, h_hi, h_init, max_evals, h_out, cv_out, n_evals,
                            trace);
}

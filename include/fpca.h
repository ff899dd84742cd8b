/*
 * fpca.h -- C ABI of the MI355X (gfx950) library for the hot path of
 * multi-dimensional functional principal component analysis
 * (Chen & Jiang, "Multi-dimensional Functional Principal Component Analysis").
 *
 * Problem statement (paper Section 2, eqs. 2.1-2.2): curves i = 1..n, each
 * observed at N_i points t_ij in a domain Omega inside [0,1]^d (d <= 3) with
 * values Y_ij = X_i(t_ij) + noise. The library computes
 *   - linear binning of the observations onto a regular grid (Section 3.2),
 *   - the binned local-linear smoother of the mean (eq. 2.3),
 *   - the same smoother of the raw covariance surface on the 2d-dimensional
 *     grid and the covariance Gamma(s,t) = b0(s,t) - mu(s) mu(t) (eq. 2.4),
 *   - the top eigenpairs of the matrixized covariance (Section 3.1, eq. 3.1)
 *     by random projection (Section 3.4).
 *
 * Conventions shared by every call
 *   Grid: M_k nodes per coordinate at m/(M_k-1), m = 0..M_k-1; P = prod_k M_k;
 *   flat node index with the last coordinate fastest. A covariance array is
 *   P x P row-major: entry (p, q) is the s-node p and t-node q.
 *   Kernel: product Epanechnikov K(u) = prod_k (1 - u_k^2)_+ (paper Section
 *   2.1 names the product Epanechnikov kernel), u_k = (y_k - x_k) / h_k.
 *   Memory: every array argument is a caller-allocated, contiguous DEVICE
 *   pointer unless marked "host". The library never frees or retains caller
 *   pointers after the stream work of the call has completed. Scratch memory
 *   is owned by the handle; it grows on demand and is released by
 *   fpca_destroy.
 *   Streams: work is queued on the handle's stream (fpca_set_stream); calls
 *   return after queueing, except where a host output is written (they then
 *   synchronize the stream).
 *   Errors: argument checks are synchronous and return a negative code with a
 *   message in fpca_last_error(). Observations outside [0,1]^d or NaN are
 *   detected on the device: they are skipped and raise a flag that the next
 *   fpca_sync (or a call that synchronizes) returns as FPCA_ERR_DOMAIN.
 *   Per-node numerical trouble in a smoother is not an error: it is reported
 *   in `status` (FPCA_STATUS_*).
 *   Handles are not thread-safe: use one handle per host thread.
 */
#ifndef FPCA_H
#define FPCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpca_context *fpca_handle;

/* Return codes. */
#define FPCA_OK 0
#define FPCA_ERR_INVALID_ARG (-1)
#define FPCA_ERR_DOMAIN (-2)      /* an observation outside [0,1]^d, or NaN */
#define FPCA_ERR_UNSUPPORTED (-3) /* a size, dtype or precision combination not built */
#define FPCA_ERR_WORKSPACE (-4)   /* scratch allocation failed or exceeded its limit */
#define FPCA_ERR_DEVICE (-5)      /* a HIP runtime error */

/* Per-node status of a smoother (the weighted least-squares solve). */
#define FPCA_STATUS_OK 0       /* b0 of the local-linear fit */
#define FPCA_STATUS_FALLBACK 1 /* singular or near-singular system: b0 = T0/S0, the local-constant fit */
#define FPCA_STATUS_EMPTY 2    /* no data in the window: b0 = NaN */

/* Binning kinds, designs, storage dtypes, compute precisions, kernels. */
#define FPCA_BIN_MEAN 0
#define FPCA_BIN_COV 1
#define FPCA_IRREGULAR 0
#define FPCA_COMMON_GRID 1
#define FPCA_F64 0
#define FPCA_F32 1
#define FPCA_PREC_F64 0
#define FPCA_PREC_F32 1
#define FPCA_PREC_BF16X3 2
#define FPCA_K_EPANECHNIKOV 0

/* Regular grid over the bounding rectangle [0,1]^d (Section 3.1): d in 1..3,
 * M[k] >= 2 nodes per coordinate. mask: optional device array of P bytes,
 * nonzero where a node lies in Omega; NULL means Omega is the rectangle. */
typedef struct {
  int d;
  int M[3];
  const uint8_t *mask;
} fpca_grid;

/* Handle on device `device` (a HIP device ordinal), using the null stream
 * until fpca_set_stream is called. */
int fpca_create(fpca_handle *handle, int device);
int fpca_destroy(fpca_handle handle);
/* stream: a hipStream_t of the handle's device, passed as void*. */
int fpca_set_stream(fpca_handle handle, void *stream);
/* A stream of device `device` whose kernels run only on the compute units
 * selected by bits cu_begin .. cu_end-1 of the device's CU mask (the HIP
 * runtime's mask for a stream; 0 <= cu_begin < cu_end <= the device's CU
 * count). For running stages of a pipeline side by side on disjoint shares of
 * the chip (for example one step's eigendecomposition beside the next step's
 * binning and smoothing). The runtime spreads consecutive mask bits over the
 * XCDs and refuses a mask that leaves one of them without a CU: on MI355X
 * (256 CUs) the top 64 bits give 8 CUs on each XCD. Returns the stream in
 * *stream (a hipStream_t, owned by the caller: fpca_stream_destroy);
 * FPCA_ERR_INVALID_ARG for a bad device or range, FPCA_ERR_UNSUPPORTED when
 * the runtime refuses the mask. */
int fpca_stream_create_cu_range(int device, int cu_begin, int cu_end, void **stream);
int fpca_stream_destroy(void *stream);
/* Waits for the handle's stream; returns FPCA_ERR_DOMAIN (and clears the flag)
 * if a binning call met an observation outside [0,1]^d since the last sync. */
int fpca_sync(fpca_handle handle);
/* Message of the last nonzero code returned on this host thread. */
const char *fpca_last_error(void);

/*
 * fpca_bin -- linear binning (Section 3.2; the weights of eqs. 2.3 and 2.4).
 * Each observation point spreads onto its 2^d surrounding grid nodes with
 * multilinear weights W_p(t): per coordinate u = t*(M-1) (one FP64 multiply),
 * lower node k = min(floor(u), M-2), weights 1-(u-k) and u-k.
 *
 * kind = FPCA_BIN_MEAN (eq. 2.3, curve weight w_i = 1/N_i):
 *   weights[p] = sum_i w_i sum_j W_p(t_ij)         (P entries)
 *   sums[p]    = sum_i w_i sum_j W_p(t_ij) Y_ij
 *   sq_sums[p] = sum_i w_i sum_j W_p(t_ij) Y_ij^2  (optional; the responses of eq. 2.5)
 * kind = FPCA_BIN_COV (eq. 2.4, ordered pairs j != l, w_i = 1/(N_i(N_i-1)),
 *   curves with N_i < 2 contribute nothing):
 *   weights[p,q] = sum_i w_i sum_{j!=l} W_p(t_ij) W_q(t_il)   (P x P)
 *   sums[p,q]    = ... times Y_ij Y_il
 *   sq_sums[p,q] = ... times (Y_ij Y_il)^2  (optional; used by cross-validation)
 *   With folds (fold_of_curve != NULL, n_folds >= 1) each of these arrays holds
 *   n_folds+1 consecutive P x P slabs: slab 0 over all curves, slab f+1 over the
 *   curves of fold f only. Such a call waits for the handle's stream once (it
 *   reads the n_folds+1 fold boundaries back to size each fold's product), so
 *   it cannot be captured in a graph; without folds nothing synchronizes.
 *
 * design = FPCA_IRREGULAR: offsets[n+1] (int64, offsets[0] = 0, nondecreasing)
 *   delimit curve i's observations; t is N x d row-major and y has N entries,
 *   N = offsets[n], both of storage dtype `dtype`.
 * design = FPCA_COMMON_GRID: every curve is observed at all P nodes; offsets and
 *   t must be NULL and y is the n x P row-major matrix of values. The pair
 *   weights are then n/(P(P-1)) off the diagonal and 0 on it; for kind = COV
 *   `weights` may be NULL, and they are then not written (fpca_smooth_cov
 *   takes them as C = NULL with c_uniform = n/(P(P-1))).
 * dtype: FPCA_F64 or FPCA_F32 storage of t, y and every value output.
 * prec (kind = COV only, the Gram product): FPCA_PREC_F64 (dtype F64),
 *   FPCA_PREC_F32 (FP32 products, FP32 accumulation) or FPCA_PREC_BF16X3
 *   (each FP32 operand split into bf16 hi + lo, three bf16 products, FP32
 *   accumulation). Ignored for kind = MEAN.
 * bin_index: optional, N int32 flat lower-corner node of each observation
 *   (irregular only). cell_count: optional int64, P entries (MEAN: observations
 *   per lower corner) or P x P (COV: ordered pairs per pair of lower corners,
 *   over all curves with N_i >= 2). Both are exact integers.
 * Returns FPCA_ERR_UNSUPPORTED for COV with P > 8192.
 */
int fpca_bin(fpca_handle handle, const fpca_grid *grid, int kind, int design, int dtype, int prec,
             int64_t n, const int64_t *offsets, const void *t, const void *y,
             const int32_t *fold_of_curve, int n_folds, void *weights, void *sums, void *sq_sums,
             int32_t *bin_index, int64_t *cell_count);

/*
 * fpca_bin_common -- both binnings of n complete common-grid curves (eqs. 2.3
 * and 2.4) in one call: the results of fpca_bin(kind = FPCA_BIN_MEAN,
 * FPCA_COMMON_GRID) into (mean_weights, mean_sums, mean_sq_sums) and of
 * fpca_bin(kind = FPCA_BIN_COV, FPCA_COMMON_GRID) into (cov_weights,
 * cov_sums), bit for bit. With dtype FPCA_F32 and prec FPCA_PREC_BF16X3 the
 * Gram product's pass that splits Y into bf16 hi/lo also forms the mean's
 * column sums, so Y (n x P) is read once for both; other combinations run
 * the two binnings one after the other.
 *   y: device, n x P row-major of `dtype`; mean_weights, mean_sums: P;
 *   mean_sq_sums: P or NULL; cov_weights: P x P or NULL (the pair weights,
 *   materialized only when given); cov_sums: P x P. Errors as fpca_bin.
 */
int fpca_bin_common(fpca_handle handle, const fpca_grid *grid, int dtype, int prec, int64_t n, const void *y,
                    void *mean_weights, void *mean_sums, void *mean_sq_sums, void *cov_weights, void *cov_sums);

/*
 * fpca_smooth_mean -- binned local-linear smoother of the mean (eq. 2.3):
 * at every node x, b0 of the weighted least-squares fit of the binned sums
 * with weights K((y-x)/h) and regressors (y-x)/h, solved in FP64:
 *   [[S0, S1^T], [S1, S2]] beta = [T0; T1],  mu[x] = beta_0,
 * with S0 = sum weights K, S1 = sum weights K u, S2 = sum weights K u u^T,
 * T0 = sum sums K, T1 = sum sums K u over the window |y_k - x_k| <= h_k.
 *   weights, sums: P entries of `dtype` (from fpca_bin kind MEAN).
 *   bandwidth: host array of d bandwidths h_k > 0.
 *   mu: P outputs of `dtype`; status: optional P int8 (FPCA_STATUS_*).
 * Status rule: EMPTY if S0 == 0; FALLBACK if a diagonal entry is 0 or the
 * Jacobi-scaled Cholesky factorization has a pivot below 1e-10; else OK.
 * Precision: the moments are accumulated and the system solved in FP64 for
 * either storage dtype, so windows that are exactly degenerate (sparse bins,
 * data on one side of the node) are recognized as such.
 */
int fpca_smooth_mean(fpca_handle handle, const fpca_grid *grid, int dtype, const void *weights,
                     const void *sums, int kernel, const double *bandwidth, void *mu,
                     int8_t *status);

/*
 * fpca_set_conv -- how the general smoother (fpca_smooth_mean, and
 * fpca_smooth_cov on grids the task-queue smoother does not take) forms its
 * 1-D moment passes: FPCA_CONV_DIRECT sums the 2R+1 taps per output
 * (default); FPCA_CONV_FFT uses the FFT strategy of Section 3.2 on binned data
 * (per line of the pass, the zero-padded line and the taps are transformed
 * with L >= M + R points, L a power of two up to 4096, multiplied and
 * transformed back; passes with M + R > 4096 stay direct); FPCA_CONV_AUTO
 * times both the first time a pass shape is met on this handle and keeps the
 * faster (no timing while the stream is being captured: direct then).
 * The FFT pass agrees with the direct one to FP64 rounding relative to the
 * largest value of the line; values below 1e-12 of (max |line| x sum |taps|)
 * are set to 0, which keeps empty windows empty.
 */
#define FPCA_CONV_DIRECT 0
#define FPCA_CONV_FFT 1
#define FPCA_CONV_AUTO 2
int fpca_set_conv(fpca_handle handle, int mode);

/*
 * fpca_set_engine -- which engine smooths the covariance for general pair
 * weights (fpca_smooth_cov with C given, fpca_cv_batched; fpca_cv_loo always
 * runs the queue kernel):
 * FPCA_ENGINE_QUEUE is the persistent task-queue kernel (one launch, FP64
 * moments kept on chip between passes; grids of P <= 4096 with M <= 64 for
 * d = 1, 32 x 64 for d = 2, 16^3 for d = 3); FPCA_ENGINE_PASSES the 1-D pass
 * engine (FP64 moment arrays in device memory between passes, any grid);
 * FPCA_ENGINE_AUTO (default) takes the queue kernel when the pass engine's
 * arrays would not fit in the 256 MB Infinity Cache, and batched CV also
 * times the job-by-job pass engine against the queue kernel's tile shapes.
 * Both engines compute the same sums in FP64 (results agree to rounding).
 */
#define FPCA_ENGINE_AUTO 0
#define FPCA_ENGINE_QUEUE 1
#define FPCA_ENGINE_PASSES 2
int fpca_set_engine(fpca_handle handle, int engine);

/*
 * fpca_smooth_cov -- the covariance (eq. 2.4): the same smoother on the
 * 2d-dimensional grid of (s, t) pairs, applied to the pair weights C and raw
 * products G from fpca_bin kind COV (slab 0), giving b0(s,t), then
 *   gamma[p,q] = (b0(p,q) + b0(q,p))/2 - mu[p] mu[q],
 * and gamma = 0 where node p or q lies outside the grid's mask (Section 3.1).
 *   C: P x P pair weights, or NULL for a complete common-grid design, whose
 *      pair weights are c_uniform off the diagonal and 0 on it (c_uniform =
 *      n/(P(P-1)) for n curves observed at all P nodes, matching fpca_bin).
 *   c_uniform: the off-diagonal pair weight used when C is NULL (> 0);
 *      ignored otherwise.
 *   G: P x P raw products. mu: P values of the mean on this grid, or NULL to
 *      return the raw second-moment surface b0 (symmetrized) instead.
 *   bandwidth: host array of d bandwidths; the s- and t-coordinates share them.
 *   gamma: P x P output of `dtype`; status: optional P x P int8.
 * Precision: with C given, FP64 moments and solve (as for the mean). With
 * C = NULL and dtype F32 on a d = 2 grid, the weight moments are exact FP64
 * closed forms and the response moments FP32 sums; only b0 at p <= q is
 * evaluated and mirrored, the two fits being equal in exact arithmetic.
 */
int fpca_smooth_cov(fpca_handle handle, const fpca_grid *grid, int dtype, const void *C,
                    double c_uniform, const void *G, const void *mu, int kernel,
                    const double *bandwidth, void *gamma, int8_t *status);

/*
 * fpca_eig_randomized -- top-k eigenpairs of the matrixized covariance
 * (Section 3.1): A = W^1/2 Gamma W^1/2 with quadrature weights w_p, by random
 * projection (Section 3.4) read as a randomized range finder:
 *   Omega_g = P x r standard normal test matrix, r = k + oversample;
 *   Q = orth(A Omega_g); power_iters times: Q = orth(A Q), Q = orth(A Q);
 *   B = Q^T A Q; B = U diag(theta) U^T; psi = Q U.
 * orth is CholeskyQR in FP64 (one pass between products, two passes for the
 * Rayleigh-Ritz basis); columns whose Cholesky pivot falls below 1e-12 of
 * their squared norm are dropped (set to zero) and left out of B.
 * The eigenvalues are the top k theta in descending order; eigenfunctions are
 * rescaled as phi = psi / sqrt(w) so that sum_p w_p phi_p^2 = 1, with the sign
 * chosen so that sum_p w_p phi_p > 0 (if that sum is below 1e-8 sum_p w_p |phi_p|,
 * the lowest-index entry within a relative 1e-6 of max |phi| is made positive).
 * fve[l] = sum_{m<=l} theta_m / sum of the positive theta over all r Ritz values
 * (0 when no Ritz value is positive). Beyond the numerical rank (fewer kept
 * basis columns than k) the eigenvalues and eigenfunctions are 0.
 * Test matrix: entry (p, j) is standard normal number j*P + p of stream `seed`,
 * drawn by the Box-Muller cosine branch from two splitmix64 outputs.
 *   gamma: P x P (P = prod grid->M) symmetric, `dtype`.
 *   quad_w: optional device array of P FP64 weights; NULL means the Riemann
 *     weights prod_k 1/(M_k-1), set to 0 outside the grid's mask.
 *   prec: FPCA_PREC_F64 (dtype F64); for dtype F32, FPCA_PREC_F32 (FP32
 *     products of A with the basis) or FPCA_PREC_BF16X3 (the same products
 *     with A and the basis split as x = hi + lo in bf16, hi*hi + hi*lo + lo*hi
 *     with FP32 accumulation: relative error of each product entry of order
 *     1e-5, eigenvalues within 1e-4 of the largest). The orthonormalization
 *     and the Rayleigh-Ritz step are FP64 in every case. FPCA_PREC_BF16X3
 *     reads gamma by rows (it must be exactly symmetric).
 *   k >= 1, oversample >= 0, k + oversample <= min(64, P).
 *   evals: host, k doubles. efuns: device, P x k column-major of `dtype`.
 *   fve: host, k doubles, or NULL. Synchronizes the handle's stream.
 */
int fpca_eig_randomized(fpca_handle handle, int dtype, int prec, const fpca_grid *grid,
                        const void *gamma, const double *quad_w, int k, int oversample,
                        int power_iters, uint64_t seed, double *evals, void *efuns, double *fve);

/*
 * The smoothed covariance of complete common-grid data as an operator
 * (Section 3.2's blockwise processing with the products of Section 3.4): the
 * P x P covariance Gamma_hat of eq. 2.4 (pair weights of the complete design,
 * the binned local-linear fit, Gamma = b0 - mu mu^T, symmetric to rounding)
 * is never stored; products Gamma_hat X are formed from the curves. For
 * covariance nodes whose s- and t-windows share no grid node the fit has a
 * closed form that factors over s and t, so off the band |s - t| <= 2R (per
 * coordinate) Gamma_hat has rank <= 2n + 1; on the band every node's
 * (2d+1)-moment system is solved in FP64 with the diagonal pairs removed.
 *
 * fpca_covop_create -- builds the operator.
 *   grid: d = 1..3, no mask; Y: device, n x P row-major FP64, every curve
 *     observed at every node (no NaN); mu: device, P FP64 (the smoothed mean,
 *     e.g. from fpca_smooth_mean), copied; bandwidth: host, d values shared by
 *     the s- and t-coordinates; each coordinate's window must span 1..R_max
 *     grid steps (R_max = 2016, 28, 6 for d = 1, 2, 3) and be non-degenerate
 *     at every node, else FPCA_ERR_UNSUPPORTED.
 *   mode: FPCA_COVOP_RECOMPUTE (the band is recomputed tile by tile in every
 *     product; the operator holds O(n P) memory) or FPCA_COVOP_STORE_BAND (the
 *     band is formed once and kept in 64 x 64 FP64 blocks, about
 *     P x 64 x prod_k (2 ceil(2R_k / b_k) + 1) doubles with tile extents
 *     b = 64 / 8 / 4 for d = 1 / 2 / 3; products then stream it).
 *   The operator allocates its own device memory (FPCA_ERR_WORKSPACE if it
 *   does not fit), keeps the handle, and uses the handle's stream at each
 *   call. Synchronizes the stream.
 * fpca_covop_apply -- out = Gamma_hat X; X, out: device, P x r row-major FP64
 *   (node-major), 1 <= r <= 64; asynchronous on the handle's stream.
 * fpca_covop_destroy -- waits for the handle's stream and frees the operator.
 * fpca_eig_covop -- fpca_eig_randomized (same algorithm, test matrix,
 *   orthonormalization, rescaling and sign rule, FP64) with every product
 *   taken through the operator; quad_w NULL means the Riemann weights.
 *   efuns: device, P x k column-major FP64.
 */
typedef struct fpca_covop_s *fpca_covop;
#define FPCA_COVOP_RECOMPUTE 0
#define FPCA_COVOP_STORE_BAND 1
int fpca_covop_create(fpca_handle handle, const fpca_grid *grid, int64_t n, const double *Y, const double *mu,
                      const double *bandwidth, int mode, fpca_covop *op);
int fpca_covop_apply(fpca_covop op, int r, const double *X, double *out);
int fpca_covop_destroy(fpca_covop op);
int fpca_eig_covop(fpca_covop op, const double *quad_w, int k, int oversample, int power_iters, uint64_t seed,
                   double *evals, double *efuns, double *fve);

/*
 * fpca_noise_variance -- measurement-error variance (eq. 2.6, from the
 * smooth of eq. 2.5). At every node t of `grid` (P nodes):
 *   sigma2_t[t] = b0[t] - gamma[t, t] - mu[t]^2
 * where b0 is fpca_smooth_mean applied to the weights and sq_sums of
 * fpca_bin(kind = MEAN) (the squared responses of eq. 2.5, curve weight
 * 1/N_i) with the bandwidth h_sigma, mu the smoothed mean and gamma the P x P
 * covariance of fpca_smooth_cov, all on the same grid. b0 estimates
 * E Y^2 = mu^2 + Gamma(t,t) + sigma^2, so mu^2 is subtracted; the paper
 * prints the product with a plus sign. Nodes outside Omega (grid mask) get 0
 * and are not counted; a node whose value is not finite (an EMPTY window of
 * either smoother) keeps NaN and is not counted.
 *   sigma2: host, one double: the average of sigma2_t over the counted nodes
 *     (the integral over Omega divided by the volume of Omega, as a node
 *     average); NaN when no node counts.
 *   count: host int64 (or NULL): the number of counted nodes.
 *   b0, mu: device, P values of `dtype`; gamma: device, P x P of `dtype`;
 *   sigma2_t: device, P values of `dtype`, or NULL. The sum is FP64 in a
 *   fixed order. Synchronizes the handle's stream.
 */
int fpca_noise_variance(fpca_handle handle, const fpca_grid *grid, int dtype, const void *b0, const void *mu,
                        const void *gamma, void *sigma2_t, double *sigma2, int64_t *count);

/*
 * fpca_pace_scores -- principal component scores by conditional expectation
 * (eq. 2.7): for every curve i,
 *   xi_i = Lambda Phi_i^T Sigma_i^{-1} (Y_i - mu_i),
 *   Sigma_i = Phi_i Lambda Phi_i^T + sigma2 I,
 * with Phi_i[j][l] = efuns_l(t_ij) and mu_i[j] = mu(t_ij) interpolated from
 * the grid by the multilinear corner weights of linear binning (the rule of
 * fpca_bin). Computed per curve as the k x k system
 *   (Phi_i^T Phi_i + sigma2 Lambda^{-1}) xi_i = Phi_i^T (Y_i - mu_i)
 * (the same result by the push-through identity), FP64 accumulation and
 * Cholesky solve. Components with evals[l] <= 0 are left out of Sigma_i and
 * score 0. Observations with t outside [0,1]^d, or a non-finite y, are left
 * out; a curve with none scores 0.
 *   design, n, offsets, t, y: as in fpca_bin (common grid: y is n x P with
 *     NaN for a missing value, offsets = t = NULL).
 *   mu: device, P values; efuns: device, P x k column-major (the output of
 *     fpca_eig_randomized); evals: host, k doubles; sigma2 > 0 (for example
 *     from fpca_noise_variance).
 *   scores: device, n x k row-major, of `dtype`.
 * Returns FPCA_ERR_INVALID_ARG for k outside 1..32 or sigma2 not positive.
 */
int fpca_pace_scores(fpca_handle handle, const fpca_grid *grid, int design, int dtype, int64_t n,
                     const int64_t *offsets, const void *t, const void *y, const void *mu, const void *efuns,
                     int k, const double *evals, double sigma2, void *scores);

/*
 * fpca_pace_scores_noalloc -- fpca_pace_scores for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, same kernels and the same
 * results, but no allocation of any kind. The common-grid design's shared
 * k x k inverse, the partial sums it is formed from and two flags live in a
 * fixed per-GPU array of 57,856 bytes (k <= 32, the limit of
 * fpca_pace_scores, so every valid call fits), set up by fpca_create and held
 * until the process ends; the irregular design needs none. Every call on one
 * GPU uses that GPU's array: calls that overlap in time on one GPU (several
 * streams or handles) race and must be serialized by the caller. Errors as
 * for fpca_pace_scores.
 */
int fpca_pace_scores_noalloc(fpca_handle handle, const fpca_grid *grid, int design, int dtype, int64_t n,
                             const int64_t *offsets, const void *t, const void *y, const void *mu,
                             const void *efuns, int k, const double *evals, double sigma2, void *scores);

/*
 * fpca_reconstruct -- curves on the grid from their scores (the display after
 * eq. 2.7): xhat[i][p] = mu[p] + sum_{l < k} scores[i][l] efuns_l[p].
 *   mu: device, P; efuns: device, P x k column-major; scores: device, n x k
 *   row-major (fpca_pace_scores); xhat: device, n x P row-major; all of
 *   `dtype`, FP64 accumulation. k in 1..32.
 */
int fpca_reconstruct(fpca_handle handle, int dtype, int64_t P, int64_t n, int k, const void *mu,
                     const void *efuns, const void *scores, void *xhat);

/*
 * fpca_cv_batched -- bandwidth selection for the covariance smoother by
 * leave-curves-out cross-validation (the CV idea of Section 3.3, on folds of
 * curves and binned data), over several datasets at once. For every dataset
 * a, bandwidth h (row of `bandwidths`) and fold f, the smoother of eq. 2.4 is
 * fitted to the pairs of the curves outside fold f, C - C_f and G - G_f,
 * giving Ghat (symmetrized, 0 outside the dataset's mask); the held-out pairs
 * are scored through their bins:
 *   scores[(a * n_h + h) * n_folds + f] = sum_{p,q} Q_f - 2 G_f Ghat + C_f Ghat^2
 * (= sum over held-out pairs of w (Y_ij Y_il - Ghat)^2 spread over the pair's
 * bins; Ghat is taken as 0 where the window is empty), accumulated in FP64.
 *   data: host array of n_data datasets. Each has its own grid (and mask;
 *     every dataset has the same d, grid sizes may differ) and its C, G, Q:
 *     (n_folds+1) x P x P device arrays of `dtype` from fpca_bin(kind = COV)
 *     with folds and sq_sums (slab 0 all curves, slab f+1 fold f).
 *   bandwidths: host, n_h x d, shared by the datasets. scores: host,
 *     n_data x n_h x n_folds.
 * All jobs run in one persistent launch on the handle's stream (moments and
 * solves in FP64); the tile shape is chosen by timing on the first call with a
 * shape, the second call captures the launch into a HIP graph and later calls
 * replay it. Grids with more than 4096 nodes, or a first coordinate longer
 * than the launch's LDS allows (d = 1: 64, d = 2: 32, d = 3: 16), run job by
 * job instead. Synchronizes; FPCA_ERR_DEVICE if a task of the launch waited
 * past its spin limit.
 */
typedef struct {
  fpca_grid grid;
  const void *C, *G, *Q;
} fpca_cv_data;

int fpca_cv_batched(fpca_handle handle, int dtype, int n_data, const fpca_cv_data *data, int n_folds, int n_h,
                    const double *bandwidths, double *scores);

/*
 * fpca_cv_select -- the selected bandwidth from a CV curve (host only): the
 * grid minimizer of cv[n_h] (scores summed over folds), refined by the vertex
 * of the parabola through it and its two neighbours in log h when the minimum
 * is interior and the parabola opens upward (clamped to the neighbours). The
 * rows of `bandwidths` (n_h x d) must be positive multiples of one vector,
 * increasing; the refinement moves along that ray. h_out: d doubles.
 */
int fpca_cv_select(int n_h, int d, const double *bandwidths, const double *cv, double *h_out);

/*
 * fpca_cv_loo -- the bandwidth criterion of Section 3.3: leave-one-observation-
 * out cross-validation of the covariance smoother, read on binned data as
 * leave-one-bin-out. For every bandwidth row h, at every node x of the
 * 2d-dimensional grid the local-linear fit of eq. 2.4 is computed with x's own
 * bin left out (its pair weight and sum leave S0 and T0; the other moments are
 * unchanged because u = 0 there), b_{-x}(x), and
 *   scores[h] = sum_x Q(x) - 2 G(x) b_{-x}(x) + C(x) b_{-x}(x)^2
 * with b_{-x} = 0 where the reduced window is empty or x lies outside the
 * mask (= sum over pairs of w (Y_ij Y_il - b)^2 spread over their bins; it is
 * exactly leave-one-observation-out CV when every bin holds one pair on its
 * node). FP64 moments and solves, FP64 sum. One persistent launch per call.
 *   C, G, Q: P x P device arrays of `dtype` (fpca_bin kind COV with sq_sums,
 *     without folds). bandwidths: host, n_h x d. scores: host, n_h.
 * Grids: P <= 4096 and M_1 <= 64 (d = 1), 32 (d = 2), 16 (d = 3); otherwise
 * FPCA_ERR_UNSUPPORTED. Synchronizes.
 */
int fpca_cv_loo(fpca_handle handle, const fpca_grid *grid, int dtype, const void *C, const void *G, const void *Q,
                int n_h, const double *bandwidths, double *scores);

/*
 * fpca_bw_search -- the bandwidth search of Section 3.3: fpca_cv_loo minimized
 * over continuous per-coordinate bandwidths (the s- and t-coordinates share
 * them) by a derivative-free trust-region method in log h whose local model is
 * a quadratic least-squares regression on the sampled criterion (the paper's
 * replacement of the interpolation step, the criterion being noisy).
 * Initial radius 0.25 x the widest side of the log box (within [0.05, 1]);
 * initial design: the start, +-r e_k, +-r/2 e_k, start + r/2 (e_k + e_l);
 * model fitted to the samples within 2r (max norm) of the centre, or to the
 * (d+1)(d+2)/2 + 1 nearest; the step minimizes the model in the ball of
 * radius r; accepted when the actual/predicted decrease is at least 0.1
 * (radius doubled at 0.75 when the step reaches 0.9 r), else the radius is
 * halved and a geometry sample centre + r e_k is added; stop when r < 0.01 or
 * after max_evals criteria. Candidates are clipped to [h_lo, h_hi]; the best
 * sample wins. Each iteration's 1-2 criteria are one launch.
 *   h_lo, h_hi, h_init: host, d each (0 < h_lo <= h_hi). max_evals >= the
 *   initial design (1 + 4d + d(d-1)/2). h_out: host, d. cv_out, n_evals:
 *   host, or NULL. trace: host, max_evals x (d + 1) (h and criterion of every
 *   sample in order), or NULL. Synchronizes.
 */
int fpca_bw_search(fpca_handle handle, const fpca_grid *grid, int dtype, const void *C, const void *G,
                   const void *Q, const double *h_lo, const double *h_hi, const double *h_init, int max_evals,
                   double *h_out, double *cv_out, int *n_evals, double *trace);

/*
 * Bandwidth surrogate (an addition to the paper's method, whose Section 3.3
 * selects bandwidths by CV with a trust-region search): a small MLP maps 32
 * summary features of the binned arrays to log h of the covariance smoother.
 * It is trained on datasets labelled by fpca_cv_batched, which remains the
 * fallback. FP32 throughout.
 *
 * fpca_bw_features: features of one dataset (FP32 binned arrays of this
 *   library): curve-size statistics from offsets[n+1]; mean-bin statistics
 *   from c, s, s2 (P; s2 = sq_sums of MEAN binning, may be NULL); pair-weight
 *   density, lag-0 raw product, noise fraction and raw-product variogram at
 *   lags 1..8 along the first and last coordinates from C, G (P x P) and Q
 *   (sq_sums of COV binning, may be NULL). feat: device, 32 floats.
 * fpca_bw_num_params: number of MLP parameters (20865), laid out as
 *   W1[128][32] b1[128] W2[128][128] b2[128] W3[128] b3[1].
 * fpca_bw_mlp_forward: out[b] = W3 gelu(W2 gelu(W1 x_b + b1) + b2) + b3 with
 *   x_b = (feat[b] - feat_mean) / feat_sd and the exact GELU z Phi(z); z1, z2
 *   (batch x 128 each, optional together) receive the pre-activations.
 * fpca_bw_mlp_backward: gradient of mean_b (out[b] - target[b])^2 with
 *   respect to the parameters, from the forward pass's out, z1, z2; work is a
 *   device scratch of batch*(2*128+1) floats; grad has fpca_bw_num_params()
 *   floats. Deterministic (fixed summation order).
 * fpca_bw_adam_step: one Adam update (step >= 1 counts updates) with
 *   decoupled weight decay; m and v are the moment buffers.
 */
int fpca_bw_features(fpca_handle handle, const fpca_grid *grid, int64_t n, const int64_t *offsets,
                     const float *c, const float *s, const float *s2, const float *C, const float *G,
                     const float *Q, float *feat);
int fpca_bw_num_params(void);
int fpca_bw_mlp_forward(fpca_handle handle, int batch, const float *feat, const float *feat_mean,
                        const float *feat_sd, const float *params, float *out, float *z1, float *z2);
int fpca_bw_mlp_backward(fpca_handle handle, int batch, const float *feat, const float *feat_mean,
                         const float *feat_sd, const float *params, const float *out,
                         const float *target, const float *z1, const float *z2, float *work,
                         float *grad);
int fpca_bw_adam_step(fpca_handle handle, int step, float lr, float beta1, float beta2, float eps,
                      float weight_decay, float *params, const float *grad, float *m, float *v);

/* Standard normal numbers 0..count-1 of stream `seed` (the test-matrix
 * generator above), FP64, into the device array out. */
int fpca_rng_normal(fpca_handle handle, uint64_t seed, int64_t count, double *out);

#ifdef __cplusplus
}
#endif

#endif /* FPCA_H */

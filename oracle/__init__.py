"""FP64 CPU oracle for the binned local-linear FPCA hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the HIP library never does, and this
package imports nothing from it. The heavy loops live in `fpca_oracle.c`
(plain C, FP64, no FP contraction); this module marshals numpy arrays and adds
the steps for which a library primitive is the plain definition (a matrix
product, a Householder QR, a symmetric eigensolver).

Each function names the passage of the paper it follows:
  - linear binning: Section 3.2 (binning strategy for irregular designs);
  - mean smoother: eq. (2.3); covariance smoother: eq. (2.4);
  - noise variance: eq. (2.6), from the smooth of eq. (2.5);
  - principal component scores: eq. (2.7); reconstruction after it;
  - matrixization and rescaling: Section 3.1, eq. (3.1);
  - random projection: Section 3.4;
  - bandwidth search (leave-one-out CV by a trust region with a quadratic
    regression model): Section 3.3, in `oracle/bw_search.py`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

from .build import LIB_PATH, build_oracle

ST_OK, ST_FALLBACK, ST_EMPTY = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_oracle()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        L.orc_bin_corners.argtypes = [I, P, I64, P, P, P, P]
        L.orc_bin_mean.argtypes = [I, P, I64, P, P, P, P, P, P, P]
        L.orc_bin_cov_pairs.argtypes = [I, P, I64, P, P, P, P, I, P, P, P, P]
        L.orc_smooth.argtypes = [I, P, P, P, P, I64, P, P, P, P, P]
        L.orc_wls_from_moments.argtypes = [I, I64, P, P, P, P]
        L.orc_num_moments.argtypes = [I]
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, I64, P]
        L.orc_normals.argtypes = [ctypes.c_uint64, I64, P]
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(rc):
    if rc == -2:
        raise ValueError("observation outside [0,1]^d or NaN")
    if rc != 0:
        raise ValueError(f"oracle error {rc}")


def grid_size(M: Sequence[int]) -> int:
    return int(np.prod(M))


# ----------------------------------------------------------------- binning
def bin_corners(M, t):
    """Corner nodes, weights and lower-corner index of each observation (Section 3.2)."""
    d = len(M)
    t = _c(np.asarray(t).reshape(-1, d), np.float64)
    N = t.shape[0]
    nc = 1 << d
    node = np.zeros((N, nc), np.int64)
    wt = np.zeros((N, nc), np.float64)
    lower = np.zeros(N, np.int64)
    Mi = _c(M, np.int32)
    _check(lib().orc_bin_corners(d, _p(Mi), N, _p(t), _p(node), _p(wt), _p(lower)))
    return node, wt, lower


def bin_mean(M, offsets, t, y):
    """Binned weights and sums for the mean smoother (eq. 2.3, weights 1/N_i).

    Returns c[P], s[P], bin_index[N] (int32 flat lower corner), cell_count[P] (int64)."""
    d = len(M)
    P = grid_size(M)
    offsets = _c(offsets, np.int64)
    t = _c(np.asarray(t).reshape(-1, d), np.float64)
    y = _c(y, np.float64)
    c = np.zeros(P)
    s = np.zeros(P)
    idx = np.zeros(t.shape[0], np.int32)
    cnt = np.zeros(P, np.int64)
    Mi = _c(M, np.int32)
    _check(lib().orc_bin_mean(d, _p(Mi), len(offsets) - 1, _p(offsets), _p(t), _p(y), _p(c),
                              _p(s), _p(idx), _p(cnt)))
    return c, s, idx, cnt


def bin_cov_pairs(M, offsets, t, y, folds=None, fold_sel=-1, want_Q=False, want_cnt=False):
    """Covariance binning by explicit ordered-pair loops j != l (eq. 2.4, weights
    1/(N_i(N_i-1))). Returns C, G (P x P), and optionally Q (squared raw products,
    for cross-validation) and the int64 pair-cell counts."""
    d = len(M)
    P = grid_size(M)
    offsets = _c(offsets, np.int64)
    t = _c(np.asarray(t).reshape(-1, d), np.float64)
    y = _c(y, np.float64)
    C = np.zeros((P, P))
    G = np.zeros((P, P))
    Q = np.zeros((P, P)) if want_Q else None
    cnt = np.zeros((P, P), np.int64) if want_cnt else None
    f = _c(folds, np.int32) if folds is not None else None
    Mi = _c(M, np.int32)
    _check(lib().orc_bin_cov_pairs(d, _p(Mi), len(offsets) - 1, _p(offsets), _p(t), _p(y), _p(f),
                                   int(fold_sel), _p(C), _p(G), _p(Q), _p(cnt)))
    out = [C, G]
    if want_Q:
        out.append(Q)
    if want_cnt:
        out.append(cnt)
    return tuple(out)


def bin_cov_identity(M, offsets, t, y, folds=None, fold_sel=-1, want_Q=False, want_cnt=False):
    """Covariance binning by the Gram identity
        G = sum_i w_i (z_i z_i^T - sum_j Y_ij^2 b_ij b_ij^T),  z_i = sum_j b_ij Y_ij,
    (b_ij the linear-binning weight vector of t_ij), and likewise C with Y = 1 and
    Q with Y^2. Algebraically equal to the pair loops; used at sizes where the
    pair loops are too slow."""
    d = len(M)
    P = grid_size(M)
    offsets = np.asarray(offsets, np.int64)
    n = len(offsets) - 1
    Ni = np.diff(offsets)
    node, wt, lower = bin_corners(M, t)
    y = np.asarray(y, np.float64)
    curve = np.repeat(np.arange(n), Ni)
    sel = np.ones(n, bool)
    if folds is not None and fold_sel >= 0:
        sel = np.asarray(folds) == fold_sel
    w = np.where((Ni >= 2) & sel, 1.0 / np.maximum(Ni * (Ni - 1), 1).astype(np.float64), 0.0)
    nc = node.shape[1]
    rows_idx = (curve[:, None] * P + node).reshape(-1)

    def rows(vals):
        R = np.zeros(n * P)
        np.add.at(R, rows_idx, (wt * vals[:, None]).reshape(-1))
        return R.reshape(n, P)

    def gram(vals, corr_vals):
        R = rows(vals)
        A = (R * w[:, None]).T @ R
        wo = w[curve]
        uu = np.repeat(node, nc, axis=1).reshape(-1)
        vv = np.tile(node, (1, nc)).reshape(-1)
        ww = (np.repeat(wt, nc, axis=1) * np.tile(wt, (1, nc))).reshape(len(curve), nc * nc)
        ww = (ww * (wo * corr_vals)[:, None]).reshape(-1)
        np.subtract.at(A, (uu, vv), ww)
        return A

    ones = np.ones_like(y)
    C = gram(ones, ones)
    G = gram(y, y * y)
    out = [C, G]
    if want_Q:
        out.append(gram(y * y, y ** 4))
    if want_cnt:
        cnt_rows = np.zeros((n, P), np.int64)
        np.add.at(cnt_rows, (curve, lower), 1)
        cnt_rows[~(sel & (Ni >= 2))] = 0
        cnt = cnt_rows.T @ cnt_rows
        diag = np.zeros((P, P), np.int64)
        ok = (sel & (Ni >= 2))[curve]
        np.add.at(diag, (lower[ok], lower[ok]), 1)
        out.append(cnt - diag)
    return tuple(out)


def bin_common_grid_mean(Y):
    """Mean part of bin_common_grid (c = n/P, s = column sums / P), without the
    pair sums, for sizes where the Gram product is not needed."""
    Y = np.asarray(Y, np.float64)
    n, P = Y.shape
    return np.full(P, n / P), Y.sum(0) / P


def bin_common_grid(Y):
    """Common-grid design: every curve observed at all P nodes, so each observation
    sits on a node (W = indicator). Mean: c = n/P, s = column sums / P.
    Covariance: C = n/(P(P-1)) off the diagonal and 0 on it; G = Y^T Y / (P(P-1))
    with the diagonal (the j = l terms) removed."""
    Y = np.asarray(Y, np.float64)
    n, P = Y.shape
    c = np.full(P, n / P)
    s = Y.sum(0) / P
    w = 1.0 / (P * (P - 1))
    G = (Y.T @ Y) * w
    np.fill_diagonal(G, 0.0)
    C = np.full((P, P), n * w)
    np.fill_diagonal(C, 0.0)
    return c, s, C, G


def bin_common_grid_entries(Y, p, q):
    """Entries G[p_i, q_i] of the common-grid pair sums (same definition as
    bin_common_grid: sum over curves of Y[:, p] Y[:, q] / (P(P-1)), zero on the
    diagonal), one dot product per entry, for sizes where the full product is
    too large."""
    Y = np.asarray(Y, np.float64)
    P = Y.shape[1]
    p = np.asarray(p, np.int64)
    q = np.asarray(q, np.int64)
    out = np.einsum("ij,ij->j", Y[:, p], Y[:, q]) / (P * (P - 1))
    out[p == q] = 0.0
    return out


# ----------------------------------------------------------------- smoothing
def num_moments(D: int) -> int:
    return 1 + D + D * (D + 1) // 2 + 1 + D


def smooth(dims, h, w, g, nodes=None, want_moments=False):
    """Binned local-linear smoother by direct window summation at the given flat
    node indices (all nodes if None). Returns b0, status (and moments, minpiv)."""
    dims = _c(dims, np.int32)
    D = len(dims)
    hh = _c(np.broadcast_to(np.asarray(h, np.float64), (D,)), np.float64)
    w = _c(w, np.float64).reshape(-1)
    g = _c(g, np.float64).reshape(-1)
    assert w.size == int(np.prod(dims)) and g.size == w.size
    nodes_a = None if nodes is None else _c(nodes, np.int64).reshape(-1)
    m = w.size if nodes_a is None else nodes_a.size
    b0 = np.zeros(m)
    st = np.zeros(m, np.int8)
    mp = np.zeros(m)
    mom = np.zeros((m, num_moments(D))) if want_moments else None
    _check(lib().orc_smooth(D, _p(dims), _p(hh), _p(w), _p(g), m, _p(nodes_a), _p(b0), _p(st),
                            _p(mom), _p(mp)))
    if want_moments:
        return b0, st, mom, mp
    return b0, st


def smooth_mean(M, h, c, s, nodes=None):
    """mu_hat = b0 of eq. (2.3) on the d-dimensional grid."""
    return smooth(tuple(M), h, c, s, nodes)


def smooth_cov_raw(M, h, C, G, nodes=None):
    """b0 of eq. (2.4) (the raw second-moment surface) on the 2d-dimensional grid.
    s- and t-coordinates share the bandwidth h."""
    d = len(M)
    hh = np.broadcast_to(np.asarray(h, np.float64), (d,))
    return smooth(tuple(M) + tuple(M), np.concatenate([hh, hh]), C, G, nodes)


def wls_from_moments(D, mom):
    mom = _c(mom, np.float64).reshape(-1, num_moments(D))
    m = mom.shape[0]
    b0 = np.zeros(m)
    st = np.zeros(m, np.int8)
    mp = np.zeros(m)
    _check(lib().orc_wls_from_moments(D, m, _p(mom), _p(b0), _p(st), _p(mp)))
    return b0, st, mp


def assemble_cov(Ghat, mu, mask=None):
    """Gamma_hat(s,t) = b0(s,t) - mu_hat(s) mu_hat(t) (eq. 2.4), zero where s or t
    lies outside the domain (Section 3.1), then symmetrized (Gamma + Gamma^T)/2."""
    Ghat = np.asarray(Ghat, np.float64)
    mu = np.asarray(mu, np.float64)
    Gam = Ghat - np.outer(mu, mu)
    if mask is not None:
        m = np.asarray(mask).astype(bool)
        Gam[~m, :] = 0.0
        Gam[:, ~m] = 0.0
    return 0.5 * (Gam + Gam.T)


def noise_variance(b0, mu, gamma, mask=None):
    """Measurement-error variance, eq. (2.6), from the smooth of eq. (2.5).

    b0 is the smooth of the squared responses Y_ij^2 with the mean's weights
    1/N_i (eq. 2.5), which estimates E Y^2 = mu^2 + Gamma(t,t) + sigma^2; so at
    every node sigma2(t) = b0(t) - Gamma(t,t) - mu(t)^2 (the paper prints the
    mean product with a plus sign; the minus sign is the reading used). The
    constant sigma^2 is the integral over Omega divided by the volume of
    Omega, taken as the average over the grid nodes of Omega where the value is
    finite. Nodes outside Omega get 0. Returns (sigma2_t, sigma2, count)."""
    b0 = np.asarray(b0, np.float64).reshape(-1)
    mu = np.asarray(mu, np.float64).reshape(-1)
    gamma = np.asarray(gamma, np.float64)
    P = b0.size
    assert mu.size == P and gamma.shape == (P, P)
    inside = np.ones(P, bool) if mask is None else np.asarray(mask).reshape(-1).astype(bool)
    s2t = np.where(inside, (b0 - np.diag(gamma)) - mu * mu, 0.0)
    counted = inside & np.isfinite(s2t)
    count = int(counted.sum())
    sigma2 = float(s2t[counted].sum() / count) if count else float("nan")
    return s2t, sigma2, count


def pace_scores(M, offsets, t, y, mu, efuns, evals, sigma2):
    """Principal component scores by conditional expectation (eq. 2.7),
    solved in the N_i x N_i form as written: xi_i = Lambda Phi_i^T Sigma_i^{-1}
    (Y_i - mu_i), Sigma_i = Phi_i Lambda Phi_i^T + sigma2 I, with phi_l and mu at
    t_ij interpolated by the corner weights of linear binning (Section 3.2).
    Components with evals <= 0 are left out (Lambda entry 0, score 0);
    observations outside [0,1]^d or with a non-finite y are left out.
    `offsets`/`t` None: common grid, y is n x P (NaN = missing).
    Returns scores [n, k]."""
    efuns = np.asarray(efuns, np.float64)
    P, k = efuns.shape
    mu = np.asarray(mu, np.float64).reshape(-1)
    lam = np.asarray(evals, np.float64)[:k]
    lam = np.where(np.isfinite(lam) & (lam > 0), lam, 0.0)
    if offsets is None:
        Y = np.asarray(y, np.float64)
        n = Y.shape[0]
        per_curve = [(np.arange(P)[np.isfinite(Y[i])], None, Y[i][np.isfinite(Y[i])]) for i in range(n)]
    else:
        d = len(M)
        tt = np.asarray(t, np.float64).reshape(-1, d)
        yy = np.asarray(y, np.float64).reshape(-1)
        inside = np.all((tt >= 0) & (tt <= 1), axis=1) & np.isfinite(yy)
        node, wt, _ = bin_corners(M, np.where(inside[:, None], tt, 0.0))
        per_curve = []
        for i in range(len(offsets) - 1):
            sl = np.arange(offsets[i], offsets[i + 1])
            sl = sl[inside[sl]]
            per_curve.append((node[sl], wt[sl], yy[sl]))
    out = np.zeros((len(per_curve), k))
    for i, (nd, w, yi) in enumerate(per_curve):
        if yi.size == 0:
            continue
        if w is None:
            Phi, mui = efuns[nd], mu[nd]
        else:
            Phi = np.einsum("jc,jcl->jl", w, efuns[nd])
            mui = (w * mu[nd]).sum(1)
        Sig = (Phi * lam) @ Phi.T + sigma2 * np.eye(yi.size)
        out[i] = lam * (Phi.T @ np.linalg.solve(Sig, yi - mui))
    return out


def reconstruct(mu, efuns, scores):
    """Curves on the grid from their scores (the display after eq. 2.7):
    X_i(t) = mu(t) + sum_l xi_il phi_l(t). Returns [n, P]."""
    return np.asarray(mu, np.float64)[None, :] + np.asarray(scores, np.float64) @ np.asarray(efuns, np.float64).T


# ----------------------------------------------------------------- eigen
def quad_weights(M, mask=None, rule="riemann"):
    """Quadrature weights omega_p of the Riemann sums of eq. (3.1):
    prod_k 1/(M_k-1) (rule 'riemann'), or the trapezoid rule; 0 outside the domain."""
    if rule == "riemann":
        w = np.full(grid_size(M), float(np.prod([1.0 / (m - 1) for m in M])))
    elif rule == "trapezoid":
        w = np.ones(1)
        for m in M:
            a = np.full(m, 1.0 / (m - 1))
            a[0] *= 0.5
            a[-1] *= 0.5
            w = np.multiply.outer(w, a).reshape(-1)
    else:
        raise ValueError(rule)
    if mask is not None:
        w = np.where(np.asarray(mask).astype(bool), w, 0.0)
    return w


def _rescale_and_sign(V, omega):
    """phi = psi / sqrt(omega) so that sum_p omega_p phi_p^2 = 1 (the rescaling of
    Section 3.1), with the sign fixed so that sum_p omega_p phi_p > 0; when that
    sum is below 1e-8 sum_p omega_p |phi_p|, the lowest-index entry whose |phi| is
    within a relative 1e-6 of max |phi| is made positive. Nodes with omega = 0
    get phi = 0."""
    sq = np.sqrt(omega)
    phi = np.zeros_like(V)
    nz = omega > 0
    phi[nz] = V[nz] / sq[nz, None]
    for j in range(phi.shape[1]):
        s = float(np.dot(omega, phi[:, j]))
        a = float(np.dot(omega, np.abs(phi[:, j])))
        if abs(s) >= 1e-8 * a:
            neg = s < 0
        else:
            mag = np.abs(phi[:, j])
            i = int(np.nonzero(mag >= (1.0 - 1e-6) * mag.max())[0][0])
            neg = phi[i, j] < 0
        if neg:
            phi[:, j] = -phi[:, j]
    return phi


def weighted_matrix(gamma, omega):
    sq = np.sqrt(np.asarray(omega, np.float64))
    return sq[:, None] * np.asarray(gamma, np.float64) * sq[None, :]


def eig_dense(gamma, omega, k):
    """Top-k eigenpairs of A = Omega^1/2 Gamma Omega^1/2 (the matrixized eq. 3.1)
    by a dense symmetric eigensolver; eigenvalues in descending order; returns
    (lambda[k], phi[P,k], fve[k]) with FVE over all positive eigenvalues."""
    A = weighted_matrix(gamma, omega)
    ev, V = np.linalg.eigh(A)
    order = np.argsort(-ev, kind="stable")
    ev = ev[order]
    V = V[:, order]
    pos = ev[ev > 0].sum()
    fve = np.cumsum(ev[:k]) / pos
    return ev[:k], _rescale_and_sign(V[:, :k], omega), fve


def normals(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count)
    _check(lib().orc_normals(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), count, _p(out)))
    return out


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.uint64)
    _check(lib().orc_splitmix64(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), count, _p(out)))
    return out


def test_matrix(P: int, r: int, seed: int) -> np.ndarray:
    """Gaussian test matrix of the random projection (Section 3.4): P x r, entry
    (p, j) is normal number j*P + p of stream `seed`. Its scale does not matter
    because the range finder orthonormalizes."""
    return normals(seed, P * r).reshape(r, P).T.copy()


def eig_randomized(gamma, omega, k, oversample, power_iters, seed, return_basis=False):
    """Random-projection eigendecomposition (Section 3.4, read as the Halko-
    Martinsson-Tropp range finder with Rayleigh-Ritz):
      1. Omega_g = P x r Gaussian, r = k + oversample;  Q = qr(A Omega_g);
      2. power_iters times: Q = qr(A Q); Q = qr(A Q)   (2 q further products);
      3. B = Q^T A Q (symmetrized); eig(B) = U diag(theta) U^T;
      4. top k by algebraic value; psi = Q U; phi = psi/sqrt(omega) with the sign rule;
      FVE_l = sum_{m<=l} theta_m / sum over the r Ritz values with theta > 0."""
    A = weighted_matrix(gamma, omega)
    P = A.shape[0]
    r = k + oversample
    Om = test_matrix(P, r, seed)
    Q, _ = np.linalg.qr(A @ Om)
    for _ in range(2 * power_iters):
        Q, _ = np.linalg.qr(A @ Q)
    B = Q.T @ (A @ Q)
    B = 0.5 * (B + B.T)
    th, U = np.linalg.eigh(B)
    order = np.argsort(-th, kind="stable")
    th = th[order]
    U = U[:, order]
    pos = th[th > 0].sum()
    # no positive Ritz value (e.g. a zero surface): the ratio is undefined; 0 by convention
    fve = np.cumsum(th[:k]) / pos if pos > 0 else np.zeros(k)
    phi = _rescale_and_sign(Q @ U[:, :k], omega)
    if return_basis:
        return th[:k], phi, fve, Q
    return th[:k], phi, fve


# ----------------------------------------------------------------- CV
def cv_score(Q_f, G_f, C_f, Ghat):
    """Binned leave-curves-out CV contribution of one fold: for the fold's own raw
    products, sum over pairs of w (Y_ij Y_il - Ghat(bin))^2 spread over the bins by
    the binning weights = sum_pq [Q_f - 2 G_f Ghat + C_f Ghat^2]."""
    Gh = np.nan_to_num(np.asarray(Ghat, np.float64), nan=0.0)
    return float(np.sum(Q_f - 2.0 * G_f * Gh + C_f * Gh * Gh))

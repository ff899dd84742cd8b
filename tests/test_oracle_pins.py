"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each checks a property that a
plausible mistake (a dropped term, a wrong sign or index, a transposed operand,
a wrong weight) would break -- exact integer arithmetic, conservation laws of
linear binning, an independent formulation of the same sums, exact reproduction
of linear functions by a local-linear fit, unbinned least squares by a library
solver, closed-form eigenpairs.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from fpca_synth import grid_points, fourier_1d, fold_assignment

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_irregular(rng, d, n, Nlo, Nhi, dtype=np.float64):
    Ni = rng.integers(Nlo, Nhi + 1, size=n)
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    t = rng.random((off[-1], d)).astype(dtype).astype(np.float64)
    y = rng.standard_normal(off[-1])
    return off, t, y


# ------------------------------------------------------------------ P1 bin index
def test_bin_index_exact_rational():
    """Lower corner = min(floor(x (M-1)), M-2) computed in exact rational arithmetic."""
    rng = np.random.default_rng(0)
    for M in (2, 3, 17, 64, 101, 4097):
        x = rng.random(2000).astype(np.float32).astype(np.float64)
        x[:3] = [0.0, 1.0, np.float32(1.0 / 3.0)]
        node, wt, lower = oracle.bin_corners((M,), x[:, None])
        for xi, lo, w in zip(x[:200], lower[:200], wt[:200]):
            u = Fraction(float(xi)) * (M - 1)
            k = min(int(u), M - 2)
            assert lo == k
            assert w[1] == float(u - k) and w[0] == 1.0 - float(u - k)


def test_bin_index_hand_cases():
    M = 11
    _, wt, lo = oracle.bin_corners((M,), np.array([[0.0], [1.0], [0.5], [0.05]]))
    assert list(lo) == [0, 9, 5, 0]
    assert wt[1].tolist() == [0.0, 1.0]          # x = 1 sits on the last node via rho = 1
    assert wt[2].tolist() == [1.0, 0.0]
    np.testing.assert_allclose(wt[3], [0.5, 0.5], rtol=0, atol=1e-15)
    # float32(m/(M-1)) may land just below the node: then rho is ~1 on the lower cell
    x = np.float64(np.float32(3.0 / 10.0))
    _, wt, lo = oracle.bin_corners((M,), np.array([[x]]))
    assert abs((lo[0] + wt[0][1]) / 10.0 - x) < 1e-15


def test_domain_error():
    with pytest.raises(ValueError):
        oracle.bin_mean((8,), np.array([0, 2]), np.array([[0.2], [1.5]]), np.zeros(2))
    with pytest.raises(ValueError):
        oracle.bin_mean((8,), np.array([0, 1]), np.array([[np.nan]]), np.zeros(1))


# ------------------------------------------------------------------ P2 conservation
@pytest.mark.parametrize("d,M", [(1, (13,)), (2, (7, 9)), (3, (5, 4, 6))])
def test_mean_binning_conserves_mass_and_first_moment(d, M):
    rng = np.random.default_rng(d)
    off, t, y = _tiny_irregular(rng, d, 9, 1, 12)
    c, s, idx, cnt = oracle.bin_mean(M, off, t, y)
    Ni = np.diff(off)
    w = np.repeat(1.0 / Ni, Ni)
    g = grid_points(M)
    assert abs(c.sum() - len(Ni)) < 1e-12
    assert abs(s.sum() - (w * y).sum()) < 1e-12
    for k in range(d):
        assert abs((c * g[:, k]).sum() - (w * t[:, k]).sum()) < 1e-12
        assert abs((s * g[:, k]).sum() - (w * y * t[:, k]).sum()) < 1e-12
    assert cnt.sum() == off[-1]
    assert np.array_equal(np.bincount(idx, minlength=c.size), cnt)


def test_cov_binning_conserves_mass_and_first_moment():
    rng = np.random.default_rng(5)
    d, M = 2, (5, 6)
    off, t, y = _tiny_irregular(rng, d, 7, 1, 8)
    C, G = oracle.bin_cov_pairs(M, off, t, y)
    Ni = np.diff(off)
    P = C.shape[0]
    g = grid_points(M)
    tot_c = tot_g = 0.0
    fm_s = np.zeros(d)
    fm_t = np.zeros(d)
    for i in range(len(Ni)):
        if Ni[i] < 2:
            continue
        w = 1.0 / (Ni[i] * (Ni[i] - 1))
        a, b = off[i], off[i + 1]
        for j in range(a, b):
            for l in range(a, b):
                if j != l:
                    tot_c += w
                    tot_g += w * y[j] * y[l]
                    fm_s += w * t[j]
                    fm_t += w * t[l]
    assert abs(C.sum() - (Ni >= 2).sum()) < 1e-12 and abs(C.sum() - tot_c) < 1e-12
    assert abs(G.sum() - tot_g) < 1e-12
    for k in range(d):
        assert abs((C * g[:, k][:, None]).sum() - fm_s[k]) < 1e-12
        assert abs((C * g[:, k][None, :]).sum() - fm_t[k]) < 1e-12


# ------------------------------------------------------------------ P3 identities
@pytest.mark.parametrize("d,M", [(1, (9,)), (2, (5, 4)), (3, (3, 4, 3))])
def test_pair_loops_equal_gram_identity(d, M):
    rng = np.random.default_rng(10 + d)
    off, t, y = _tiny_irregular(rng, d, 11, 1, 9)
    folds = fold_assignment(11, 3, seed=3)
    for fs in (-1, 0, 2):
        C1, G1, Q1, n1 = oracle.bin_cov_pairs(M, off, t, y, folds, fs, want_Q=True, want_cnt=True)
        C2, G2, Q2, n2 = oracle.bin_cov_identity(M, off, t, y, folds, fs, want_Q=True, want_cnt=True)
        for A, B in ((C1, C2), (G1, G2), (Q1, Q2)):
            assert np.abs(A - B).max() <= 1e-13 * max(1.0, np.abs(A).max())
        assert np.array_equal(n1, n2)
    # fold additivity (integers exact, values to rounding)
    Ct, Gt, _, nt = oracle.bin_cov_pairs(M, off, t, y, want_Q=True, want_cnt=True)
    parts = [oracle.bin_cov_pairs(M, off, t, y, folds, f, want_Q=True, want_cnt=True) for f in range(3)]
    assert np.array_equal(sum(p[3] for p in parts), nt)
    assert np.abs(sum(p[0] for p in parts) - Ct).max() < 1e-14
    assert np.abs(sum(p[1] for p in parts) - Gt).max() < 1e-13


def test_common_grid_closed_form():
    """Observations at all P nodes: C = n/(P(P-1)) off the diagonal, 0 on it, and
    G = Y^T Y/(P(P-1)) with the diagonal removed."""
    rng = np.random.default_rng(3)
    M = (4, 3)
    P = 12
    n = 5
    Y = rng.standard_normal((n, P))
    pts = grid_points(M)
    off = np.arange(n + 1, dtype=np.int64) * P
    t = np.tile(pts, (n, 1))
    C, G = oracle.bin_cov_pairs(M, off, t, Y.reshape(-1))
    c2, s2, C2, G2 = oracle.bin_common_grid(Y)
    assert np.abs(C - C2).max() < 1e-15
    assert np.abs(G - G2).max() < 1e-14
    c, s, _, _ = oracle.bin_mean(M, off, t, Y.reshape(-1))
    assert np.abs(c - c2).max() < 1e-15 and np.abs(s - s2).max() < 1e-14
    c3, s3 = oracle.bin_common_grid_mean(Y)
    assert np.abs(c - c3).max() < 1e-15 and np.abs(s - s3).max() < 1e-14
    pp, qq = np.meshgrid(np.arange(P), np.arange(P), indexing="ij")
    Ge = oracle.bin_common_grid_entries(Y, pp.ravel(), qq.ravel()).reshape(P, P)
    assert np.abs(G - Ge).max() < 1e-14


# ------------------------------------------------------------------ P4 linear reproduction
@pytest.mark.parametrize("dims,h", [((23,), 0.13), ((9, 11), 0.3), ((5, 6, 7), 0.45),
                                    ((7, 6, 7, 6), 0.4), ((5, 4, 5, 4, 5), 0.5), ((4, 5, 4, 4, 5, 4), 0.6)])
def test_local_linear_reproduces_linear_functions(dims, h):
    """If g_p = c_p (a + b^T x_p) then b0(x) = a + b^T x at every node with an OK
    status -- boundaries included (Fan & Gijbels' reproduction property)."""
    rng = np.random.default_rng(len(dims))
    P = int(np.prod(dims))
    c = rng.random(P) + 0.05
    c[rng.random(P) < 0.2] = 0.0
    x = grid_points(dims)
    a = 0.7
    b = rng.standard_normal(len(dims))
    g = c * (a + x @ b)
    b0, st = oracle.smooth(dims, h, c, g)
    ok = st == oracle.ST_OK
    assert ok.mean() > 0.5
    err = np.abs(b0[ok] - (a + x[ok] @ b)).max()
    assert err < 1e-11, err


def test_linear_reproduction_breaks_with_sign_error():
    """Sanity: a linear function is NOT reproduced by the local-constant estimate
    (so the pin above would catch a solver that drops the slope terms)."""
    dims = (15,)
    c = np.ones(15)
    x = grid_points(dims)[:, 0]
    g = c * (1 + 2 * x)
    mom = oracle.smooth(dims, 0.3, c, g, want_moments=True)[2]
    local_const = mom[:, 2] / mom[:, 0]
    assert np.abs(local_const[0] - 1.0) > 0.05


# ------------------------------------------------------------------ P7 brute force
def _epan(u):
    return np.where(np.abs(u) < 1, 1 - u * u, 0.0)


def test_mean_bruteforce_unbinned_on_nodes():
    """Observations on grid nodes: binned smoother == direct weighted least squares
    of eq. (2.3) over the raw observations (numpy lstsq)."""
    rng = np.random.default_rng(1)
    M = (6, 5)
    pts = grid_points(M)
    n = 4
    Ni = [3, 6, 2, 5]
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    t = pts[rng.integers(0, len(pts), off[-1])]
    y = rng.standard_normal(off[-1])
    h = 0.45
    c, s, _, _ = oracle.bin_mean(M, off, t, y)
    b0, st = oracle.smooth_mean(M, h, c, s)
    w_obs = np.repeat(1.0 / np.asarray(Ni, float), Ni)
    for p in range(len(pts)):
        K = np.prod(_epan((t - pts[p]) / h), axis=1) * w_obs
        sel = K > 0
        if st[p] != oracle.ST_OK:
            continue
        X = np.column_stack([np.ones(sel.sum()), (t[sel] - pts[p])])
        sw = np.sqrt(K[sel])
        beta = np.linalg.lstsq(X * sw[:, None], y[sel] * sw, rcond=None)[0]
        assert abs(beta[0] - b0[p]) < 1e-11 * max(1, abs(beta[0]))


def test_cov_bruteforce_unbinned_on_nodes():
    """Same for eq. (2.4): ordered pairs j != l with weight K K / (N_i (N_i - 1))."""
    rng = np.random.default_rng(2)
    M = (5,)
    pts = grid_points(M)
    Ni = [4, 3, 5, 2, 1]
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    t = pts[rng.integers(0, len(pts), off[-1])]
    y = rng.standard_normal(off[-1])
    h = 0.6
    C, G = oracle.bin_cov_pairs(M, off, t, y)
    b0, st = oracle.smooth_cov_raw(M, h, C, G)
    S, T, W, Z = [], [], [], []
    for i in range(len(Ni)):
        if Ni[i] < 2:
            continue
        for j in range(off[i], off[i + 1]):
            for l in range(off[i], off[i + 1]):
                if j != l:
                    S.append(t[j, 0]); T.append(t[l, 0])
                    W.append(1.0 / (Ni[i] * (Ni[i] - 1))); Z.append(y[j] * y[l])
    S, T, W, Z = map(np.asarray, (S, T, W, Z))
    checked = 0
    for p in range(len(pts)):
        for q in range(len(pts)):
            e = p * len(pts) + q
            if st[e] != oracle.ST_OK:
                continue
            K = _epan((S - pts[p, 0]) / h) * _epan((T - pts[q, 0]) / h) * W
            sel = K > 0
            X = np.column_stack([np.ones(sel.sum()), S[sel] - pts[p, 0], T[sel] - pts[q, 0]])
            sw = np.sqrt(K[sel])
            beta = np.linalg.lstsq(X * sw[:, None], Z[sel] * sw, rcond=None)[0]
            assert abs(beta[0] - b0[e]) < 1e-10 * max(1, abs(beta[0]))
            checked += 1
    assert checked > 10


# ------------------------------------------------------------------ P8 WLS solver
def test_wls_matches_library_solver_and_status_rules():
    rng = np.random.default_rng(4)
    D = 4
    nm = oracle.num_moments(D)
    moms = []
    ref = []
    for _ in range(50):
        X = np.column_stack([np.ones(30), rng.standard_normal((30, D))])
        w = rng.random(30)
        yv = rng.standard_normal(30)
        A = X.T @ (w[:, None] * X)
        r = X.T @ (w * yv)
        o = [A[0, 0]] + list(A[0, 1:]) + [A[1 + k, 1 + l] for k in range(D) for l in range(k, D)]
        o += [r[0]] + list(r[1:])
        moms.append(o)
        ref.append(np.linalg.solve(A, r)[0])
    b0, st, mp = oracle.wls_from_moments(D, np.array(moms))
    assert (st == 0).all()
    np.testing.assert_allclose(b0, ref, rtol=1e-10, atol=1e-12)
    # EMPTY: S0 = 0
    z = np.zeros(nm)
    b0, st, _ = oracle.wls_from_moments(D, z[None])
    assert st[0] == oracle.ST_EMPTY and np.isnan(b0[0])
    # FALLBACK: all data on one line (singular) -> local constant T0/S0
    X = np.column_stack([np.ones(10), np.zeros((10, D))])
    X[:, 1] = np.linspace(-1, 1, 10)
    yv = rng.standard_normal(10)
    A = X.T @ X
    r = X.T @ yv
    o = [A[0, 0]] + list(A[0, 1:]) + [A[1 + k, 1 + l] for k in range(D) for l in range(k, D)]
    o += [r[0]] + list(r[1:])
    b0, st, _ = oracle.wls_from_moments(D, np.array([o]))
    assert st[0] == oracle.ST_FALLBACK and abs(b0[0] - yv.mean()) < 1e-14


# ------------------------------------------------------------------ P5, P10, P11
def test_symmetry_constant_and_scaling():
    rng = np.random.default_rng(6)
    d, M = 1, (9,)
    off, t, y = _tiny_irregular(rng, d, 12, 2, 10)
    C, G = oracle.bin_cov_pairs(M, off, t, y)
    assert np.abs(C - C.T).max() < 1e-15 and np.abs(G - G.T).max() < 1e-15
    h = 0.3
    Gh, st = oracle.smooth_cov_raw(M, h, C, G)
    Gh = Gh.reshape(9, 9)
    ok = (st.reshape(9, 9) == 0) & (st.reshape(9, 9).T == 0)
    assert np.abs((Gh - Gh.T)[ok]).max() < 1e-12 * np.abs(Gh[ok]).max()
    # constant data: mu = c, Ghat = c^2, Gamma = 0
    yc = np.full_like(y, 1.7)
    c, s, _, _ = oracle.bin_mean(M, off, t, yc)
    mu, stm = oracle.smooth_mean(M, h, c, s)
    C, G = oracle.bin_cov_pairs(M, off, t, yc)
    Gh, st = oracle.smooth_cov_raw(M, h, C, G)
    assert np.abs(mu[stm == 0] - 1.7).max() < 1e-13
    assert np.abs(Gh[st == 0] - 1.7 ** 2).max() < 1e-12
    Gam = oracle.assemble_cov(Gh.reshape(9, 9), mu)
    okm = (st.reshape(9, 9) == 0)
    assert np.abs(Gam[okm]).max() < 1e-12
    # scaling: Y * a -> mu * a, Ghat * a^2; weights scaled by a constant leave b0 unchanged
    a = -2.5
    c1, s1, _, _ = oracle.bin_mean(M, off, t, y)
    m1, _ = oracle.smooth_mean(M, h, c1, s1)
    c2, s2, _, _ = oracle.bin_mean(M, off, t, a * y)
    m2, _ = oracle.smooth_mean(M, h, c2, s2)
    np.testing.assert_allclose(m2, a * m1, rtol=1e-12, atol=1e-14)
    m3, _ = oracle.smooth_mean(M, h, 3.0 * c1, 3.0 * s1)
    np.testing.assert_allclose(m3, m1, rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------ P6, P9 eigen
def _fourier_cov(M, index, lambdas):
    pts = grid_points(M)
    Phi = np.stack([np.prod([fourier_1d(a, pts[:, k]) for k, a in enumerate(tup)], axis=0)
                    for tup in index], axis=1)
    return Phi @ np.diag(lambdas) @ Phi.T, Phi


@pytest.mark.parametrize("M,index", [((33,), [(2,), (1,), (4,)]),
                                     ((17, 13), [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1)])])
def test_closed_form_eigenpairs_trapezoid(M, index):
    """Gamma = sum_k lambda_k phi_k phi_k on the grid, trapezoid weights: the
    matrixized eq. (3.1) has exactly these eigenpairs (discrete orthonormality of
    the Fourier basis under the trapezoid rule)."""
    lambdas = 2.0 ** -np.arange(1, len(index) + 1)
    Gam, Phi = _fourier_cov(M, index, lambdas)
    om = oracle.quad_weights(M, rule="trapezoid")
    k = len(index)
    ev, phi, fve = oracle.eig_dense(Gam, om, k)
    np.testing.assert_allclose(ev, lambdas, rtol=1e-12)
    for j in range(k):
        err = min(np.abs(phi[:, j] - Phi[:, j]).max(), np.abs(phi[:, j] + Phi[:, j]).max())
        assert err < 1e-10
    np.testing.assert_allclose(fve[-1], 1.0, rtol=1e-12)
    # random projection is exact when rank <= r (Section 3.4's premise)
    ev2, phi2, fve2 = oracle.eig_randomized(Gam, om, k, 4, 1, seed=7)
    np.testing.assert_allclose(ev2, lambdas, rtol=1e-10)
    for j in range(k):
        assert np.abs(phi2[:, j] - phi[:, j]).max() < 1e-8
    np.testing.assert_allclose(fve2, fve, rtol=1e-10)


def test_randomized_full_rank_within_hmt_bound():
    """Full-rank A: the range-finder residual obeys the Halko-Martinsson-Tropp
    expected bound (Thm 10.5, q = 0) computed from the dense spectrum."""
    rng = np.random.default_rng(9)
    P = 200
    U, _ = np.linalg.qr(rng.standard_normal((P, P)))
    s = 1.0 / np.arange(1, P + 1) ** 1.5
    A = (U * s) @ U.T
    om = np.ones(P)
    k, p = 5, 5
    _, _, _, Q = oracle.eig_randomized(A, om, k, p, 0, seed=3, return_basis=True)
    resid = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    r = k + p
    bound = (1 + np.sqrt(k / (p - 1))) * s[k] + np.e * np.sqrt(r) / p * np.sqrt((s[k:] ** 2).sum())
    assert resid <= bound


def test_rng_published_values_and_normals():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.startswith("0x")]
    got = [int(x) for x in oracle.splitmix64(0, 3)]
    assert got == want
    z = oracle.normals(123, 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    assert abs((z ** 3).mean()) < 0.03 and abs((z ** 4).mean() - 3) < 0.05


# ------------------------------------------------------------------ P12 CV
def test_binned_cv_equals_pairwise_on_nodes():
    rng = np.random.default_rng(12)
    M = (6,)
    pts = grid_points(M)
    Ni = [4, 5, 3, 6]
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    t = pts[rng.integers(0, 6, off[-1])]
    y = rng.standard_normal(off[-1])
    Ghat = rng.standard_normal((6, 6))
    Ghat = Ghat + Ghat.T
    C, G, Q = oracle.bin_cov_pairs(M, off, t, y, want_Q=True)
    score = oracle.cv_score(Q, G, C, Ghat)
    direct = 0.0
    node = np.rint(t[:, 0] * 5).astype(int)
    for i in range(len(Ni)):
        w = 1.0 / (Ni[i] * (Ni[i] - 1))
        for j in range(off[i], off[i + 1]):
            for l in range(off[i], off[i + 1]):
                if j != l:
                    direct += w * (y[j] * y[l] - Ghat[node[j], node[l]]) ** 2
    assert abs(score - direct) < 1e-12 * abs(direct)


# ------------------------------------------------------------------ P13 surrogate reference
def test_mlp_gradient_matches_central_differences():
    from oracle import mlp
    rng = np.random.default_rng(21)
    theta = rng.standard_normal(mlp.NPARAM) * 0.1
    X = rng.standard_normal((7, mlp.NF))
    y = rng.standard_normal(7)
    loss, g = mlp.loss_and_grad(theta, X, y)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 4096, 4096 + 128]])
    eps = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        fd = (mlp.loss_and_grad(tp, X, y)[0] - mlp.loss_and_grad(tm, X, y)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_is_signed_learning_rate():
    """Bias-corrected Adam moves each parameter by lr * sign(g) at step 1."""
    from oracle import mlp
    rng = np.random.default_rng(2)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    th2, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3, eps=1e-12)
    np.testing.assert_allclose(th - th2, 1e-3 * np.sign(g), rtol=1e-9)


def test_features_lag_structure_and_counts():
    """Pair arrays with G = rho^lag C along each coordinate give variogram
    features rho^l; curve-size features equal their definitions."""
    from oracle import mlp
    M = (6, 5)
    P = 30
    coords = np.stack(np.unravel_index(np.arange(P), M), axis=1)
    diff = np.abs(coords[:, None, :] - coords[None, :, :])
    C = 1.0 + 0.1 * (coords[:, None, 0] + coords[None, :, 1])
    rho = 0.7
    G = C * rho ** diff.sum(-1) * 2.0
    off = np.array([0, 3, 7, 12], np.int64)
    c = np.ones(P)
    s = np.full(P, 0.5)
    s2 = np.full(P, 3.0)
    f = mlp.features(M, off, c, s, s2, C, G)
    assert abs(f[0] - np.log(3)) < 1e-15 and abs(f[2] - np.log(3 * 2 + 4 * 3 + 5 * 4)) < 1e-15
    np.testing.assert_allclose(f[12:12 + 5], rho ** np.arange(1, 6), rtol=1e-12)
    np.testing.assert_allclose(f[20:20 + 4], rho ** np.arange(1, 5), rtol=1e-12)
    assert abs(f[9] - np.log(2.0)) < 1e-12 and abs(f[10] - (3.0 - 2.0) / 3.0) < 1e-12
    # curvature of the variogram at lag 0: (2 rho^2 - 4 rho + 2) / 2 = (1 - rho)^2 along both coordinates
    assert abs(f[28] - (1 - rho) ** 2) < 1e-12 and abs(f[29] - (1 - rho) ** 2) < 1e-12
    # pair-weight level: sum C = P^2 + 0.1 P (sum of first coordinates + sum of second coordinates)
    #                          = 900 + 3 (5 * 15 + 6 * 10) = 1305
    assert abs(f[30] - np.log(1305.0 / 900.0)) < 1e-12
    assert abs(f[31] - np.log(1.0 / 5.0)) < 1e-15 and abs(f[4] - np.log(30.0)) < 1e-15


def test_features_occupancy_moments_and_spread():
    """Hand-built arrays with known values of the curve-size spread, occupancy,
    pair density, response moments and the raw-product variance."""
    from oracle import mlp
    M = (6, 5)
    P = 30
    off = np.array([0, 3, 7, 12], np.int64)           # N_i = 3, 4, 5
    c = np.zeros(P)
    c[:12] = 2.0                                       # 12 of 30 nodes occupied, equal weights
    s = 0.5 * c                                        # E Y = 0.5
    s2 = 3.0 * c                                       # E Y^2 = 3
    C = np.ones((P, P))
    C[:5, :] = 0.0                                     # 150 of 900 pair cells empty
    a, tau = 0.8, 0.09
    G = a * C                                          # raw products a on every pair
    Q = (a * a + tau) * C                              # squared products: variance tau about a
    f = mlp.features(M, off, c, s, s2, C, G, Q)
    assert abs(f[1] - np.log(4.0)) < 1e-15
    assert abs(f[3] - np.sqrt(2.0 / 3.0) / 4.0) < 1e-15   # E N^2 = 50/3, (E N)^2 = 16
    assert abs(f[5] - 12.0 / 30.0) < 1e-15
    assert abs(f[6] - 750.0 / 900.0) < 1e-15
    assert abs(f[7] - np.log(3.0)) < 1e-15
    assert abs(f[8] - 0.25 / 3.0) < 1e-15
    assert abs(f[11] - np.log(tau)) < 1e-12
    # without Q the raw-product variance feature is left at 0
    assert mlp.features(M, off, c, s, s2, C, G)[11] == 0.0


# ------------------------------------------------------------------ noise variance (eq. 2.6)
@pytest.mark.parametrize("M,h", [((7,), 0.4), ((3, 3), 0.8)])
def test_noise_variance_hadamard_design(M, h):
    """Closed form: curves Y_i = a + s r_i on a common grid, with r_i the rows of
    a Hadamard matrix without its constant column (columns orthogonal and
    summing to zero). Then the binned mean is a, the binned second moment
    a^2 + s^2, the off-diagonal raw covariance a^2, so Gamma = 0 and the noise
    variance is exactly s^2 at every node (the printed plus sign would give
    s^2 + 2 a^2)."""
    from scipy.linalg import hadamard
    P = int(np.prod(M))
    H = 1
    while H < P + 1:
        H *= 2
    r = hadamard(H)[:, 1:P + 1].astype(np.float64)
    a, sd = 0.8, 0.3
    Y = a + sd * r
    c, s = oracle.bin_common_grid_mean(Y)
    _, sq = oracle.bin_common_grid_mean(Y * Y)
    mu, st = oracle.smooth_mean(M, h, c, s)
    b0, st2 = oracle.smooth_mean(M, h, c, sq)
    _, _, C, G = oracle.bin_common_grid(Y)
    Ghat, st3 = oracle.smooth_cov_raw(M, h, C, G)
    assert np.all(st == 0) and np.all(st2 == 0) and np.all(st3 == 0)
    gam = oracle.assemble_cov(Ghat.reshape(P, P), mu)
    s2t, s2, cnt = oracle.noise_variance(b0, mu, gam)
    assert cnt == P
    assert np.abs(s2t - sd * sd).max() < 1e-12
    assert abs(s2 - sd * sd) < 1e-12


def test_noise_variance_linear_surfaces_and_mask():
    """Synthesized binned arrays whose smooths are exact (local-linear
    reproduction): mu = a, Gamma(s,t) = alpha + beta (s + t), b0(t) = a^2 +
    alpha + 2 beta t + sigma^2. The noise variance is sigma^2 at every node,
    which needs Gamma's diagonal (Gamma(t,0) would leave beta t). Nodes
    outside the mask get 0 and are not counted."""
    M = (9,)
    P = 9
    x = grid_points(M)[:, 0]
    rng = np.random.default_rng(5)
    c = rng.random(P) + 0.5
    a, alpha, beta, sig2 = 0.6, 0.3, 0.25, 0.04
    s = c * a
    sq = c * (a * a + alpha + 2 * beta * x + sig2)
    C = np.outer(c, c)
    np.fill_diagonal(C, 0.0)
    G = C * (a * a + alpha + beta * (x[:, None] + x[None, :]))
    h = 0.3
    mu, _ = oracle.smooth_mean(M, h, c, s)
    b0, _ = oracle.smooth_mean(M, h, c, sq)
    Ghat, st = oracle.smooth_cov_raw(M, h, C, G)
    assert np.all(st == 0)
    gam = oracle.assemble_cov(Ghat.reshape(P, P), mu)
    s2t, s2, cnt = oracle.noise_variance(b0, mu, gam)
    assert cnt == P and abs(s2 - sig2) < 1e-12 and np.abs(s2t - sig2).max() < 1e-12
    mask = np.ones(P, np.uint8)
    mask[[0, 4]] = 0
    s2t, s2, cnt = oracle.noise_variance(b0, mu, gam, mask)
    assert cnt == P - 2 and s2t[0] == 0 and s2t[4] == 0 and abs(s2 - sig2) < 1e-12
    b0n = b0.copy()
    b0n[2] = np.nan
    s2t, s2, cnt = oracle.noise_variance(b0n, mu, gam)
    assert cnt == P - 1 and np.isnan(s2t[2]) and abs(s2 - sig2) < 1e-12


# ------------------------------------------------------------------ PACE scores (eq. 2.7)
def _pace_case(rng, M, n, k, Nlo, Nhi):
    d = len(M)
    P = int(np.prod(M))
    Ni = rng.integers(Nlo, Nhi + 1, size=n)
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    t = rng.random((int(off[-1]), d))
    efuns = rng.standard_normal((P, k))
    mu = rng.standard_normal(P)
    return off, t, efuns, mu


def test_pace_noise_free_limit_recovers_scores():
    """Curves built exactly as mu + sum_l xi_l phi_l at their points (values
    interpolated from the grid): as sigma2 -> 0 the conditional expectation
    tends to the least-squares coefficients, i.e. the generating xi. A missing
    Lambda in front (or a transposed Phi) would give other values."""
    rng = np.random.default_rng(11)
    M, n, k = (9, 7), 6, 4
    off, t, efuns, mu = _pace_case(rng, M, n, k, 12, 30)
    node, wt, _ = oracle.bin_corners(M, t)
    Phi = np.einsum("jc,jcl->jl", wt, efuns[node])
    mut = (wt * mu[node]).sum(1)
    xi = rng.standard_normal((n, k))
    y = mut.copy()
    for i in range(n):
        sl = slice(off[i], off[i + 1])
        y[sl] += Phi[sl] @ xi[i]
    lam = np.array([2.0, 1.0, 0.5, 0.25])
    got = oracle.pace_scores(M, off, t, y, mu, efuns, lam, 1e-12)
    assert np.abs(got - xi).max() < 1e-8


def test_pace_single_observation_closed_form():
    """N_i = 1: xi_l = lambda_l phi_l(t) (y - mu(t)) / (sum_m lambda_m phi_m(t)^2 + sigma2);
    a component with lambda <= 0 scores 0."""
    rng = np.random.default_rng(12)
    M, k = (11,), 3
    off, t, efuns, mu = _pace_case(rng, M, 5, k, 1, 1)
    y = rng.standard_normal(5)
    lam = np.array([1.5, -0.2, 0.7])
    s2 = 0.3
    got = oracle.pace_scores(M, off, t, y, mu, efuns, lam, s2)
    node, wt, _ = oracle.bin_corners(M, t)
    for i in range(5):
        ph = wt[i] @ efuns[node[i]]
        m = wt[i] @ mu[node[i]]
        lp = np.array([1.5, 0.0, 0.7])
        ref = lp * ph * (y[i] - m) / ((lp * ph * ph).sum() + s2)
        assert np.abs(got[i] - ref).max() < 1e-13
    assert np.all(got[:, 1] == 0)


def test_pace_common_grid_missing_values():
    """Common grid with NaN entries: those observations are left out, which
    equals the irregular design over the observed nodes; a curve with no
    observation scores 0."""
    rng = np.random.default_rng(13)
    M, n, k = (5, 4), 4, 3
    P = 20
    efuns = rng.standard_normal((P, k))
    mu = rng.standard_normal(P)
    Y = rng.standard_normal((n, P))
    Y[rng.random((n, P)) < 0.3] = np.nan
    Y[3] = np.nan
    lam = np.array([1.0, 0.5, 0.2])
    got = oracle.pace_scores(M, None, None, Y, mu, efuns, lam, 0.1)
    pts = grid_points(M)
    obs = [np.nonzero(np.isfinite(Y[i]))[0] for i in range(n)]
    off = np.concatenate([[0], np.cumsum([o.size for o in obs])]).astype(np.int64)
    t = np.concatenate([pts[o] for o in obs])
    y = np.concatenate([Y[i][o] for i, o in enumerate(obs)])
    ref = oracle.pace_scores(M, off, t, y, mu, efuns, lam, 0.1)
    assert np.abs(got - ref).max() < 1e-12
    assert np.all(got[3] == 0)


def test_reconstruction_of_noise_free_curves():
    """Common-grid curves mu + sum_l xi_l phi_l observed at every node: PACE in
    the noise-free limit returns xi, and the reconstruction (the display after
    eq. 2.7) returns the curves themselves."""
    rng = np.random.default_rng(14)
    M, n, k = (6, 5), 7, 4
    P = 30
    efuns = rng.standard_normal((P, k))
    mu = rng.standard_normal(P)
    xi = rng.standard_normal((n, k))
    X = mu[None, :] + xi @ efuns.T
    sc = oracle.pace_scores(M, None, None, X, mu, efuns, np.array([3.0, 2.0, 1.0, 0.5]), 1e-12)
    assert np.abs(sc - xi).max() < 1e-8
    Xh = oracle.reconstruct(mu, efuns, sc)
    assert Xh.shape == (n, P) and np.abs(Xh - X).max() < 1e-8

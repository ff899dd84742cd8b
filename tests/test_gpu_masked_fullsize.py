"""GPU parity of the covariance smoother and batched CV on masked domains
(Section 3.1: Gamma = 0 where s or t lies outside Omega) and at the full sizes
of the benchmark workloads.

- masked fpca_smooth_cov on the general path (pair weights given, d = 2 and 3)
  and on the complete common-grid path (C = NULL, d = 2), against the oracle's
  direct-window smoother and assembly with the mask; exact zeros outside Omega;
- masked fpca_cv_batched against the oracle's scores;
- the fused common-grid smoother at 64 x 64, h = 0.1 (R = 6 taps each side)
  with the GPU's own Gram product fed to both sides, at the FP32 bar of 1e-5
  on the whole near-diagonal band, the four boundary strips and random nodes;
- the d = 3 disk x time workload at its full size (n = 800, 16^6 covariance
  nodes): binning against the oracle's Gram identity, the masked smoother on
  sampled nodes, and one CV job's score recomputed from the GPU's own smooth.
"""
import sys

import numpy as np
import pytest

import oracle
from fpca_synth import disk_time_mask, fold_assignment, make_c3, make_c4
from tests._util import engine, normwise_rel, rand_irregular, status_agreement

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


@pytest.fixture(scope="module")
def F(torch):
    import paper_1510_04439_amd as F
    F.load_library()
    return F


@pytest.fixture(scope="module")
def h(F):
    hh = F.Handle(0)
    yield hh
    hh.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(x):
    return x.detach().cpu().numpy()


def _disk_mask_2d(M):
    x = np.arange(M[0]) / (M[0] - 1)
    y = np.arange(M[1]) / (M[1] - 1)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return (((X - 0.5) ** 2 + (Y - 0.5) ** 2) <= 0.25 + 1e-12).astype(np.uint8).reshape(-1)


def _check_masked(gam_h, st_h, ref, rst, mask, tol):
    P = mask.size
    out = ~mask.astype(bool)
    assert np.all(gam_h[out, :] == 0) and np.all(gam_h[:, out] == 0)
    st2 = rst.reshape(P, P)
    okm = (st2 == 0) & (st2.T == 0)
    assert status_agreement(st_h, rst)[0] == 0
    assert normwise_rel(gam_h, ref, okm) < tol
    assert np.array_equal(gam_h, gam_h.T)


@pytest.mark.parametrize("M,hb", [((12, 12), 0.25), ((6, 6, 6), 0.45), ((7, 5, 6), 0.5)])
@pytest.mark.parametrize("eng", ["queue", "passes"])
def test_smooth_cov_masked_general(torch, F, h, M, hb, eng):
    with engine(F, h, F.FPCA_ENGINE_QUEUE if eng == "queue" else F.FPCA_ENGINE_PASSES):
        _masked_general(torch, F, h, M, hb)


def _masked_general(torch, F, h, M, hb):
    """Pair weights from irregular curves (the general FP64-moment path) on a
    masked grid: disk in the first two coordinates (times [0,1] for d = 3)."""
    _say(f"masked smooth_cov general M={M} h={hb}")
    rng = np.random.default_rng(500 + sum(M))
    d = len(M)
    P = int(np.prod(M))
    mask = _disk_mask_2d(M) if d == 2 else disk_time_mask(M)
    off, t, y = rand_irregular(rng, d, 60, 2, 25, np.float64)
    C, G = oracle.bin_cov_pairs(M, off, t, y)
    C, G = C.astype(np.float32), G.astype(np.float32)
    mu = rng.standard_normal(P).astype(np.float32)
    gam = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
    st = torch.empty(P, P, dtype=torch.int8, device="cuda:0")
    F.fpca_smooth_cov(h, F.Grid(M, dev(torch, mask)), F.FPCA_F32, dev(torch, C), 0.0, dev(torch, G),
                      dev(torch, mu), F.FPCA_K_EPANECHNIKOV, hb, gam, st)
    h.sync()
    rb, rst = oracle.smooth_cov_raw(M, hb, C.astype(np.float64), G.astype(np.float64))
    ref = oracle.assemble_cov(rb.reshape(P, P), mu.astype(np.float64), mask)
    _check_masked(host(gam), host(st), ref, rst, mask, 1e-5)


@pytest.mark.parametrize("M,hb", [((16, 16), 0.3), ((20, 20), 0.16)])
def test_smooth_cov_masked_common_grid(torch, F, h, M, hb):
    """C = NULL (complete common grid, the fused two-stage kernels) with a disk
    mask: values and statuses against the oracle with C = c0 (1 - delta)."""
    _say(f"masked smooth_cov common grid M={M} h={hb}")
    rng = np.random.default_rng(600 + M[0])
    P = int(np.prod(M))
    mask = _disk_mask_2d(M)
    c0 = 0.41
    G = rng.standard_normal((P, P)) * c0
    G = ((G + G.T) / 2).astype(np.float32)
    np.fill_diagonal(G, 0)
    C = np.full((P, P), c0)
    np.fill_diagonal(C, 0)
    mu = rng.standard_normal(P).astype(np.float32)
    gam = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
    st = torch.empty(P, P, dtype=torch.int8, device="cuda:0")
    F.fpca_smooth_cov(h, F.Grid(M, dev(torch, mask)), F.FPCA_F32, None, c0, dev(torch, G), dev(torch, mu),
                      F.FPCA_K_EPANECHNIKOV, hb, gam, st)
    h.sync()
    rb, rst = oracle.smooth_cov_raw(M, hb, C, G.astype(np.float64))
    ref = oracle.assemble_cov(rb.reshape(P, P), mu.astype(np.float64), mask)
    _check_masked(host(gam), host(st), ref, rst, mask, 1e-5)


@pytest.mark.parametrize("M,nf,hs", [((6, 6, 6), 3, [0.3, 0.5]), ((10, 10), 4, [0.15, 0.3])])
@pytest.mark.parametrize("eng", ["queue", "passes"])
def test_cv_batched_masked(torch, F, h, M, nf, hs, eng):
    with engine(F, h, F.FPCA_ENGINE_QUEUE if eng == "queue" else F.FPCA_ENGINE_PASSES):
        _cv_masked(torch, F, h, M, nf, hs)


def _cv_masked(torch, F, h, M, nf, hs):
    """Masked CV: the held-out pairs are scored against the training smooth,
    which is 0 at nodes outside Omega (as the covariance there)."""
    _say(f"masked cv M={M} folds={nf} h={hs}")
    rng = np.random.default_rng(70 + len(M))
    d = len(M)
    P = int(np.prod(M))
    mask = _disk_mask_2d(M) if d == 2 else disk_time_mask(M)
    n = 36
    off, t, y = rand_irregular(rng, d, n, 1, 16, np.float32)
    folds = fold_assignment(n, nf, seed=9)
    t64, y64 = t.astype(np.float64), y.astype(np.float64)
    slabs = [oracle.bin_cov_pairs(M, off, t64, y64, folds, fs, want_Q=True) for fs in [-1] + list(range(nf))]
    Ch, Gh, Qh = (np.stack([s[i] for s in slabs]).astype(np.float32).astype(np.float64) for i in range(3))
    C, G, Q = (dev(torch, a.astype(np.float32)) for a in (Ch, Gh, Qh))
    scores = F.fpca_cv_batched(h, F.FPCA_F32, [(F.Grid(M, dev(torch, mask)), C, G, Q)], nf, hs)[0]
    ref = np.zeros((len(hs), nf))
    for i, hb in enumerate(hs):
        for f in range(nf):
            b, _ = oracle.smooth_cov_raw(M, hb, Ch[0] - Ch[f + 1], Gh[0] - Gh[f + 1])
            Ghat = oracle.assemble_cov(b.reshape(P, P), np.zeros(P), mask)
            ref[i, f] = oracle.cv_score(Qh[f + 1], Gh[f + 1], Ch[f + 1], Ghat)
    np.testing.assert_allclose(scores, ref, rtol=1e-5)


def _band_and_strips(M, R, rng, n_rand):
    """Covariance nodes (p, q) of a d = 2 grid: every node of a few s-rows whose
    t-window meets the diagonal (|s_k - t_k| <= 2R in both coordinates), rows on
    the four boundary strips (s_1 or s_2 within R of 0 or M-1), and random nodes."""
    M1, M2 = M
    P = M1 * M2
    ps, qs = [], []
    for s1, s2 in [(0, 0), (R - 1, M2 - 1), (M1 // 2, M2 // 2), (M1 - 1, R), (M1 - R, M2 - 2), (3, M2 // 3)]:
        p = s1 * M2 + s2
        t1, t2 = np.meshgrid(np.arange(max(0, s1 - 2 * R), min(M1, s1 + 2 * R + 1)),
                             np.arange(max(0, s2 - 2 * R), min(M2, s2 + 2 * R + 1)), indexing="ij")
        q = (t1 * M2 + t2).reshape(-1)
        ps.append(np.full(q.size, p))
        qs.append(q)
    for strip in range(4):
        k = rng.integers(0, R + 1, 150)
        o = rng.integers(0, M1, 150)
        s1, s2 = [(k, o), (M1 - 1 - k, o), (o, k), (o, M2 - 1 - k)][strip]
        ps.append(s1 * M2 + s2)
        qs.append(rng.integers(0, P, 150))
    ps.append(rng.integers(0, P, n_rand))
    qs.append(rng.integers(0, P, n_rand))
    return np.concatenate(ps), np.concatenate(qs)


def test_fused_smoother_64x64_own_gram(torch, F, h):
    """The benchmark's smoother instance (64 x 64 common grid, h = 0.1: 13 taps
    per coordinate, a full 64-lane wave per t-row, the near-diagonal LDS path)
    with the GPU's own BF16x3 Gram product and mean fed to the oracle as well,
    so the 1e-5 FP32 bar measures the smoother alone."""
    _say("fused smoother 64x64 h=0.1 on the GPU's own Gram")
    from paper_1510_04439_amd import pipeline as PL
    ds = make_c3(n=5000)
    dd = PL.to_device(ds)
    bufs = PL.alloc(dd, ds.k, with_status=True, analytic_C=True)
    F.fpca_bin(h, dd.grid_mean, F.FPCA_BIN_MEAN, dd.design, dd.dtype, F.FPCA_PREC_F32, dd.n, None, None, dd.y,
               None, 0, bufs.c, bufs.s)
    F.fpca_smooth_mean(h, dd.grid_mean, dd.dtype, bufs.c, bufs.s, F.FPCA_K_EPANECHNIKOV, ds.h_mean, bufs.mu,
                       bufs.mu_status)
    F.fpca_bin(h, dd.grid_cov, F.FPCA_BIN_COV, dd.design, dd.dtype, F.FPCA_PREC_BF16X3, dd.n, None, None, dd.y,
               None, 0, None, bufs.G)
    c0 = PL.uniform_pair_weight(dd)
    F.fpca_smooth_cov(h, dd.grid_cov, dd.dtype, None, c0, bufs.G, bufs.mu, F.FPCA_K_EPANECHNIKOV, ds.h_cov,
                      bufs.gamma, bufs.status)
    h.sync()
    M = ds.M_cov
    P = int(np.prod(M))
    G = host(bufs.G).astype(np.float64)
    mu = host(bufs.mu).astype(np.float64)
    C = np.full((P, P), c0)
    np.fill_diagonal(C, 0.0)
    R = int(np.floor(ds.h_cov * (M[0] - 1)))
    assert R == 6
    rng = np.random.default_rng(88)
    p, q = _band_and_strips(M, R, rng, 400)
    nodes = np.concatenate([p * P + q, q * P + p])
    rb, rst = oracle.smooth_cov_raw(M, ds.h_cov, C, G, nodes)
    m = len(p)
    ref = 0.5 * (rb[:m] + rb[m:]) - mu[p] * mu[q]
    ok = (rst[:m] == 0) & (rst[m:] == 0)
    assert ok.mean() > 0.99
    gam = host(bufs.gamma)
    err = normwise_rel(gam[p, q], ref, ok)
    _say(f"  {m} nodes, normwise error {err:.2e}")
    assert err < 1e-5
    assert status_agreement(host(bufs.status).reshape(-1)[nodes], rst)[0] == 0
    assert np.array_equal(gam[p, q], gam[q, p])


@pytest.fixture(scope="module")
def c4_binned(torch, F, h):
    """The d = 3 disk x time workload at full size, binned with its folds."""
    ds = make_c4()
    P = int(np.prod(ds.M_cov))
    d = "cuda:0"
    mask = dev(torch, ds.mask)
    grid = F.Grid(ds.M_cov, mask)
    C, G, Q = (torch.empty(ds.n_folds + 1, P, P, dtype=torch.float32, device=d) for _ in range(3))
    F.fpca_bin(h, grid, F.FPCA_BIN_COV, F.FPCA_IRREGULAR, F.FPCA_F32, F.FPCA_PREC_F32, ds.n,
               dev(torch, ds.offsets), dev(torch, ds.t), dev(torch, ds.y), dev(torch, ds.folds), ds.n_folds,
               C, G, Q)
    h.sync()
    return ds, grid, mask, C, G, Q


def test_c4_full_size_binning(torch, F, h, c4_binned):
    _say("c4 full size: fold binning against the Gram identity")
    ds, grid, mask, C, G, Q = c4_binned
    t64, y64 = ds.t.astype(np.float64), ds.y.astype(np.float64)
    for f in (-1, 2):
        rC, rG, rQ = oracle.bin_cov_identity(ds.M_cov, ds.offsets, t64, y64, ds.folds, f, want_Q=True)
        i = f + 1
        assert normwise_rel(host(C[i]), rC) < 1e-5
        assert normwise_rel(host(G[i]), rG) < 1e-5
        assert normwise_rel(host(Q[i]), rQ) < 1e-5


def test_c4_full_size_masked_smoother_sampled(torch, F, h, c4_binned):
    """fpca_smooth_cov on the training pairs of fold 0 (all 16^6 nodes, 7 x 7
    systems, domain mask) at two bandwidths, sampled nodes and their
    transposes against the oracle's direct-window smoother of the same arrays."""
    ds, grid, mask, C, G, Q = c4_binned
    P = int(np.prod(ds.M_cov))
    W = (C[0] - C[1]).contiguous()
    S = (G[0] - G[1]).contiguous()
    Wh, Sh = host(W).astype(np.float64), host(S).astype(np.float64)
    mk = ds.mask.astype(bool)
    rng = np.random.default_rng(4)
    inside = np.flatnonzero(mk)
    for hb, ns in ((0.1, 3000), (0.2, 400), (float(ds.h_grid[-1]), 24)):
        _say(f"c4 full size: masked smoother h={hb:.3f} on {ns} sampled nodes")
        gam = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
        st = torch.empty(P, P, dtype=torch.int8, device="cuda:0")
        F.fpca_smooth_cov(h, grid, F.FPCA_F32, W, 0.0, S, None, F.FPCA_K_EPANECHNIKOV, hb, gam, st)
        h.sync()
        p = rng.choice(inside, ns)
        q = rng.choice(inside, ns)
        p[:4] = inside[[0, 0, -1, -1]]
        q[:4] = inside[[0, -1, 0, -1]]
        nodes = np.concatenate([p * P + q, q * P + p])
        rb, rst = oracle.smooth_cov_raw(ds.M_cov, hb, Wh, Sh, nodes)
        ref = 0.5 * (rb[:ns] + rb[ns:])
        ok = (rst[:ns] == 0) & (rst[ns:] == 0)
        g = host(gam)
        assert ok.mean() > 0.9
        assert normwise_rel(g[p, q], ref, ok) < 1e-5
        assert status_agreement(host(st).reshape(-1)[nodes], rst)[0] == 0
        out = np.flatnonzero(~mk)
        assert np.all(g[out[:50], :] == 0) and np.all(g[:, out[:50]] == 0)
        del gam, st


def test_c4_full_size_cv_job(torch, F, h, c4_binned):
    """Batched CV at full size (smallest and largest bandwidth of the grid, 5
    folds): every score equals the binned score of the GPU's own masked smooth
    of that fold's training pairs, summed in FP64 on the host; the smooth itself
    is pinned by the sampled-node test above."""
    ds, grid, mask, C, G, Q = c4_binned
    P = int(np.prod(ds.M_cov))
    hs = [float(ds.h_grid[0]), float(ds.h_grid[-1])]
    _say(f"c4 full size: batched CV h={hs}")
    scores = F.fpca_cv_batched(h, F.FPCA_F32, [(grid, C, G, Q)], ds.n_folds, hs)[0]
    assert scores.shape == (2, ds.n_folds) and np.all(np.isfinite(scores))
    for i, f in ((0, 0), (1, 3)):
        W = (C[0] - C[f + 1]).contiguous()
        S = (G[0] - G[f + 1]).contiguous()
        gh = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
        F.fpca_smooth_cov(h, grid, F.FPCA_F32, W, 0.0, S, None, F.FPCA_K_EPANECHNIKOV, hs[i], gh)
        h.sync()
        ref = oracle.cv_score(host(Q[f + 1]).astype(np.float64), host(G[f + 1]).astype(np.float64),
                              host(C[f + 1]).astype(np.float64), host(gh).astype(np.float64))
        _say(f"  job h={hs[i]:.3f} fold {f}: {scores[i, f]:.9e} vs {ref:.9e}")
        assert abs(scores[i, f] - ref) <= 1e-6 * abs(ref)

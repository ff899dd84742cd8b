"""GPU parity: every ABI call against the FP64 oracle on the same seeded inputs.

Bars: integers (bin indices, counts) bit-exact; FP64 paths to 1e-10 normwise;
FP32 paths to 1e-5 normwise (||x - ref||_inf <= 1e-5 ||ref||_inf over nodes
whose status is OK on both sides); the BF16x3 Gram product to 1e-4.
"""
import sys

import numpy as np
import pytest

import oracle
from fpca_synth import grid_points, make_c1, make_c2, fourier_1d, disk_time_mask, fold_assignment
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


def dev(torch, a, dt=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dt is not None:
        t = t.to(dt)
    return t.to("cuda:0")


def host(x):
    return x.detach().cpu().numpy()


# ------------------------------------------------------------------ RNG
def test_rng_normal_matches_oracle(torch, F, h):
    _say("rng")
    n = 100_000
    out = torch.empty(n, dtype=torch.float64, device="cuda:0")
    F.fpca_rng_normal(h, 7, n, out)
    torch.cuda.synchronize()
    ref = oracle.normals(7, n)
    assert np.abs(host(out) - ref).max() < 1e-13


# ------------------------------------------------------------------ binning
@pytest.mark.parametrize("d,M,dt", [(1, (101,), "f64"), (2, (32, 32), "f32"), (3, (7, 9, 5), "f32"),
                                    (2, (13, 17), "f64")])
def test_bin_mean_parity(torch, F, h, d, M, dt):
    _say(f"bin_mean d={d} M={M} {dt}")
    rng = np.random.default_rng(100 + d)
    npdt = np.float64 if dt == "f64" else np.float32
    off, t, y = rand_irregular(rng, d, 300, 0, 60, npdt)
    t[:4] = 0.0
    t[4:8] = 1.0
    tdt = torch.float64 if dt == "f64" else torch.float32
    P = int(np.prod(M))
    c = torch.empty(P, dtype=tdt, device="cuda:0")
    s = torch.empty_like(c)
    s2 = torch.empty_like(c)
    idx = torch.empty(len(y), dtype=torch.int32, device="cuda:0")
    cnt = torch.empty(P, dtype=torch.int64, device="cuda:0")
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_MEAN, F.FPCA_IRREGULAR, F.FPCA_F64 if dt == "f64" else F.FPCA_F32,
               F.FPCA_PREC_F64 if dt == "f64" else F.FPCA_PREC_F32, len(off) - 1, dev(torch, off),
               dev(torch, t), dev(torch, y), None, 0, c, s, s2, idx, cnt)
    h.sync()
    rc, rs, ridx, rcnt = oracle.bin_mean(M, off, t.astype(np.float64), y.astype(np.float64))
    _, rs2, _, _ = oracle.bin_mean(M, off, t.astype(np.float64), y.astype(np.float64) ** 2)
    assert np.array_equal(host(idx), ridx)
    assert np.array_equal(host(cnt), rcnt)
    tol = 1e-12 if dt == "f64" else 1e-5
    assert normwise_rel(host(c), rc) < tol
    assert normwise_rel(host(s), rs) < tol
    assert normwise_rel(host(s2), rs2) < tol


@pytest.mark.parametrize("d,M,dt,nf,bf", [(1, (21,), "f64", 0, False), (2, (9, 8), "f32", 3, False),
                                          (3, (5, 4, 6), "f32", 5, False), (2, (16, 16), "f32", 0, False),
                                          (2, (9, 8), "f32", 3, True), (2, (12, 11), "f32", 0, True),
                                          (3, (5, 4, 6), "f32", 0, False), (3, (4, 5, 3), "f64", 0, False)])
def test_bin_cov_parity(torch, F, h, d, M, dt, nf, bf):
    """bf: the Gram product in BF16x3 (bf16 hi/lo split, three products, FP32
    accumulation); its stated bound is 1e-4 normwise."""
    _say(f"bin_cov d={d} M={M} {dt} folds={nf} bf16x3={bf}")
    rng = np.random.default_rng(200 + d)
    npdt = np.float64 if dt == "f64" else np.float32
    n = 40
    off, t, y = rand_irregular(rng, d, n, 0, 30, npdt)
    folds = fold_assignment(n, nf, seed=5) if nf else None
    tdt = torch.float64 if dt == "f64" else torch.float32
    P = int(np.prod(M))
    ns = nf + 1 if nf else 1
    C = torch.empty(ns, P, P, dtype=tdt, device="cuda:0")
    G = torch.empty_like(C)
    Q = torch.empty_like(C)
    cnt = torch.empty(P, P, dtype=torch.int64, device="cuda:0")
    prec = F.FPCA_PREC_F64 if dt == "f64" else (F.FPCA_PREC_BF16X3 if bf else F.FPCA_PREC_F32)
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_COV, F.FPCA_IRREGULAR, F.FPCA_F64 if dt == "f64" else F.FPCA_F32,
               prec, n, dev(torch, off), dev(torch, t),
               dev(torch, y), dev(torch, folds) if nf else None, nf, C, G, Q, None, cnt)
    h.sync()
    t64, y64 = t.astype(np.float64), y.astype(np.float64)
    tol = 1e-12 if dt == "f64" else (1e-4 if bf else 1e-5)
    for s in range(ns):
        fs = -1 if s == 0 else s - 1
        rC, rG, rQ, rn = oracle.bin_cov_pairs(M, off, t64, y64, folds, fs, want_Q=True, want_cnt=True)
        assert normwise_rel(host(C[s]), rC) < tol, s
        assert normwise_rel(host(G[s]), rG) < tol, s
        assert normwise_rel(host(Q[s]), rQ) < tol, s
        if s == 0:
            assert np.array_equal(host(cnt), rn)


@pytest.mark.parametrize("prec,tol,M", [("f32", 1e-5, (20, 13)), ("bf16x3", 1e-4, (20, 13)), ("f32", 1e-5, (7, 9))])
def test_bin_cov_common_grid(torch, F, h, prec, tol, M):
    """Common-grid binning: Gram product with the diagonal removed, the pair
    weights (or none when weights = NULL), and the mean sums and sums of
    squares (column sums over row chunks with a ragged last chunk; P = 63
    leaves a partial group of four columns)."""
    _say(f"bin_cov common {prec} M={M}")
    rng = np.random.default_rng(7)
    P = int(np.prod(M))
    n = 333
    Y = rng.standard_normal((n, P)).astype(np.float32)
    C = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
    G = torch.empty_like(C)
    G2 = torch.empty_like(C)
    pr = F.FPCA_PREC_F32 if prec == "f32" else F.FPCA_PREC_BF16X3
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_COV, F.FPCA_COMMON_GRID, F.FPCA_F32, pr, n, None, None, dev(torch, Y), None,
               0, C, G)
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_COV, F.FPCA_COMMON_GRID, F.FPCA_F32, pr, n, None, None, dev(torch, Y), None,
               0, None, G2)
    c = torch.empty(P, dtype=torch.float32, device="cuda:0")
    s = torch.empty_like(c)
    s2 = torch.empty_like(c)
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_MEAN, F.FPCA_COMMON_GRID, F.FPCA_F32, F.FPCA_PREC_F32, n, None, None,
               dev(torch, Y), None, 0, c, s, s2)
    h.sync()
    Y64 = Y.astype(np.float64)
    rc, rs, rC, rG = oracle.bin_common_grid(Y64)
    rs2 = oracle.bin_common_grid(Y64 ** 2)[1]
    assert normwise_rel(host(C), rC) < 1e-7
    assert normwise_rel(host(G), rG) < tol
    assert np.array_equal(host(G), host(G2))
    assert np.all(np.diag(host(G)) == 0)
    assert np.array_equal(host(G), host(G).T)
    assert normwise_rel(host(c), rc) < 1e-7 and normwise_rel(host(s), rs) < 1e-5
    assert normwise_rel(host(s2), rs2) < 1e-5


@pytest.mark.parametrize("M,n", [((64, 64), 5000), ((64, 70), 3001), ((64, 96), 1000), ((61, 71), 777)])
def test_bin_cov_common_grid_bf16x3_full(torch, F, h, M, n):
    """BF16x3 Gram product at full size, where the upper-triangle tiles outnumber
    the resident workgroups and the last tiles are split along the curves
    (K ragged for n = 3001 and 777; P = 4331 is odd, so the tile rows leave
    without vector stores): sampled entries and whole rows against the oracle's
    per-entry sums; exact symmetry and a zero diagonal over the whole matrix."""
    _say(f"bin_cov common bf16x3 full M={M} n={n}")
    rng = np.random.default_rng(17)
    P = int(np.prod(M))
    Y = rng.standard_normal((n, P)).astype(np.float32)
    G = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_COV, F.FPCA_COMMON_GRID, F.FPCA_F32, F.FPCA_PREC_BF16X3, n, None, None,
               dev(torch, Y), None, 0, None, G)
    h.sync()
    Gh = host(G)
    assert np.array_equal(Gh, Gh.T)
    assert np.all(np.diag(Gh) == 0)
    rows = np.concatenate([rng.integers(0, P, 4), rng.integers(P - P // 8, P, 4)])
    pr = np.repeat(rows, P)
    qr = np.tile(np.arange(P), len(rows))
    ps, qs = rng.integers(0, P, 4000), rng.integers(0, P, 4000)
    p, q = np.concatenate([pr, ps]), np.concatenate([qr, qs])
    ref = oracle.bin_common_grid_entries(Y, p, q)
    assert normwise_rel(Gh[p, q], ref) < 1e-4


@pytest.mark.parametrize("M,n,dt,prec", [((20, 13), 333, "f32", "bf16x3"), ((64, 64), 5000, "f32", "bf16x3"),
                                          ((61, 71), 777, "f32", "bf16x3"), ((7, 9), 1, "f32", "bf16x3"),
                                          ((7, 9), 0, "f32", "bf16x3"), ((20, 13), 333, "f32", "f32"),
                                          ((7, 9), 70, "f64", "f64"), ((2, 2), 200, "f32", "bf16x3"),
                                          ((4, 4), 65, "f32", "bf16x3"), ((4, 4), 64, "f32", "bf16x3")])
def test_bin_common_one_pass(torch, F, h, M, n, dt, prec):
    """fpca_bin_common against fpca_bin(MEAN) and fpca_bin(COV) on the same
    curves, bit for bit (FP32 data with BF16x3 products: the mean's column
    sums come from the Gram product's split pass, in the same chunks and the
    same order of addition; other precisions run the two calls), and the
    mean's sums against the oracle. P = 4331 is odd (scalar loads in the
    split); n = 777 leaves a ragged 64-row chunk; n = 1 and n = 0 are the
    edges (a zero Gram product, no chunks); P = 4 and 16 are far below one
    128-node tile (rows past P read from row P - 1), n = 64 and 65 put the
    curves exactly at and one past a 64-row step."""
    _say(f"bin_common M={M} n={n} {dt} {prec}")
    rng = np.random.default_rng(5 + n)
    P = int(np.prod(M))
    npdt, tdt = (np.float32, torch.float32) if dt == "f32" else (np.float64, torch.float64)
    dty = F.FPCA_F32 if dt == "f32" else F.FPCA_F64
    pr = {"bf16x3": F.FPCA_PREC_BF16X3, "f32": F.FPCA_PREC_F32, "f64": F.FPCA_PREC_F64}[prec]
    Y = rng.standard_normal((max(n, 1), P)).astype(npdt)[:n]
    Yd = dev(torch, Y).to(tdt) if n else torch.empty(0, P, dtype=tdt, device="cuda:0")
    z = lambda *sh: torch.full(sh, float("nan"), dtype=tdt, device="cuda:0")
    c1, s1, q1, C1, G1 = z(P), z(P), z(P), z(P, P), z(P, P)
    F.fpca_bin_common(h, F.Grid(M), dty, pr, n, Yd, c1, s1, q1, C1, G1)
    c2, s2, q2, C2, G2 = z(P), z(P), z(P), z(P, P), z(P, P)
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_MEAN, F.FPCA_COMMON_GRID, dty, pr, n, None, None, Yd, None, 0, c2, s2, q2)
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_COV, F.FPCA_COMMON_GRID, dty, pr, n, None, None, Yd, None, 0, C2, G2)
    # without the optional outputs (no sums of squares, pair weights not materialized)
    c3, s3, G3 = z(P), z(P), z(P, P)
    F.fpca_bin_common(h, F.Grid(M), dty, pr, n, Yd, c3, s3, None, None, G3)
    h.sync()
    for a, b in ((c1, c2), (s1, s2), (q1, q2), (C1, C2), (G1, G2), (c3, c2), (s3, s2), (G3, G2)):
        assert np.array_equal(host(a), host(b))
    if n:
        Y64 = Y.astype(np.float64)
        rc, rs, _, _ = oracle.bin_common_grid(Y64)
        rq = oracle.bin_common_grid(Y64 ** 2)[1]
        tol = 1e-6 if dt == "f32" else 1e-13
        assert normwise_rel(host(s1), rs) < tol and normwise_rel(host(q1), rq) < tol
        assert normwise_rel(host(c1), rc) < tol
    else:
        assert np.all(host(G1) == 0) and np.all(host(s1) == 0)


def test_domain_error_reported(torch, F, h):
    _say("domain")
    off = np.array([0, 3], np.int64)
    t = np.array([[0.2], [1.5], [0.4]], np.float32)
    y = np.ones(3, np.float32)
    c = torch.empty(9, dtype=torch.float32, device="cuda:0")
    s = torch.empty_like(c)
    F.fpca_bin(h, F.Grid((9,)), F.FPCA_BIN_MEAN, F.FPCA_IRREGULAR, F.FPCA_F32, F.FPCA_PREC_F32, 1,
               dev(torch, off), dev(torch, t), dev(torch, y), None, 0, c, s)
    with pytest.raises(F.FpcaError) as e:
        h.sync()
    assert e.value.code == F.FPCA_ERR_DOMAIN
    h.sync()  # flag cleared


# ------------------------------------------------------------------ smoothers
def _smooth_case(rng, dims, sparse=0.2):
    P = int(np.prod(dims))
    w = rng.random(P) + 0.02
    w[rng.random(P) < sparse] = 0.0
    g = w * rng.standard_normal(P)
    return w, g


@pytest.mark.parametrize("M,hb,dt", [((101,), 0.1, "f64"), ((32, 32), 0.08, "f32"), ((16, 16, 16), 0.2, "f32"),
                                     ((40,), 0.013, "f32"), ((9, 23), 0.3, "f64")])
def test_smooth_mean_parity(torch, F, h, M, hb, dt):
    _say(f"smooth_mean M={M} h={hb} {dt}")
    rng = np.random.default_rng(len(M) * 10 + M[0])
    w, g = _smooth_case(rng, M)
    npdt = np.float64 if dt == "f64" else np.float32
    w, g = w.astype(npdt), g.astype(npdt)
    tdt = torch.float64 if dt == "f64" else torch.float32
    P = w.size
    mu = torch.empty(P, dtype=tdt, device="cuda:0")
    st = torch.empty(P, dtype=torch.int8, device="cuda:0")
    F.fpca_smooth_mean(h, F.Grid(M), F.FPCA_F64 if dt == "f64" else F.FPCA_F32, dev(torch, w), dev(torch, g),
                       F.FPCA_K_EPANECHNIKOV, hb, mu, st)
    h.sync()
    rb, rst, _, rmp = oracle.smooth(M, hb, w.astype(np.float64), g.astype(np.float64), want_moments=True)
    bad, band = status_agreement(host(st), rst, rmp)
    assert bad == 0
    ok = (host(st) == 0) & (rst == 0)
    tol = 1e-10 if dt == "f64" else 1e-5
    assert normwise_rel(host(mu), rb, ok) < tol
    fb = (host(st) == 1) & (rst == 1)
    if fb.any():
        assert normwise_rel(host(mu), rb, fb) < tol
    assert np.all(np.isnan(host(mu)[rst == 2]))


def test_mean_common_grid_full_size(torch, F, h):
    """Mean stage of the benchmark at its full size: common-grid binning of
    n = 5000 curves on 64 x 64 nodes (column sums over 79 row chunks with a
    ragged last chunk) and the smoother at h = 0.1, against the oracle."""
    _say("mean common grid 64x64 n=5000")
    from fpca_synth import make_c3
    ds = make_c3(n=5000)
    from paper_1510_04439_amd import pipeline as PL
    dd = PL.to_device(ds)
    P = int(np.prod(ds.M_mean))
    c = torch.empty(P, dtype=torch.float32, device="cuda:0")
    s = torch.empty_like(c)
    mu = torch.empty_like(c)
    st = torch.empty(P, dtype=torch.int8, device="cuda:0")
    F.fpca_bin(h, dd.grid_mean, F.FPCA_BIN_MEAN, dd.design, dd.dtype, F.FPCA_PREC_F32, dd.n, None, None, dd.y,
               None, 0, c, s)
    F.fpca_smooth_mean(h, dd.grid_mean, dd.dtype, c, s, F.FPCA_K_EPANECHNIKOV, ds.h_mean, mu, st)
    h.sync()
    Y = np.asarray(ds.y, np.float64).reshape(ds.n, P)
    rc, rs = oracle.bin_common_grid_mean(Y)
    assert normwise_rel(host(c), rc) < 1e-7 and normwise_rel(host(s), rs) < 1e-5
    rb, rst = oracle.smooth_mean(ds.M_mean, ds.h_mean, rc, rs)
    assert np.array_equal(host(st), rst)
    assert normwise_rel(host(mu), rb, rst == 0) < 1e-5


def test_end_to_end_c3_sampled(torch, F, h):
    """The benchmark's path at full size (64 x 64 common grid, n = 5000): mean,
    BF16x3 Gram binning and the analytic-weight covariance smoother, checked
    at sampled covariance nodes (and their transposes) against the oracle's
    FP64 Gram of the same data and its direct-window smoother."""
    _say("end-to-end c3 sampled")
    from fpca_synth import make_c3
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
    F.fpca_smooth_cov(h, dd.grid_cov, dd.dtype, None, PL.uniform_pair_weight(dd), bufs.G, bufs.mu,
                      F.FPCA_K_EPANECHNIKOV, ds.h_cov, bufs.gamma, bufs.status)
    h.sync()
    P = int(np.prod(ds.M_cov))
    Y = np.asarray(ds.y, np.float64).reshape(ds.n, P)
    rc, rs = oracle.bin_common_grid_mean(Y)
    mu, _ = oracle.smooth_mean(ds.M_mean, ds.h_mean, rc, rs)
    _, _, C, G = oracle.bin_common_grid(Y)
    rng = np.random.default_rng(33)
    idx = rng.integers(0, P * P, 300)
    p, q = idx // P, idx % P
    near = rng.integers(0, P, 60)  # nodes near the diagonal s = t, where the full system is solved
    p = np.concatenate([p, near])
    q = np.concatenate([q, np.clip(near + rng.integers(-2, 3, 60) * 64 + rng.integers(-2, 3, 60), 0, P - 1)])
    nodes = np.concatenate([p * P + q, q * P + p])
    rb, rst = oracle.smooth_cov_raw(ds.M_cov, ds.h_cov, C, G, nodes)
    m = len(p)
    ref = 0.5 * (rb[:m] + rb[m:]) - mu[p] * mu[q]
    ok = (rst[:m] == 0) & (rst[m:] == 0)
    gam = host(bufs.gamma)
    assert normwise_rel(gam[p, q], ref, ok) < 1e-4
    assert status_agreement(host(bufs.status).reshape(-1)[nodes], rst)[0] == 0


def _cov_inputs(rng, M, d):
    """Pair weights and raw products on the 2d-grid from random curves (oracle binning)."""
    off, t, y = rand_irregular(rng, d, 60, 2, 25, np.float64)
    C, G = oracle.bin_cov_pairs(M, off, t, y)
    return C.astype(np.float32), G.astype(np.float32)


_COV_CASES = [((51,), 0.1, "f64", 0), ((12, 12), 0.2, "f32", 0), ((6, 6, 6), 0.45, "f32", 0),
              ((32, 32), 0.08, "f32", 3000), ((11, 14), 0.25, "f32", 0), ((24, 24), 0.27, "f32", 1500),
              ((7, 9), 0.6, "f32", 0), ((64, 64), 0.1, "f32", 800)]


# both engines on the small grids; the large ones (sampled nodes) run the
# queue kernel, as AUTO does for them
@pytest.mark.parametrize("M,hb,dt,sample,eng", [c + ("queue",) for c in _COV_CASES] +
                         [c + ("passes",) for c in _COV_CASES if c[3] == 0])
def test_smooth_cov_parity(torch, F, h, M, hb, dt, sample, eng):
    with engine(F, h, F.FPCA_ENGINE_QUEUE if eng == "queue" else F.FPCA_ENGINE_PASSES):
        _smooth_cov_parity(torch, F, h, M, hb, dt, sample)


def _smooth_cov_parity(torch, F, h, M, hb, dt, sample):
    _say(f"smooth_cov M={M} h={hb} {dt} sample={sample}")
    rng = np.random.default_rng(300 + sum(M))
    d = len(M)
    P = int(np.prod(M))
    if P <= 300:
        C, G = _cov_inputs(rng, M, d)
    else:
        C = (rng.random((P, P)) + 0.01)
        C = (C + C.T) * 0.5
        G = C * rng.standard_normal((P, P))
        G = (G + G.T) * 0.5
    npdt = np.float64 if dt == "f64" else np.float32
    C, G = C.astype(npdt), G.astype(npdt)
    mu = rng.standard_normal(P).astype(npdt)
    tdt = torch.float64 if dt == "f64" else torch.float32
    gam = torch.empty(P, P, dtype=tdt, device="cuda:0")
    st = torch.empty(P, P, dtype=torch.int8, device="cuda:0")
    F.fpca_smooth_cov(h, F.Grid(M), F.FPCA_F64 if dt == "f64" else F.FPCA_F32, dev(torch, C), 0.0,
                      dev(torch, G), dev(torch, mu), F.FPCA_K_EPANECHNIKOV, hb, gam, st)
    h.sync()
    gam_h, st_h = host(gam), host(st)
    tol = 1e-10 if dt == "f64" else 1e-5
    if sample == 0:
        rb, rst = oracle.smooth_cov_raw(M, hb, C.astype(np.float64), G.astype(np.float64))
        ref = oracle.assemble_cov(rb.reshape(P, P), mu.astype(np.float64))
        assert status_agreement(st_h, rst)[0] == 0
        okm = (rst.reshape(P, P) == 0) & (rst.reshape(P, P).T == 0)
        assert normwise_rel(gam_h, ref, okm) < tol
    else:
        # sampled nodes (pairs (p,q) and (q,p) both evaluated) incl. the corners
        idx = rng.integers(0, P * P, sample)
        idx[:4] = [0, P - 1, (P - 1) * P, P * P - 1]
        p, q = idx // P, idx % P
        nodes = np.concatenate([idx, q * P + p])
        rb, rst = oracle.smooth_cov_raw(M, hb, C.astype(np.float64), G.astype(np.float64), nodes)
        m = len(idx)
        ref = 0.5 * (rb[:m] + rb[m:]) - mu[p].astype(np.float64) * mu[q]
        ok = (rst[:m] == 0) & (rst[m:] == 0)
        assert normwise_rel(gam_h[p, q], ref, ok) < tol
        assert status_agreement(st_h.reshape(-1)[nodes], rst)[0] == 0
    assert np.array_equal(gam_h, gam_h.T)


@pytest.mark.parametrize("M,hb", [((10, 10), 0.3), ((16, 16), 0.3), ((9, 12), 0.25)])
def test_smooth_cov_analytic_common_grid(torch, F, h, M, hb):
    """C = NULL (complete common-grid design, pair weight c_uniform off the
    diagonal) equals passing C = c_uniform (1 - delta) explicitly."""
    _say(f"smooth_cov analytic C M={M} h={hb}")
    rng = np.random.default_rng(11)
    P = int(np.prod(M))
    c0 = 0.37
    G = rng.standard_normal((P, P)) * c0
    G = ((G + G.T) / 2).astype(np.float32)
    np.fill_diagonal(G, 0)
    C = np.full((P, P), c0, np.float32)
    np.fill_diagonal(C, 0)
    mu = rng.standard_normal(P).astype(np.float32)
    outs = []
    for Cin in (None, dev(torch, C)):
        gam = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
        F.fpca_smooth_cov(h, F.Grid(M), F.FPCA_F32, Cin, c0, dev(torch, G), dev(torch, mu),
                          F.FPCA_K_EPANECHNIKOV, hb, gam)
        outs.append(host(gam))
    h.sync()
    rb, rst = oracle.smooth_cov_raw(M, hb, C.astype(np.float64), G.astype(np.float64))
    ref = oracle.assemble_cov(rb.reshape(P, P), mu.astype(np.float64))
    ok = (rst.reshape(P, P) == 0) & (rst.reshape(P, P).T == 0)
    for o in outs:
        assert normwise_rel(o, ref, ok) < 1e-5
    with pytest.raises(F.FpcaError):
        F.fpca_smooth_cov(h, F.Grid(M), F.FPCA_F32, None, 0.0, dev(torch, G), None, F.FPCA_K_EPANECHNIKOV, hb,
                          torch.empty(P, P, dtype=torch.float32, device="cuda:0"))


# ------------------------------------------------------------------ batched CV
@pytest.mark.parametrize("M,nf,hs", [((7, 6), 3, [0.2, 0.35, 0.6]), ((4, 5, 4), 5, [0.3, 0.55]),
                                     ((12, 12), 4, [0.1, 0.25])])
def test_cv_batched_parity(torch, F, h, M, nf, hs):
    """Scores of every (bandwidth, fold) job against the oracle: smoother on the
    other folds' pairs (full grid), then sum [Q_f - 2 G_f Ghat + C_f Ghat^2]."""
    _say(f"cv M={M} folds={nf} h={hs}")
    rng = np.random.default_rng(40 + len(M))
    d = len(M)
    n = 30
    off, t, y = rand_irregular(rng, d, n, 1, 14, np.float32)
    folds = fold_assignment(n, nf, seed=9)
    P = int(np.prod(M))
    t64, y64 = t.astype(np.float64), y.astype(np.float64)
    slabs = [oracle.bin_cov_pairs(M, off, t64, y64, folds, fs, want_Q=True) for fs in [-1] + list(range(nf))]
    Ch, Gh, Qh = (np.stack([s[i] for s in slabs]).astype(np.float32).astype(np.float64) for i in range(3))
    C, G, Q = (dev(torch, a.astype(np.float32)) for a in (Ch, Gh, Qh))
    scores = F.fpca_cv_batched(h, F.FPCA_F32, [(F.Grid(M), C, G, Q)], nf, hs)[0]
    ref = np.zeros((len(hs), nf))
    for i, hb in enumerate(hs):
        for f in range(nf):
            b, st = oracle.smooth_cov_raw(M, hb, Ch[0] - Ch[f + 1], Gh[0] - Gh[f + 1])
            Ghat = oracle.assemble_cov(b.reshape(P, P), np.zeros(P))
            ref[i, f] = oracle.cv_score(Qh[f + 1], Gh[f + 1], Ch[f + 1], Ghat)
    np.testing.assert_allclose(scores, ref, rtol=1e-5)


# ------------------------------------------------------------------ eigen
def test_eig_closed_form_and_oracle(torch, F, h):
    _say("eig closed form")
    M = (24, 20)
    P = 480
    index = [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1)]
    lam = 2.0 ** -np.arange(1, 7)
    pts = grid_points(M)
    Phi = np.stack([fourier_1d(a, pts[:, 0]) * fourier_1d(b, pts[:, 1]) for a, b in index], 1)
    Gam = (Phi * lam) @ Phi.T
    rng = np.random.default_rng(3)
    E = rng.standard_normal((P, P)) * 1e-4
    Gam = Gam + (E + E.T) / 2
    om = oracle.quad_weights(M, rule="trapezoid")
    k, p, q, seed = 6, 10, 2, 7
    for dt in ("f64", "f32"):
        npdt = np.float64 if dt == "f64" else np.float32
        tdt = torch.float64 if dt == "f64" else torch.float32
        ef = torch.empty(k, P, dtype=tdt, device="cuda:0")
        ev, fve = F.fpca_eig_randomized(h, F.FPCA_F64 if dt == "f64" else F.FPCA_F32,
                                        F.FPCA_PREC_F64 if dt == "f64" else F.FPCA_PREC_F32, F.Grid(M),
                                        dev(torch, Gam.astype(npdt)), dev(torch, om), k, p, q, seed, ef)
        rev, rphi, rfve = oracle.eig_randomized(Gam.astype(npdt).astype(np.float64), om, k, p, q, seed)
        tol = 1e-10 if dt == "f64" else 1e-5
        assert np.abs(ev - rev).max() <= tol * np.abs(rev).max()
        assert np.abs(fve - rfve).max() <= tol
        phi = host(ef).T
        for j in range(k):
            err = min(np.abs(phi[:, j] - rphi[:, j]).max(), np.abs(phi[:, j] + rphi[:, j]).max())
            assert err <= 100 * tol * np.abs(rphi[:, j]).max(), (dt, j, err)
        np.testing.assert_allclose(ev, lam, rtol=2e-3)


@pytest.mark.parametrize("k,p,dt,rank", [(6, 24, "f32", 0), (8, 32, "f32", 0), (10, 54, "f32", 0),
                                          (8, 32, "f64", 0), (10, 54, "f64", 0), (6, 24, "f32", 12),
                                          (10, 38, "f32", 20)])
def test_eig_basis_widths(torch, F, h, k, p, dt, rank):
    """Basis widths r = k + p of 30, 40 and 64 (the 32-, 48- and 64-column
    Cholesky and Jacobi kernels; at 48 every thread forms both of its
    rotations), against the oracle's randomized eig. rank > 0: the surface has
    that rank, so the orthonormalizations drop columns."""
    _say(f"eig widths k={k} p={p} {dt} rank={rank}")
    M = (24, 20)
    P = 480
    rng = np.random.default_rng(40 + k + p + rank)
    nv = rank if rank else 60
    V = np.linalg.qr(rng.standard_normal((P, nv)))[0]
    lam = 1.5 ** -np.arange(nv)
    Gam = (V * lam) @ V.T
    if not rank:
        E = rng.standard_normal((P, P)) * 1e-6
        Gam = Gam + (E + E.T) / 2
    om = oracle.quad_weights(M, rule="trapezoid")
    npdt = np.float64 if dt == "f64" else np.float32
    tdt = torch.float64 if dt == "f64" else torch.float32
    ef = torch.empty(k, P, dtype=tdt, device="cuda:0")
    ev, fve = F.fpca_eig_randomized(h, F.FPCA_F64 if dt == "f64" else F.FPCA_F32,
                                    F.FPCA_PREC_F64 if dt == "f64" else F.FPCA_PREC_F32, F.Grid(M),
                                    dev(torch, Gam.astype(npdt)), dev(torch, om), k, p, 2, 11, ef)
    rev, rphi, rfve = oracle.eig_randomized(Gam.astype(npdt).astype(np.float64), om, k, p, 2, 11)
    tol = 1e-10 if dt == "f64" else 1e-5
    assert np.abs(ev - rev).max() <= tol * np.abs(rev).max()
    assert np.abs(fve - rfve).max() <= tol
    phi = host(ef).T
    for j in range(k):
        # eigenvector tolerance scales with the gap to the neighbouring eigenvalues
        gap = min(abs(rev[j] - rev[j - 1]) if j else np.inf, abs(rev[j] - rev[j + 1]) if j + 1 < k else np.inf)
        scale = max(1.0, 0.1 * rev[0] / gap) if np.isfinite(gap) else 1.0
        err = min(np.abs(phi[:, j] - rphi[:, j]).max(), np.abs(phi[:, j] + rphi[:, j]).max())
        assert err <= 100 * tol * scale * np.abs(rphi[:, j]).max(), (j, err)


@pytest.mark.parametrize("M,k,p,rank", [((24, 20), 6, 24, 0), ((24, 20), 10, 54, 0), ((23, 19), 8, 32, 0),
                                          ((24, 20), 6, 24, 12), ((64, 64), 20, 10, 0), ((9, 7), 3, 5, 0)])
def test_eig_bf16x3_products(torch, F, h, M, k, p, rank):
    """FP32 surfaces with the products of A and the basis on BF16x3 MFMA
    (k_panel_bf16x3), against the oracle's FP64 randomized eig. Grids: P = 480
    (a partial 64-node column block), P = 437 (rows not 16-byte aligned: the
    scalar loads), the benchmark's P = 4096 with r = 30, and P = 63 with a
    16-column basis (one 64-node column block, one K chunk). Bars from the
    split: each product drops lo*lo and rounds the lo parts, <= 3 2^-16 of
    |x y| per term and about 2^-17 typically, so A Q carries a relative error
    of order 1e-5 and the eigenvalues 1e-4 of the largest (the Gram product's
    stated BF16x3 bound); eigenfunctions 1e-2 times the gap factor."""
    _say(f"eig bf16x3 M={M} k={k} p={p} rank={rank}")
    P = int(np.prod(M))
    rng = np.random.default_rng(90 + P + k + rank)
    nv = rank if rank else min(60, P // 4)
    V = np.linalg.qr(rng.standard_normal((P, nv)))[0]
    lam = 1.5 ** -np.arange(nv) if P < 1000 else (1.0 + np.arange(nv)) ** -2.0
    Gam = (V * lam) @ V.T
    if not rank:
        E = rng.standard_normal((P, P)) * 1e-6
        Gam = Gam + (E + E.T) / 2
    Gam = Gam.astype(np.float32)
    om = oracle.quad_weights(M, rule="trapezoid")
    out = {}
    for prec in (F.FPCA_PREC_BF16X3, F.FPCA_PREC_F32):
        ef = torch.empty(k, P, dtype=torch.float32, device="cuda:0")
        ev, fve = F.fpca_eig_randomized(h, F.FPCA_F32, prec, F.Grid(M), dev(torch, Gam), dev(torch, om), k, p, 2, 13,
                                        ef)
        out[prec] = (ev, fve, host(ef).T)
    rev, rphi, rfve = oracle.eig_randomized(Gam.astype(np.float64), om, k, p, 2, 13)
    ev, fve, phi = out[F.FPCA_PREC_BF16X3]
    tol = 1e-4
    assert np.abs(ev - rev).max() <= tol * np.abs(rev).max()
    assert np.abs(fve - rfve).max() <= tol
    assert np.abs(ev - out[F.FPCA_PREC_F32][0]).max() <= tol * np.abs(rev).max()
    for j in range(k):
        gap = min(abs(rev[j] - rev[j - 1]) if j else np.inf, abs(rev[j] - rev[j + 1]) if j + 1 < k else np.inf)
        scale = max(1.0, 0.1 * rev[0] / gap) if np.isfinite(gap) else 1.0
        err = min(np.abs(phi[:, j] - rphi[:, j]).max(), np.abs(phi[:, j] + rphi[:, j]).max())
        assert err <= 100 * tol * scale * np.abs(rphi[:, j]).max(), (j, err)


def test_eig_full_size(torch, F, h):
    """The benchmark's eig configuration at its full size: P = 64^2 = 4096 nodes,
    k = 20, oversample 10, two power iterations, FP32 surface (the launch
    configuration of the benchmark: 32-column basis, 16-way K split of the
    products), against the oracle's FP64 randomized eig on the same surface."""
    _say("eig full size P=4096 k=20 p=10 q=2")
    M = (64, 64)
    P = 4096
    rng = np.random.default_rng(77)
    nv = 200
    V = np.linalg.qr(rng.standard_normal((P, nv)))[0]
    lam = (1.0 + np.arange(nv)) ** -2.0
    Gam = ((V * lam) @ V.T).astype(np.float32)
    ef = torch.empty(20, P, dtype=torch.float32, device="cuda:0")
    ev, fve = F.fpca_eig_randomized(h, F.FPCA_F32, F.FPCA_PREC_F32, F.Grid(M), dev(torch, Gam), None, 20, 10, 2, 7,
                                    ef)
    om = oracle.quad_weights(M)
    rev, rphi, rfve = oracle.eig_randomized(Gam.astype(np.float64), om, 20, 10, 2, 7)
    assert np.abs(ev - rev).max() <= 1e-5 * rev[0]
    assert np.abs(fve - rfve).max() <= 1e-5
    phi = host(ef).T
    for j in range(20):
        gap = min(abs(rev[j] - rev[j - 1]) if j else np.inf, abs(rev[j] - rev[j + 1]) if j + 1 < 20 else np.inf)
        scale = max(1.0, 0.1 * rev[0] / gap)
        err = min(np.abs(phi[:, j] - rphi[:, j]).max(), np.abs(phi[:, j] + rphi[:, j]).max())
        assert err <= 1e-3 * scale * np.abs(rphi[:, j]).max(), (j, err)


def test_eig_degenerate_surfaces(torch, F, h):
    """A zero surface (every basis column dropped: eigenvalues, FVE and
    eigenfunctions 0) and a rank-one surface (one eigenpair, the rest 0; FVE 1)."""
    _say("eig degenerate")
    M = (8, 8)
    P = 64
    om = oracle.quad_weights(M)
    x = np.arange(P) / P
    for name, Gam in (("zero", np.zeros((P, P))), ("rank1", np.outer(x, x))):
        ef = torch.empty(3, P, dtype=torch.float64, device="cuda:0")
        ev, fve = F.fpca_eig_randomized(h, F.FPCA_F64, F.FPCA_PREC_F64, F.Grid(M), dev(torch, Gam), dev(torch, om),
                                        3, 5, 1, 3, ef)
        phi = host(ef).T
        rev, rphi, rfve = oracle.eig_randomized(Gam, om, 3, 5, 1, 3)
        assert np.all(np.isfinite(ev)) and np.all(np.isfinite(fve)) and np.all(np.isfinite(phi))
        assert np.abs(ev - rev).max() <= 1e-10 * max(1.0, np.abs(rev).max()), name
        assert np.abs(fve - rfve).max() <= 1e-10, name
        if name == "zero":
            assert np.all(ev == 0) and np.all(phi == 0)
        else:
            err = min(np.abs(phi[:, 0] - rphi[:, 0]).max(), np.abs(phi[:, 0] + rphi[:, 0]).max())
            assert err <= 1e-8 * np.abs(rphi[:, 0]).max()
            assert np.all(phi[:, 1:] == 0) and np.all(ev[1:] == 0)


def test_eig_riemann_default_weights_and_mask(torch, F, h):
    _say("eig default weights")
    M = (8, 8, 8)
    P = 512
    mask = disk_time_mask(M)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((P, 5))
    Gam = X @ np.diag([5, 4, 3, 2, 1.0]) @ X.T
    Gam[mask == 0, :] = 0
    Gam[:, mask == 0] = 0
    om = oracle.quad_weights(M, mask)
    ef = torch.empty(4, P, dtype=torch.float32, device="cuda:0")
    ev, fve = F.fpca_eig_randomized(h, F.FPCA_F32, F.FPCA_PREC_F32, F.Grid(M, dev(torch, mask)),
                                    dev(torch, Gam.astype(np.float32)), None, 4, 6, 1, 9, ef)
    rev, rphi, rfve = oracle.eig_dense(Gam.astype(np.float32).astype(np.float64), om, 4)
    assert np.abs(ev - rev).max() <= 1e-5 * rev.max()
    phi = host(ef).T
    for j in range(4):
        assert np.abs(phi[:, j] - rphi[:, j]).max() <= 1e-3 * np.abs(rphi[:, j]).max()
    assert np.all(phi[mask == 0] == 0)


# ------------------------------------------------------------------ end to end
def test_end_to_end_c1(torch, F, h):
    """d=1 FP64 workload, whole path, against the oracle's whole path."""
    _say("end-to-end c1")
    from paper_1510_04439_amd import pipeline as PL
    ds = make_c1()
    dd = PL.to_device(ds)
    bufs = PL.alloc(dd, ds.k)
    PL.fit(h, dd, bufs, ds.h_mean, ds.h_cov, ds.k, ds.oversample, ds.power_iters, ds.rp_seed)
    h.sync()
    c, s, _, _ = oracle.bin_mean(ds.M_mean, ds.offsets, ds.t, ds.y)
    mu, mst = oracle.smooth_mean(ds.M_mean, ds.h_mean, c, s)
    assert normwise_rel(host(bufs.mu), mu) < 1e-12
    C, G = oracle.bin_cov_pairs(ds.M_cov, ds.offsets, ds.t, ds.y)
    assert normwise_rel(host(bufs.G), G) < 1e-12
    gh, gst = oracle.smooth_cov_raw(ds.M_cov, ds.h_cov, C, G)
    gam = oracle.assemble_cov(gh.reshape(51, 51), mu[::2])
    assert normwise_rel(host(bufs.gamma), gam) < 1e-11
    om = oracle.quad_weights(ds.M_cov)
    ev, phi, fve = oracle.eig_randomized(gam, om, ds.k, ds.oversample, ds.power_iters, ds.rp_seed)
    assert np.abs(bufs.evals - ev).max() < 1e-10 * ev.max()
    for j in range(ds.k):
        assert np.abs(host(bufs.efuns)[j] - phi[:, j]).max() < 1e-8
    # statistical sanity against the generating model (not parity)
    np.testing.assert_allclose(bufs.evals, ds.lambdas, rtol=0.35)

"""GPU parity of the PACE scores (eq. 2.7) against the oracle.

The oracle solves the N_i x N_i system as the equations write it; the HIP
kernel solves the equivalent k x k system. Bars: FP64 1e-10 and FP32 storage
1e-5, normwise (max |got - ref| <= tol * max |ref|).
"""
import sys

import numpy as np
import pytest

import oracle

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


def _run(torch, F, h, M, design, off, t, y, mu, efuns, lam, s2, dt):
    npdt = np.float64 if dt == "f64" else np.float32
    n = (len(off) - 1) if off is not None else y.shape[0]
    k = efuns.shape[1]
    P = efuns.shape[0]
    y, mu = y.astype(npdt), mu.astype(npdt)
    efc = np.ascontiguousarray(efuns.T).astype(npdt)  # P x k column-major
    tt = None if t is None else t.astype(npdt)
    out = torch.empty(n * k, dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda:0")
    F.fpca_pace_scores(h, F.Grid(M), design, F.FPCA_F64 if dt == "f64" else F.FPCA_F32, n,
                       None if off is None else dev(torch, off), None if tt is None else dev(torch, tt),
                       dev(torch, y), dev(torch, mu), dev(torch, efc), k, lam, s2, out)
    h.sync()
    got = out.cpu().numpy().astype(np.float64).reshape(n, k)
    ref = oracle.pace_scores(M, off, None if tt is None else tt.astype(np.float64), y.astype(np.float64),
                             mu.astype(np.float64), efc.T.astype(np.float64).reshape(P, k), lam, s2)
    return got, ref


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("M,k", [((12, 10), 5), ((41,), 32), ((6, 5, 4), 9)])
def test_pace_irregular(torch, F, h, dt, M, k):
    _say(f"pace irregular M={M} k={k} {dt}")
    rng = np.random.default_rng(len(M) * 100 + k)
    d = len(M)
    P = int(np.prod(M))
    n = 40
    Ni = rng.integers(0, 61, size=n)
    Ni[3] = 0
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    N = int(off[-1])
    t = rng.random((N, d))
    t[5, 0] = 1.25  # outside the domain: left out on both sides
    y = rng.standard_normal(N)
    mu = rng.standard_normal(P)
    efuns = rng.standard_normal((P, k)) / np.sqrt(P)
    lam = np.abs(rng.standard_normal(k)) + 0.1
    lam[k // 2] = -0.3  # a negative Ritz value: left out
    got, ref = _run(torch, F, h, M, F.FPCA_IRREGULAR, off, t, y, mu, efuns, lam, 0.05, dt)
    assert np.all(got[3] == 0) and np.all(got[:, k // 2] == 0)
    tol = 1e-10 if dt == "f64" else 1e-5
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("mixed", [False, True])
def test_pace_common_grid(torch, F, h, dt, mixed):
    """mixed = False: every curve has missing values (per-curve systems);
    mixed = True: most curves are complete and take the shared factor, a few
    have missing values, one component has a negative Ritz value."""
    _say(f"pace common grid {dt} mixed={mixed}")
    rng = np.random.default_rng(77 + mixed)
    M = (8, 9)
    P = 72
    n, k = 30, 12
    Y = rng.standard_normal((n, P))
    if mixed:
        Y[[2, 11, 19], [5, 40, 71]] = np.nan
    else:
        Y[rng.random((n, P)) < 0.25] = np.nan
    Y[7] = np.nan
    mu = rng.standard_normal(P)
    efuns = rng.standard_normal((P, k)) / np.sqrt(P)
    lam = np.linspace(2.0, 0.05, k)
    if mixed:
        lam[4] = -0.1
    got, ref = _run(torch, F, h, M, F.FPCA_COMMON_GRID, None, None, Y, mu, efuns, lam, 0.2, dt)
    assert np.all(got[7] == 0)
    if mixed:
        assert np.all(got[:, 4] == 0)
    tol = 1e-10 if dt == "f64" else 1e-5
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("M,k", [((16, 12), 17), ((9, 7), 20), ((64,), 19), ((10, 10), 24)])
def test_pace_common_grid_components_past_16(torch, F, h, M, k, dt):
    """k > 16 on the common grid: the components past the first 16 take the
    second MFMA tile of the shared matrix and of the right-hand sides; node
    loads by 16-byte vectors (P % 4 == 0) or one at a time; 40 complete
    curves and one with a missing value (solved on its own)."""
    _say(f"pace common grid M={M} k={k} {dt}")
    rng = np.random.default_rng(k + len(M))
    P = int(np.prod(M))
    n = 41
    Y = rng.standard_normal((n, P))
    Y[13, P // 3] = np.nan
    mu = rng.standard_normal(P)
    efuns = rng.standard_normal((P, k)) / np.sqrt(P)
    lam = np.geomspace(2.0, 0.02, k)
    got, ref = _run(torch, F, h, M, F.FPCA_COMMON_GRID, None, None, Y, mu, efuns, lam, 0.1, dt)
    tol = 1e-10 if dt == "f64" else 1e-5
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_pace_argument_errors(torch, F, h):
    _say("pace argument errors")
    M = (5,)
    y = torch.zeros(10, dtype=torch.float64, device="cuda:0")
    mu = torch.zeros(5, dtype=torch.float64, device="cuda:0")
    ef = torch.zeros(5 * 33, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(2 * 33, dtype=torch.float64, device="cuda:0")
    for k, s2 in ((33, 0.1), (2, 0.0), (2, float("nan"))):
        with pytest.raises(F.FpcaError):
            F.fpca_pace_scores(h, F.Grid(M), F.FPCA_COMMON_GRID, F.FPCA_F64, 2, None, None, y, mu, ef, k,
                               np.ones(k), s2, out)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("P,n,k", [(300, 37, 7), (4096, 50, 20), (17, 1, 32), (300, 130, 9), (257, 64, 24),
                                   (1000, 65, 17)])
def test_reconstruct_parity(torch, F, h, dt, P, n, k):
    _say(f"reconstruct P={P} n={n} k={k} {dt}")
    rng = np.random.default_rng(P + n + k)
    npdt = np.float64 if dt == "f64" else np.float32
    mu = rng.standard_normal(P).astype(npdt)
    ef = rng.standard_normal((P, k)).astype(npdt)
    sc = rng.standard_normal((n, k)).astype(npdt)
    out = torch.empty(n * P, dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda:0")
    F.fpca_reconstruct(h, F.FPCA_F64 if dt == "f64" else F.FPCA_F32, P, n, k, dev(torch, mu),
                       dev(torch, np.ascontiguousarray(ef.T)), dev(torch, sc), out)
    h.sync()
    got = out.cpu().numpy().astype(np.float64).reshape(n, P)
    ref = oracle.reconstruct(mu.astype(np.float64), ef.astype(np.float64), sc.astype(np.float64))
    tol = 1e-13 if dt == "f64" else 1e-6
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


def test_scores_and_reconstruction_end_to_end_c1(torch, F, h):
    """d = 1 FP64 workload on the 51-node grid, all on the GPU: binning, mean
    and second-moment smooths, covariance, randomized eigendecomposition,
    noise variance, PACE scores and reconstruction, against the oracle's
    chain. Then, statistically (not parity), the reconstruction is closer to
    the noisy observations' curves than the mean alone."""
    _say("scores and reconstruction end-to-end c1")
    from fpca_synth import make_c1
    ds = make_c1()
    M = ds.M_cov
    P = int(np.prod(M))
    grid = F.Grid(M)
    n, k, hs = ds.n, ds.k, 0.04
    off, t, y = dev(torch, ds.offsets), dev(torch, ds.t), dev(torch, ds.y)
    f64 = torch.float64
    c = torch.empty(P, dtype=f64, device="cuda:0")
    s, sq, mu, b0 = (torch.empty_like(c) for _ in range(4))
    F.fpca_bin(h, grid, F.FPCA_BIN_MEAN, F.FPCA_IRREGULAR, F.FPCA_F64, F.FPCA_PREC_F64, n, off, t, y, None, 0,
               c, s, sq)
    F.fpca_smooth_mean(h, grid, F.FPCA_F64, c, s, F.FPCA_K_EPANECHNIKOV, hs, mu)
    F.fpca_smooth_mean(h, grid, F.FPCA_F64, c, sq, F.FPCA_K_EPANECHNIKOV, hs, b0)
    C = torch.empty(P * P, dtype=f64, device="cuda:0")
    G, gam = torch.empty_like(C), torch.empty_like(C)
    F.fpca_bin(h, grid, F.FPCA_BIN_COV, F.FPCA_IRREGULAR, F.FPCA_F64, F.FPCA_PREC_F64, n, off, t, y, None, 0, C, G)
    F.fpca_smooth_cov(h, grid, F.FPCA_F64, C, 0.0, G, mu, F.FPCA_K_EPANECHNIKOV, hs, gam)
    ef = torch.empty(k * P, dtype=f64, device="cuda:0")
    ev, _ = F.fpca_eig_randomized(h, F.FPCA_F64, F.FPCA_PREC_F64, grid, gam, None, k, ds.oversample,
                                  ds.power_iters, ds.rp_seed, ef)
    s2, _ = F.fpca_noise_variance(h, grid, F.FPCA_F64, b0, mu, gam, None)
    sc = torch.empty(n * k, dtype=f64, device="cuda:0")
    F.fpca_pace_scores(h, grid, F.FPCA_IRREGULAR, F.FPCA_F64, n, off, t, y, mu, ef, k, ev, s2, sc)
    xh = torch.empty(n * P, dtype=f64, device="cuda:0")
    F.fpca_reconstruct(h, F.FPCA_F64, P, n, k, mu, ef, sc, xh)
    h.sync()

    rc, rs, _, _ = oracle.bin_mean(M, ds.offsets, ds.t, ds.y)
    _, rsq, _, _ = oracle.bin_mean(M, ds.offsets, ds.t, np.asarray(ds.y, np.float64) ** 2)
    rmu, _ = oracle.smooth_mean(M, hs, rc, rs)
    rb0, _ = oracle.smooth_mean(M, hs, rc, rsq)
    rC, rG = oracle.bin_cov_pairs(M, ds.offsets, ds.t, ds.y)
    gh, _ = oracle.smooth_cov_raw(M, hs, rC, rG)
    rgam = oracle.assemble_cov(gh.reshape(P, P), rmu)
    rev, rphi, _ = oracle.eig_randomized(rgam, oracle.quad_weights(M), k, ds.oversample, ds.power_iters,
                                         ds.rp_seed)
    _, rs2, _ = oracle.noise_variance(rb0, rmu, rgam)
    rsc = oracle.pace_scores(M, ds.offsets, ds.t, ds.y, rmu, rphi, rev, rs2)
    rxh = oracle.reconstruct(rmu, rphi, rsc)
    assert abs(s2 - rs2) < 1e-9 * abs(rs2)
    got_sc = sc.cpu().numpy().reshape(n, k)
    assert np.abs(got_sc - rsc).max() < 1e-7 * np.abs(rsc).max()
    got_xh = xh.cpu().numpy().reshape(n, P)
    assert np.abs(got_xh - rxh).max() < 1e-7 * np.abs(rxh).max()
    # statistical: at the observation points, the reconstruction explains
    # more of the data than the mean does
    node, wt, _ = oracle.bin_corners(M, ds.t)
    curve = np.repeat(np.arange(n), np.diff(ds.offsets))
    fit = (wt * got_xh[curve[:, None], node]).sum(1)
    base = (wt * rmu[node]).sum(1)
    assert np.mean((ds.y - fit) ** 2) < 0.5 * np.mean((ds.y - base) ** 2)


def test_pace_common_grid_full_size(torch, F, h):
    """The benchmark's shape: 5000 complete curves on 64 x 64 nodes, k = 20,
    FP32 storage; 12 sampled curves against the oracle's N_i x N_i solve
    (4096 x 4096 per curve)."""
    _say("pace common grid 64x64 n=5000 k=20")
    rng = np.random.default_rng(5)
    M = (64, 64)
    P = 4096
    n, k = 5000, 20
    Y = rng.standard_normal((n, P)).astype(np.float32)
    mu = (0.1 * rng.standard_normal(P)).astype(np.float32)
    efuns = (rng.standard_normal((P, k)) / np.sqrt(P)).astype(np.float32)
    lam = np.geomspace(1.0, 0.01, k)
    out = torch.empty(n * k, dtype=torch.float32, device="cuda:0")
    F.fpca_pace_scores(h, F.Grid(M), F.FPCA_COMMON_GRID, F.FPCA_F32, n, None, None, dev(torch, Y), dev(torch, mu),
                       dev(torch, np.ascontiguousarray(efuns.T)), k, lam, 0.05, out)
    h.sync()
    got = out.cpu().numpy().reshape(n, k).astype(np.float64)
    rows = rng.choice(n, 12, replace=False)
    ref = oracle.pace_scores(M, None, None, Y[rows].astype(np.float64), mu.astype(np.float64),
                             efuns.astype(np.float64), lam, 0.05)
    assert np.abs(got[rows] - ref).max() <= 1e-5 * np.abs(ref).max()

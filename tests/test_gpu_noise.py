"""GPU parity of the noise-variance estimator (eq. 2.6) against the oracle.

Bars: FP64 inputs to 1e-12 (the same FP64 formula, summed in another order);
FP32 inputs: per-node values within the FP32 rounding of the output, the
FP64 average to 1e-12; the counted-node total exact.
"""
import sys

import numpy as np
import pytest

import oracle
from fpca_synth import disk_time_mask, make_c1

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


@pytest.mark.parametrize("M", [(37,), (24, 19), (9, 8, 7)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("masked", [False, True])
def test_noise_variance_parity(torch, F, h, M, dt, masked):
    _say(f"noise_variance M={M} {dt} masked={masked}")
    rng = np.random.default_rng(sum(M) + masked)
    P = int(np.prod(M))
    npdt = np.float64 if dt == "f64" else np.float32
    b0 = (1.0 + rng.random(P)).astype(npdt)
    b0[rng.random(P) < 0.05] = np.nan  # EMPTY windows of the second-moment smoother
    mu = rng.standard_normal(P).astype(npdt)
    g = rng.standard_normal((P, P))
    gam = (0.5 * (g + g.T)).astype(npdt)
    mask = None
    if masked:
        if len(M) == 3:
            mask = disk_time_mask(M).astype(np.uint8).reshape(-1)
        else:
            mask = (rng.random(P) < 0.7).astype(np.uint8)
    grid = F.Grid(M, None if mask is None else dev(torch, mask))
    out = torch.empty(P, dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda:0")
    s2, cnt = F.fpca_noise_variance(h, grid, F.FPCA_F64 if dt == "f64" else F.FPCA_F32, dev(torch, b0),
                                    dev(torch, mu), dev(torch, gam), out)
    rt, rs2, rcnt = oracle.noise_variance(b0.astype(np.float64), mu.astype(np.float64), gam.astype(np.float64),
                                          mask)
    got = out.cpu().numpy().astype(np.float64)
    assert cnt == rcnt
    assert np.array_equal(np.isnan(got), np.isnan(rt))
    fin = np.isfinite(rt)
    scale = np.abs(rt[fin]).max()
    tol = 1e-12 if dt == "f64" else 2.0 ** -23
    assert np.abs(got[fin] - rt[fin]).max() <= tol * scale
    if mask is not None:
        assert np.all(got[mask == 0] == 0)
    assert abs(s2 - rs2) <= 1e-12 * scale


def test_noise_variance_empty_domain(torch, F, h):
    """No node counts (all outside Omega): NaN and count 0."""
    _say("noise_variance empty")
    M = (5, 4)
    P = 20
    mask = np.zeros(P, np.uint8)
    b0 = np.ones(P)
    grid = F.Grid(M, dev(torch, mask))
    s2, cnt = F.fpca_noise_variance(h, grid, F.FPCA_F64, dev(torch, b0), dev(torch, b0),
                                    dev(torch, np.eye(P)), None)
    assert cnt == 0 and np.isnan(s2)


def test_noise_variance_end_to_end_c1(torch, F, h):
    """d = 1 FP64 workload (noise sd 0.1): binned squared responses, mean and
    second-moment smooths, covariance, noise variance on the 51-node covariance
    grid, all on the GPU, against the oracle's chain; then the estimate
    against the generating noise variance (statistical, not parity). The
    smoothing bias of b0 and of Gamma's diagonal grows like h^2 (about 0.2 at
    h = 0.1 for these curves), so all three smooths use h = 0.04 here."""
    _say("noise_variance end-to-end c1")
    ds = make_c1()
    M = ds.M_cov
    P = int(np.prod(M))
    grid = F.Grid(M)
    hs = 0.04
    n = ds.n
    off, t, y = dev(torch, ds.offsets), dev(torch, ds.t), dev(torch, ds.y)
    f64 = torch.float64
    c = torch.empty(P, dtype=f64, device="cuda:0")
    s = torch.empty_like(c)
    sq = torch.empty_like(c)
    F.fpca_bin(h, grid, F.FPCA_BIN_MEAN, F.FPCA_IRREGULAR, F.FPCA_F64, F.FPCA_PREC_F64, n, off, t, y, None, 0,
               c, s, sq)
    mu = torch.empty_like(c)
    b0 = torch.empty_like(c)
    F.fpca_smooth_mean(h, grid, F.FPCA_F64, c, s, F.FPCA_K_EPANECHNIKOV, hs, mu)
    F.fpca_smooth_mean(h, grid, F.FPCA_F64, c, sq, F.FPCA_K_EPANECHNIKOV, hs, b0)
    C = torch.empty(P * P, dtype=f64, device="cuda:0")
    G = torch.empty_like(C)
    F.fpca_bin(h, grid, F.FPCA_BIN_COV, F.FPCA_IRREGULAR, F.FPCA_F64, F.FPCA_PREC_F64, n, off, t, y, None, 0,
               C, G)
    gam = torch.empty_like(C)
    F.fpca_smooth_cov(h, grid, F.FPCA_F64, C, 0.0, G, mu, F.FPCA_K_EPANECHNIKOV, hs, gam)
    s2t = torch.empty_like(c)
    s2, cnt = F.fpca_noise_variance(h, grid, F.FPCA_F64, b0, mu, gam, s2t)
    h.sync()
    rc, rs, _, _ = oracle.bin_mean(M, ds.offsets, ds.t, ds.y)
    _, rsq, _, _ = oracle.bin_mean(M, ds.offsets, ds.t, np.asarray(ds.y, np.float64) ** 2)
    rmu, _ = oracle.smooth_mean(M, hs, rc, rs)
    rb0, _ = oracle.smooth_mean(M, hs, rc, rsq)
    rC, rG = oracle.bin_cov_pairs(M, ds.offsets, ds.t, ds.y)
    gh, _ = oracle.smooth_cov_raw(M, hs, rC, rG)
    rgam = oracle.assemble_cov(gh.reshape(P, P), rmu)
    rt, rs2, rcnt = oracle.noise_variance(rb0, rmu, rgam)
    scale = np.abs(rb0).max()
    assert cnt == rcnt == P
    assert np.abs(s2t.cpu().numpy() - rt).max() < 1e-10 * scale
    assert abs(s2 - rs2) < 1e-10 * scale
    assert 0.5 * 0.01 < s2 < 3.0 * 0.01, s2  # generating noise sd 0.1

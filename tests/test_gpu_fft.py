"""GPU parity of the FFT moment passes (Section 3.2's FFT strategy on binned
data) against the FP64 oracle, which sums every window directly.

Bars: FP64 to 1e-10 normwise and FP32 inputs to 1e-5 over nodes OK on both
sides; statuses equal except where the oracle's smallest pivot is within a
factor 10 of the 1e-10 threshold or the oracle's window sum S0 is below
1e-9 of its largest value (the FFT pass sets sums below 1e-12 of the line's
scale to zero); empty windows stay EMPTY (exact zeros after the flush).
"""
import sys

import numpy as np
import pytest

import oracle
from tests._util import normwise_rel, status_agreement

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


def _mean_case(rng, M, gap=None):
    P = int(np.prod(M))
    w = rng.integers(0, 6, P).astype(np.float64) * (rng.random(P) < 0.7)
    x = np.stack(np.meshgrid(*[np.linspace(0, 1, m) for m in M], indexing="ij"), -1).reshape(P, -1)
    g = w * (np.sin(3 * x).sum(1) + 0.1 * rng.standard_normal(P))
    if gap is not None:
        sel = (x[:, 0] >= gap[0]) & (x[:, 0] <= gap[1])
        w[sel] = 0.0
        g[sel] = 0.0
    return w, g


def _check_mean(F, torch, h, M, hb, w, g, dt, mode):
    npdt = np.float64 if dt == "f64" else np.float32
    tdt = torch.float64 if dt == "f64" else torch.float32
    P = w.size
    mu = torch.empty(P, dtype=tdt, device="cuda:0")
    st = torch.empty(P, dtype=torch.int8, device="cuda:0")
    F.fpca_set_conv(h, mode)
    try:
        F.fpca_smooth_mean(h, F.Grid(M), F.FPCA_F64 if dt == "f64" else F.FPCA_F32,
                           dev(torch, w.astype(npdt)), dev(torch, g.astype(npdt)), F.FPCA_K_EPANECHNIKOV, hb, mu, st)
        h.sync()
    finally:
        F.fpca_set_conv(h, F.FPCA_CONV_DIRECT)
    w64 = w.astype(npdt).astype(np.float64)
    g64 = g.astype(npdt).astype(np.float64)
    rb, rst, rmom, rmp = oracle.smooth(M, hb, w64, g64, want_moments=True)
    stg, mug = host(st), host(mu)
    s0 = rmom[:, 0]
    tiny = s0 < 1e-9 * s0.max()
    bad, _ = status_agreement(stg[~tiny], rst[~tiny], rmp[~tiny])
    assert bad == 0
    # a window the oracle finds empty is empty on the GPU too
    assert np.all(stg[rst == 2] == 2)
    ok = (stg == 0) & (rst == 0)
    tol = 1e-10 if dt == "f64" else 1e-5
    assert normwise_rel(mug, rb, ok) < tol
    fb = (stg == 1) & (rst == 1)
    if fb.any():
        assert normwise_rel(mug, rb, fb) < tol
    return stg, rst


@pytest.mark.parametrize("M,hb,dt", [((1000,), 0.1, "f64"), ((1000,), 0.1, "f32"), ((3001,), 0.3, "f64"),
                                     ((200, 150), (0.2, 0.15), "f64"), ((97, 61), 0.35, "f32"),
                                     ((40, 33, 29), 0.4, "f64")])
def test_fft_mean_parity(torch, F, h, M, hb, dt):
    """Long windows (R up to 900 grid steps; L up to 4096) on one to three
    coordinates, FP64 and FP32 inputs."""
    _say(f"fft mean M={M} h={hb} {dt}")
    rng = np.random.default_rng(sum(M))
    w, g = _mean_case(rng, M)
    _check_mean(F, torch, h, M, hb, w, g, dt, F.FPCA_CONV_FFT)


def test_fft_keeps_empty_windows_empty(torch, F, h):
    """A gap of zero weight wider than the window: the nodes inside see exact
    zeros through the FFT (the flush) and are EMPTY, as in the direct sums."""
    _say("fft empty windows")
    M = (512,)
    hb = 20.5 / 511  # R = 20, edge tap 1 - (20/20.5)^2 ~ 0.05
    rng = np.random.default_rng(3)
    w, g = _mean_case(rng, M, gap=(100 / 511, 300 / 511))
    stg, rst = _check_mean(F, torch, h, M, hb, w, g, "f64", F.FPCA_CONV_FFT)
    assert (rst == 2).sum() > 100
    assert np.array_equal(stg == 2, rst == 2)


def test_fft_auto_matches_direct(torch, F, h):
    """AUTO times both methods per pass shape and keeps the faster; either
    way the result is the oracle's, and a second call (cached choice) agrees
    with the first."""
    _say("fft auto")
    M = (2000,)
    hb = 0.25
    rng = np.random.default_rng(5)
    w, g = _mean_case(rng, M)
    outs = []
    for _ in range(2):
        mu = torch.empty(w.size, dtype=torch.float64, device="cuda:0")
        F.fpca_set_conv(h, F.FPCA_CONV_AUTO)
        try:
            F.fpca_smooth_mean(h, F.Grid(M), F.FPCA_F64, dev(torch, w), dev(torch, g), F.FPCA_K_EPANECHNIKOV, hb, mu)
            h.sync()
        finally:
            F.fpca_set_conv(h, F.FPCA_CONV_DIRECT)
        outs.append(host(mu))
    rb, rst = oracle.smooth(M, hb, w, g)
    ok = rst == 0
    for o in outs:
        assert normwise_rel(o, rb, ok) < 1e-10
    assert normwise_rel(outs[0], outs[1], ok) < 1e-12


@pytest.mark.parametrize("M,hb", [((100,), 0.3), ((3, 70), (0.5, 0.3))])
def test_fft_cov_general_path(torch, F, h, M, hb):
    """The covariance on grids the task-queue smoother does not take runs the
    general pass engine: with FFT passes it matches the oracle."""
    _say(f"fft cov M={M} h={hb}")
    rng = np.random.default_rng(77 + len(M))
    P = int(np.prod(M))
    C = rng.random((P, P)) + 0.01
    C = (C + C.T) * 0.5
    G = C * rng.standard_normal((P, P))
    G = (G + G.T) * 0.5
    mu = rng.standard_normal(P)
    gam = torch.empty(P, P, dtype=torch.float64, device="cuda:0")
    st = torch.empty(P, P, dtype=torch.int8, device="cuda:0")
    F.fpca_set_conv(h, F.FPCA_CONV_FFT)
    try:
        F.fpca_smooth_cov(h, F.Grid(M), F.FPCA_F64, dev(torch, C), 0.0, dev(torch, G), dev(torch, mu),
                          F.FPCA_K_EPANECHNIKOV, hb, gam, st)
        h.sync()
    finally:
        F.fpca_set_conv(h, F.FPCA_CONV_DIRECT)
    rb, rst = oracle.smooth_cov_raw(M, hb, C, G)
    ref = oracle.assemble_cov(rb.reshape(P, P), mu)
    assert status_agreement(host(st), rst)[0] == 0
    okm = (rst.reshape(P, P) == 0) & (rst.reshape(P, P).T == 0)
    assert normwise_rel(host(gam), ref, okm) < 1e-10


def test_set_conv_rejects_bad_mode(F, h):
    with pytest.raises(F.FpcaError):
        F.fpca_set_conv(h, 7)

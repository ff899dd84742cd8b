"""GPU parity of the covariance operator (the smoothed covariance of complete
common-grid curves, never stored) and of the eigendecomposition taken through
it, against the oracle's stored covariance: common-grid pair sums, the
direct-window local-linear smoother of eq. 2.4 at every covariance node,
Gamma = b0 - mu mu^T symmetrized, then plain products and the randomized
eigendecomposition of Section 3.4.

Bars (FP64 on both sides): products 1e-10 normwise; the whole covariance
(columns by unit vectors) 1e-10 normwise; eigenvalues 1e-9 relative to the
largest; eigenfunctions 1e-7 normwise. Grids are ragged against the band tiles
(64; 8 x 8; 4 x 4 x 4) and the band covers part of the grid.
"""
import sys

import numpy as np
import pytest

import oracle
from tests._util import normwise_rel

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
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")


def host(x):
    return x.detach().cpu().numpy()


def _curves(rng, M, n):
    """Complete curves on the grid: a few smooth random surfaces plus noise."""
    P = int(np.prod(M))
    x = np.stack(np.meshgrid(*[np.linspace(0, 1, m) for m in M], indexing="ij"), -1).reshape(P, -1)
    basis = [np.ones(P)]
    for k in range(len(M)):
        basis += [np.sin(2 * np.pi * x[:, k]), np.cos(2 * np.pi * x[:, k]), x[:, k] ** 2]
    B = np.stack(basis, 1)
    A = rng.standard_normal((n, B.shape[1])) * np.linspace(1.0, 0.3, B.shape[1])
    return A @ B.T + 0.3 * rng.standard_normal((n, P))


def _oracle_gamma(M, hb, Y, mu):
    P = int(np.prod(M))
    _, _, C, G = oracle.bin_common_grid(Y)
    rb, rst = oracle.smooth_cov_raw(M, hb, C, G)
    return oracle.assemble_cov(rb.reshape(P, P), mu), rst


CASES = [((200,), 0.05), ((70,), 0.12), ((20, 18), 0.15), ((12, 10), (0.3, 0.35)), ((7, 6, 5), 0.4),
         ((9, 8, 6), (0.3, 0.3, 0.45))]


@pytest.mark.parametrize("M,hb", CASES)
@pytest.mark.parametrize("mode", [0, 1])
def test_covop_apply_parity(torch, F, h, M, hb, mode):
    _say(f"covop apply M={M} h={hb} mode={mode}")
    rng = np.random.default_rng(sum(M) + 7 * mode)
    P = int(np.prod(M))
    n = 37
    Y = _curves(rng, M, n)
    mu = Y.mean(0) + 0.05 * rng.standard_normal(P)
    gam, rst = _oracle_gamma(M, hb, Y, mu)
    op = F.CovOp(h, F.Grid(M), dev(torch, Y), dev(torch, mu), hb, mode)
    try:
        # a block of random vectors
        X = rng.standard_normal((P, 24))
        out = torch.empty(P, 24, dtype=torch.float64, device="cuda:0")
        op.apply(dev(torch, X), out)
        h.sync()
        assert normwise_rel(host(out), gam @ X) < 1e-10
        # the whole covariance, 64 unit vectors at a time
        cols = []
        for c0 in range(0, P, 64):
            w = min(64, P - c0)
            E = np.zeros((P, w))
            E[c0 + np.arange(w), np.arange(w)] = 1.0
            o = torch.empty(P, w, dtype=torch.float64, device="cuda:0")
            op.apply(dev(torch, E), o)
            cols.append(host(o))
        h.sync()
        full = np.concatenate(cols, 1)
        assert normwise_rel(full, gam) < 1e-10
        assert normwise_rel(full, full.T) < 1e-12
    finally:
        op.close()


def test_covop_sampled_columns_wide_band(torch, F, h):
    """d = 3 with windows of 4/4/3 grid steps (the band reaches most of the
    grid): three columns of the covariance against the oracle at those nodes."""
    M, hb = (10, 9, 8), 0.5
    _say(f"covop sampled columns M={M} h={hb}")
    rng = np.random.default_rng(5)
    P = int(np.prod(M))
    Y = _curves(rng, M, 20)
    mu = Y.mean(0)
    _, _, C, G = oracle.bin_common_grid(Y)
    cols = np.array([0, 377, P - 1])
    E = np.zeros((P, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    for mode in (0, 1):
        op = F.CovOp(h, F.Grid(M), dev(torch, Y), dev(torch, mu), hb, mode)
        try:
            out = torch.empty(P, len(cols), dtype=torch.float64, device="cuda:0")
            op.apply(dev(torch, E), out)
            h.sync()
            got = host(out)
        finally:
            op.close()
        for j, q in enumerate(cols):
            p = np.arange(P)
            nodes = np.concatenate([p * P + q, q * P + p])
            rb, _ = oracle.smooth_cov_raw(M, hb, C, G, nodes)
            ref = 0.5 * (rb[:P] + rb[P:]) - mu * mu[q]
            assert normwise_rel(got[:, j], ref) < 1e-10


def test_covop_widest_d3_window(torch, F, h):
    """d = 3 at the largest window the operator takes (6 grid steps in every
    coordinate: shared-node boxes of 16 nodes per coordinate, the tile-pair
    limit): one column of the covariance against the oracle."""
    M, hb = (13, 13, 13), 0.5
    _say(f"covop widest window M={M} h={hb}")
    rng = np.random.default_rng(8)
    P = int(np.prod(M))
    Y = _curves(rng, M, 12)
    mu = Y.mean(0)
    _, _, C, G = oracle.bin_common_grid(Y)
    q = P // 2 + 7
    E = np.zeros((P, 1))
    E[q, 0] = 1.0
    op = F.CovOp(h, F.Grid(M), dev(torch, Y), dev(torch, mu), hb, 0)
    try:
        out = torch.empty(P, 1, dtype=torch.float64, device="cuda:0")
        op.apply(dev(torch, E), out)
        h.sync()
        got = host(out)[:, 0]
    finally:
        op.close()
    p = np.arange(P)
    rb, _ = oracle.smooth_cov_raw(M, hb, C, G, np.concatenate([p * P + q, q * P + p]))
    ref = 0.5 * (rb[:P] + rb[P:]) - mu * mu[q]
    assert normwise_rel(got, ref) < 1e-10


@pytest.mark.parametrize("M,hb", [((70,), 0.12), ((20, 18), 0.15), ((9, 8, 6), (0.3, 0.3, 0.45))])
def test_covop_eig_matches_oracle(torch, F, h, M, hb):
    """fpca_eig_covop against the oracle's randomized eigendecomposition of the
    stored covariance (same test matrix, FP64), and against fpca_eig_randomized
    on the stored covariance."""
    _say(f"covop eig M={M} h={hb}")
    rng = np.random.default_rng(11 + len(M))
    P = int(np.prod(M))
    Y = _curves(rng, M, 40)
    mu = Y.mean(0)
    gam, _ = _oracle_gamma(M, hb, Y, mu)
    k, p_over, q = 5, 10, 2
    omega = oracle.quad_weights(M)
    ev_ref, phi_ref, fve_ref = oracle.eig_randomized(gam, omega, k, p_over, q, 7)
    op = F.CovOp(h, F.Grid(M), dev(torch, Y), dev(torch, mu), hb, 0)
    try:
        ef = torch.empty(k, P, dtype=torch.float64, device="cuda:0")
        ev, fve = op.eig(None, k, p_over, q, 7, ef)
        h.sync()
    finally:
        op.close()
    assert np.abs(ev - ev_ref).max() < 1e-9 * abs(ev_ref[0])
    assert np.abs(fve - fve_ref).max() < 1e-9
    phi = host(ef)
    for l in range(k):
        assert normwise_rel(phi[l], phi_ref[:, l]) < 1e-7, l
    ef2 = torch.empty(k, P, dtype=torch.float64, device="cuda:0")
    ev2, _ = F.fpca_eig_randomized(h, F.FPCA_F64, F.FPCA_PREC_F64, F.Grid(M), dev(torch, gam), None, k, p_over, q, 7,
                                   ef2)
    h.sync()
    assert np.abs(ev - ev2).max() < 1e-9 * abs(ev2[0])


def test_covop_rejects_unsupported(torch, F, h):
    P = 64
    Y = dev(torch, np.ones((3, P)))
    mu = dev(torch, np.zeros(P))
    with pytest.raises(F.FpcaError):  # a window narrower than one grid step
        F.CovOp(h, F.Grid((64,)), Y, mu, 0.001)
    Y3 = dev(torch, np.ones((3, 1000)))
    mu3 = dev(torch, np.zeros(1000))
    with pytest.raises(F.FpcaError):  # d = 3 windows beyond 6 grid steps (here 8)
        F.CovOp(h, F.Grid((10, 10, 10)), Y3, mu3, 0.9)
    m = torch.ones(P, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(F.FpcaError):  # domain masks are not taken
        F.CovOp(h, F.Grid((64,), mask=m), Y, mu, 0.2)

"""Whole-path parity on the d=2 irregular FP32 workload (reduced to n = 120
curves so that the oracle's pair loops and direct-window smoother over all
32^4 nodes finish in seconds), plus the masked d=3 workload's binning and
smoothing of the mean on 16^3 against the oracle."""
import numpy as np
import pytest

import oracle
from fpca_synth import make_c2, make_c4
from tests._util import normwise_rel, status_agreement

pytestmark = pytest.mark.gpu


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


def test_end_to_end_d2_irregular(torch, F, h):
    print("end-to-end d=2 irregular, n=120", flush=True)
    from paper_1510_04439_amd import pipeline as PL
    ds = make_c2(n=120)
    dd = PL.to_device(ds)
    bufs = PL.alloc(dd, ds.k)
    PL.fit(h, dd, bufs, ds.h_mean, ds.h_cov, ds.k, ds.oversample, ds.power_iters, ds.rp_seed)
    h.sync()
    t64, y64 = ds.t.astype(np.float64), ds.y.astype(np.float64)
    c, s, _, _ = oracle.bin_mean(ds.M_mean, ds.offsets, t64, y64)
    mu, mst = oracle.smooth_mean(ds.M_mean, ds.h_mean, c, s)
    assert normwise_rel(bufs.mu.cpu().numpy(), mu, mst == 0) < 1e-5
    C, G = oracle.bin_cov_pairs(ds.M_cov, ds.offsets, t64, y64)
    assert normwise_rel(bufs.C.cpu().numpy(), C) < 1e-5
    assert normwise_rel(bufs.G.cpu().numpy(), G) < 1e-5
    P = 1024
    gh, gst = oracle.smooth_cov_raw(ds.M_cov, ds.h_cov, C, G)
    gam = oracle.assemble_cov(gh.reshape(P, P), mu)
    st = gst.reshape(P, P)
    ok = (st == 0) & (st.T == 0)
    assert status_agreement(bufs.status.cpu().numpy(), gst)[0] == 0
    assert normwise_rel(bufs.gamma.cpu().numpy(), gam, ok) < 1e-5
    om = oracle.quad_weights(ds.M_cov)
    ev, phi, fve = oracle.eig_randomized(np.nan_to_num(gam), om, ds.k, ds.oversample, ds.power_iters,
                                         ds.rp_seed)
    assert np.abs(bufs.evals[:6] - ev[:6]).max() <= 1e-4 * ev[0]
    # eigenfunctions of the whole chain, with a tolerance that grows as the
    # neighbouring eigenvalues close in (a perturbation of the surface by e
    # turns an eigenvector by about e / gap)
    phi_gpu = bufs.efuns.cpu().numpy()
    for j in range(6):
        gap = min(abs(ev[j] - ev[j - 1]) if j else np.inf, abs(ev[j] - ev[j + 1]))
        scale = max(1.0, 0.1 * ev[0] / gap)
        err = min(np.abs(phi_gpu[j] - phi[:, j]).max(), np.abs(phi_gpu[j] + phi[:, j]).max())
        assert err <= 1e-2 * scale * np.abs(phi[:, j]).max(), (j, err, scale)
    # the eigendecomposition alone: the oracle's randomized eig of the GPU's own surface
    gam_gpu = bufs.gamma.cpu().numpy().astype(np.float64)
    ev2, phi2, fve2 = oracle.eig_randomized(np.nan_to_num(gam_gpu), om, ds.k, ds.oversample, ds.power_iters,
                                            ds.rp_seed)
    assert np.abs(bufs.evals - ev2).max() <= 1e-5 * ev2[0]
    for j in range(ds.k):
        gap = min(abs(ev2[j] - ev2[j - 1]) if j else np.inf, abs(ev2[j] - ev2[j + 1]) if j + 1 < ds.k else np.inf)
        scale = max(1.0, 0.1 * ev2[0] / gap)
        err = min(np.abs(phi_gpu[j] - phi2[:, j]).max(), np.abs(phi_gpu[j] + phi2[:, j]).max())
        assert err <= 1e-3 * scale * np.abs(phi2[:, j]).max(), (j, err, scale)


def test_d3_masked_mean(torch, F, h):
    """d=3 disk x time domain: binning and mean smoothing on 16^3 nodes."""
    print("d=3 masked mean", flush=True)
    ds = make_c4(n=60)
    M = ds.M_mean
    P = int(np.prod(M))
    off = torch.from_numpy(ds.offsets).cuda()
    t = torch.from_numpy(ds.t).cuda()
    y = torch.from_numpy(ds.y).cuda()
    c = torch.empty(P, dtype=torch.float32, device="cuda:0")
    s = torch.empty_like(c)
    idx = torch.empty(len(ds.y), dtype=torch.int32, device="cuda:0")
    cnt = torch.empty(P, dtype=torch.int64, device="cuda:0")
    F.fpca_bin(h, F.Grid(M), F.FPCA_BIN_MEAN, F.FPCA_IRREGULAR, F.FPCA_F32, F.FPCA_PREC_F32, ds.n, off, t, y,
               None, 0, c, s, None, idx, cnt)
    mu = torch.empty_like(c)
    st = torch.empty(P, dtype=torch.int8, device="cuda:0")
    F.fpca_smooth_mean(h, F.Grid(M), F.FPCA_F32, c, s, F.FPCA_K_EPANECHNIKOV, ds.h_mean, mu, st)
    h.sync()
    rc, rs, ridx, rcnt = oracle.bin_mean(M, ds.offsets, ds.t.astype(np.float64), ds.y.astype(np.float64))
    assert np.array_equal(idx.cpu().numpy(), ridx) and np.array_equal(cnt.cpu().numpy(), rcnt)
    rb, rst = oracle.smooth_mean(M, ds.h_mean, rc.astype(np.float32).astype(np.float64),
                                 rs.astype(np.float32).astype(np.float64))
    assert normwise_rel(c.cpu().numpy(), rc) < 1e-5
    # the smoother alone, on the oracle's binned arrays rounded to FP32
    c2 = torch.from_numpy(rc.astype(np.float32)).cuda()
    s2 = torch.from_numpy(rs.astype(np.float32)).cuda()
    F.fpca_smooth_mean(h, F.Grid(M), F.FPCA_F32, c2, s2, F.FPCA_K_EPANECHNIKOV, ds.h_mean, mu, st)
    h.sync()
    ok = (st.cpu().numpy() == 0) & (rst == 0)
    assert normwise_rel(mu.cpu().numpy(), rb, ok) < 1e-5

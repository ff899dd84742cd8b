"""Streams restricted to a range of compute units (fpca_stream_create_cu_range):
the library's kernels give the same bits on such a stream as on an
unrestricted one (the benchmark runs the eigendecomposition on the top
quarter of the chip beside the next step's binning and smoothing), and bad
ranges are refused."""
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


def _run(torch, F, h, stream, M, Gm, mu, hb):
    P = int(np.prod(M))
    with torch.cuda.stream(stream):
        G = torch.from_numpy(Gm).to("cuda:0")
        m = torch.from_numpy(mu).to("cuda:0")
        gam = torch.empty(P, P, dtype=torch.float32, device="cuda:0")
        st = torch.empty(P, P, dtype=torch.int8, device="cuda:0")
        F.fpca_smooth_cov(h, F.Grid(M), F.FPCA_F32, None, 0.02, G, m, F.FPCA_K_EPANECHNIKOV, hb, gam, st)
        ef = torch.empty(5, P, dtype=torch.float32, device="cuda:0")
        ev, fve = F.fpca_eig_randomized(h, F.FPCA_F32, F.FPCA_PREC_F32, F.Grid(M), gam, None, 5, 10, 2, 3, ef)
        h.sync()
        return gam.cpu().numpy(), st.cpu().numpy(), ev, fve, ef.cpu().numpy()


def test_cu_range_stream_gives_the_same_bits(torch, F):
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    q = max(32, (ncu // 4) // 32 * 32)
    _say(f"cu-range streams on {ncu} CUs: [0, {ncu - q}) and [{ncu - q}, {ncu})")
    rng = np.random.default_rng(4)
    M, hb = (12, 12), 0.2  # the fused common-grid smoother (R = 2 on both coordinates)
    P = int(np.prod(M))
    A = rng.standard_normal((60, P))
    Gm = ((A.T @ A) / 60).astype(np.float32)
    mu = (0.1 * rng.standard_normal(P)).astype(np.float32)
    h = F.Handle(0)
    raw = []
    try:
        ref = _run(torch, F, h, torch.cuda.Stream(), M, Gm, mu, hb)
        for lo, hi in ((0, ncu - q), (ncu - q, ncu)):
            raw.append(F.fpca_stream_create_cu_range(0, lo, hi))
            got = _run(torch, F, h, torch.cuda.ExternalStream(raw[-1]), M, Gm, mu, hb)
            for a, b in zip(got, ref):
                assert np.array_equal(np.asarray(a), np.asarray(b))
    finally:
        torch.cuda.synchronize()
        for r in raw:
            F.fpca_stream_destroy(r)
        h.close()
    # and the smoother output is the oracle's (FP32 bar)
    rb, rst = oracle.smooth_cov_raw(M, hb, np.full((P, P), 0.02) * (1 - np.eye(P)), Gm.astype(np.float64))
    gam = oracle.assemble_cov(rb.reshape(P, P), mu.astype(np.float64))
    ok = (rst.reshape(P, P) == 0) & (rst.reshape(P, P).T == 0)
    err = np.linalg.norm((ref[0] - gam)[ok]) / np.linalg.norm(gam[ok])
    assert err < 1e-5


def test_cu_range_rejects_bad_ranges(torch, F):
    _say("cu-range stream argument errors")
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    for dev, lo, hi in ((0, 0, 0), (0, -1, 8), (0, 8, 4), (0, 0, ncu + 1), (99, 0, 8)):
        with pytest.raises(F.FpcaError):
            F.fpca_stream_create_cu_range(dev, lo, hi)

"""GPU parity of the paper's bandwidth search (Section 3.3): the binned
leave-one-out criterion (fpca_cv_loo) against the oracle's, and the
trust-region search (fpca_bw_search) against the oracle's search driven by
the oracle's criterion: the same samples in the same order, the same
selected bandwidth."""
import sys

import numpy as np
import pytest

import oracle
from oracle import bw_search as OB
from fpca_synth import disk_time_mask
from tests._util import rand_irregular

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


def _data(rng, M, n, npdt, nlo=2, nhi=12, smooth=False):
    d = len(M)
    off, t, y = rand_irregular(rng, d, n, nlo, nhi, npdt)
    if smooth:
        # curves sum_k xi_ik prod_c cos(pi k_c t_c) with decaying variances, plus noise:
        # a smooth covariance, so the criterion has an interior minimum in h
        ks = [(1,) * d, (2,) + (1,) * (d - 1), (1,) * (d - 1) + (3,)]
        ci = np.repeat(np.arange(n), np.diff(off))
        xi = rng.standard_normal((n, len(ks))) * np.array([1.0, 0.6, 0.4])
        tt = t.astype(np.float64)
        y = np.zeros(len(tt))
        for j, kv in enumerate(ks):
            y += xi[ci, j] * np.prod([np.cos(np.pi * kv[c] * tt[:, c]) for c in range(d)], axis=0)
        y = (y + 0.3 * rng.standard_normal(len(tt))).astype(npdt)
    C, G, Q = oracle.bin_cov_pairs(M, off, t.astype(np.float64), y.astype(np.float64), want_Q=True)
    return [a.astype(npdt) for a in (C, G, Q)]


@pytest.mark.parametrize("M,dt,masked", [((21,), "f64", False), ((9, 8), "f32", False), ((9, 9), "f32", True),
                                         ((4, 5, 4), "f32", False), ((5, 5, 4), "f64", True)])
def test_cv_loo_parity(torch, F, h, M, dt, masked):
    _say(f"cv_loo M={M} {dt} masked={masked}")
    rng = np.random.default_rng(1200 + sum(M))
    npdt = np.float64 if dt == "f64" else np.float32
    C, G, Q = _data(rng, M, 40, npdt)
    d = len(M)
    mask = None
    if masked:
        if d == 3:
            mask = disk_time_mask(M)
        else:
            x = np.arange(M[0]) / (M[0] - 1)
            yv = np.arange(M[1]) / (M[1] - 1)
            X, Y = np.meshgrid(x, yv, indexing="ij")
            mask = (((X - .5) ** 2 + (Y - .5) ** 2) <= .25 + 1e-12).astype(np.uint8).reshape(-1)
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    hs = np.stack([np.geomspace(0.12, 0.6, 5)] * d, axis=1) * np.linspace(1.0, 0.9, d)
    g = F.Grid(M, None if mask is None else D(mask))
    got = F.fpca_cv_loo(h, g, F.FPCA_F64 if dt == "f64" else F.FPCA_F32, D(C), D(G), D(Q), hs)
    ref = np.array([OB.loo_cv_score(M, hr, C, G, Q, mask) for hr in hs])
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=0)


@pytest.mark.parametrize("M,dt", [((25,), "f64"), ((13, 12), "f32"), ((6, 6, 5), "f32")])
def test_bw_search_follows_oracle(torch, F, h, M, dt):
    _say(f"bw_search M={M} {dt}")
    rng = np.random.default_rng(1300 + sum(M))
    npdt = np.float64 if dt == "f64" else np.float32
    # dense enough (and bandwidths wide enough, at least 1.5 grid steps) that
    # every reduced window is well conditioned: the two criteria then agree to
    # rounding and the searches take the same decisions
    C, G, Q = _data(rng, M, 300, npdt, 6, 16, smooth=True)
    d = len(M)
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    lo, hi, h0 = [1.5 / (M[0] - 1)] * d, [0.9] * d, [0.4] * d
    hg, vg, ng, trace = F.fpca_bw_search(h, F.Grid(M), F.FPCA_F64 if dt == "f64" else F.FPCA_F32, D(C), D(G),
                                         D(Q), lo, hi, h0, max_evals=40)
    fb = lambda hs: [OB.loo_cv_score(M, hv, C, G, Q) for hv in hs]
    hr, vr, nr, tr = OB.trust_region_search(fb, d, lo, hi, h0, max_evals=40)
    _say(f"  gpu h={hg} cv={vg:.9e} n={ng}; oracle h={hr} cv={vr:.9e} n={nr}")
    assert ng == nr
    for (hq, vq), row in zip(tr, trace):
        np.testing.assert_allclose(row[:d], hq, rtol=1e-6)
        np.testing.assert_allclose(row[d], vq, rtol=1e-8)
    np.testing.assert_allclose(hg, hr, rtol=1e-6)
    assert abs(vg - vr) <= 1e-8 * abs(vr)
    # the selected criterion is the smallest sampled one
    assert vg == trace[:, d].min()

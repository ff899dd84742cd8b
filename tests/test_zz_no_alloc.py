"""fpca_pace_scores_noalloc (for callers that cannot allocate) against
fpca_pace_scores on the same inputs, through the C ABI: two calls in a row,
the second on a smaller input, on the common-grid design (the one whose
kernels use scratch memory) with missing values, and on the irregular design.
A handle whose scratch limit is one byte shows that the variant allocates
nothing: the allocating entry point is refused there, the variant is not.
Same kernels on the same inputs, so the two outputs are bitwise equal."""
import os
import sys

import numpy as np
import pytest

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


def _case(rng, M, n, k, missing):
    P = int(np.prod(M))
    efuns = np.linalg.qr(rng.standard_normal((P, k)))[0] * np.sqrt(P)
    lam = np.sort(rng.uniform(0.2, 2.0, k))[::-1].copy()
    lam[-1] = -0.1 if k > 2 else lam[-1]  # a non-positive eigenvalue is left out
    mu = rng.standard_normal(P)
    xi = rng.standard_normal((n, k)) * np.sqrt(np.abs(lam))
    y = mu + xi @ efuns.T + 0.3 * rng.standard_normal((n, P))
    if missing:
        y[rng.random((n, P)) < 0.1] = np.nan
        y[0] = y[0] if n < 2 else np.where(np.isnan(y[0]), 0.0, y[0])  # one complete curve
    return efuns, lam, mu, y


def _both(torch, F, h, M, efuns, lam, mu, y, s2, dt):
    n, k = y.shape[0], efuns.shape[1]
    npdt = np.float64 if dt == F.FPCA_F64 else np.float32
    tdt = torch.float64 if dt == F.FPCA_F64 else torch.float32
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a, npdt)).to("cuda:0")
    yy, mm, ef = D(y), D(mu), D(efuns.T)
    outs = []
    for fn in (F.fpca_pace_scores, F.fpca_pace_scores_noalloc):
        o = torch.full((n * k,), 7.0, dtype=tdt, device="cuda:0")
        fn(h, F.Grid(M), F.FPCA_COMMON_GRID, dt, n, None, None, yy, mm, ef, k, lam, s2, o)
        h.sync()
        outs.append(o.cpu().numpy())
    return outs


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_matches_pace_scores_common_grid(torch, F, dt):
    rng = np.random.default_rng(77)
    dtc = F.FPCA_F64 if dt == "f64" else F.FPCA_F32
    h = F.Handle(0)
    try:
        for (M, n, k) in (((12, 10), 40, 7), ((6, 5), 9, 3)):
            _say(f"noalloc common grid {dt} M={M} n={n} k={k}")
            efuns, lam, mu, y = _case(rng, M, n, k, missing=True)
            ref, got = _both(torch, F, h, M, efuns, lam, mu, y, 0.09, dtc)
            assert np.all(np.isfinite(ref))
            assert np.array_equal(ref, got)
    finally:
        h.close()


def test_noalloc_irregular_and_no_scratch(torch, F):
    rng = np.random.default_rng(78)
    M = (9, 8)
    P = int(np.prod(M))
    k = 4
    efuns, lam, mu, y = _case(rng, M, 20, k, missing=False)
    os.environ["FPCA_DEBUG_WS_LIMIT"] = "1"
    try:
        h1 = F.Handle(0)
    finally:
        del os.environ["FPCA_DEBUG_WS_LIMIT"]
    h2 = F.Handle(0)
    try:
        _say("noalloc on a handle with a one-byte scratch limit")
        D = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to("cuda:0")
        yy, mm, ef = D(y), D(mu), D(efuns.T)
        o1 = torch.empty(20 * k, dtype=torch.float64, device="cuda:0")
        with pytest.raises(F.FpcaError) as ei:
            F.fpca_pace_scores(h1, F.Grid(M), F.FPCA_COMMON_GRID, F.FPCA_F64, 20, None, None, yy, mm, ef, k, lam,
                               0.09, o1)
        assert ei.value.code == F.FPCA_ERR_WORKSPACE
        F.fpca_pace_scores_noalloc(h1, F.Grid(M), F.FPCA_COMMON_GRID, F.FPCA_F64, 20, None, None, yy, mm, ef, k,
                                   lam, 0.09, o1)
        h1.sync()
        o2 = torch.empty_like(o1)
        F.fpca_pace_scores(h2, F.Grid(M), F.FPCA_COMMON_GRID, F.FPCA_F64, 20, None, None, yy, mm, ef, k, lam,
                           0.09, o2)
        h2.sync()
        assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
        _say("noalloc irregular design")
        g = np.stack(np.meshgrid(*[np.arange(m) / (m - 1) for m in M], indexing="ij"), -1).reshape(P, 2)
        off = np.arange(0, 20 * 30 + 1, 30, dtype=np.int64)
        idx = rng.integers(0, P, 20 * 30)
        t = g[idx] + rng.uniform(-0.02, 0.02, (20 * 30, 2))
        t = np.clip(t, 0.0, 1.0)
        yi = rng.standard_normal(20 * 30)
        outs = []
        for fn in (F.fpca_pace_scores, F.fpca_pace_scores_noalloc):
            o = torch.empty(20 * k, dtype=torch.float64, device="cuda:0")
            fn(h2, F.Grid(M), F.FPCA_IRREGULAR, F.FPCA_F64, 20, D(off.astype(np.float64)).to(torch.int64), D(t),
               D(yi), mm, ef, k, lam, 0.09, o)
            h2.sync()
            outs.append(o.cpu().numpy())
        assert np.all(np.isfinite(outs[0]))
        assert np.array_equal(outs[0], outs[1])
    finally:
        h1.close()
        h2.close()

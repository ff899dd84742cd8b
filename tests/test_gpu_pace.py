"""GPU parity of the PACE scores (eqs. 2.6, 2.7) against the oracle.

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
def test_pace_common_grid(torch, F, h, dt):
    _say(f"pace common grid {dt}")
    rng = np.random.default_rng(77)
    M = (8, 9)
    P = 72
    n, k = 30, 12
    Y = rng.standard_normal((n, P))
    Y[rng.random((n, P)) < 0.25] = np.nan
    Y[7] = np.nan
    mu = rng.standard_normal(P)
    efuns = rng.standard_normal((P, k)) / np.sqrt(P)
    lam = np.linspace(2.0, 0.05, k)
    got, ref = _run(torch, F, h, M, F.FPCA_COMMON_GRID, None, None, Y, mu, efuns, lam, 0.2, dt)
    assert np.all(got[7] == 0)
    tol = 1e-10 if dt == "f64" else 1e-5
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

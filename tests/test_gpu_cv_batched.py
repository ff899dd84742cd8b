"""Batched CV over several datasets of uneven size in one call (one persistent
launch of the task-queue smoother), against the oracle job by job: for each
dataset, bandwidth and fold, the direct-window smooth of the other folds'
pairs, symmetrized (and masked), scored by sum [Q_f - 2 G_f Ghat + C_f Ghat^2].
Datasets differ in curve count and grid size; d = 1, 2, 3; FP32 and FP64
storage. Also the engine's selected bandwidth (fpca_cv_select) against the
oracle's scores, and a call whose jobs outnumber the intermediate slots
several times (the slots are reused)."""
import sys

import numpy as np
import pytest

import oracle
from fpca_synth import disk_time_mask, fold_assignment
from tests._util import rand_irregular, engine

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


def _dataset(rng, M, n, nf, npdt, seed):
    d = len(M)
    off, t, y = rand_irregular(rng, d, n, 1, 14, npdt)
    folds = fold_assignment(n, nf, seed=seed)
    t64, y64 = t.astype(np.float64), y.astype(np.float64)
    slabs = [oracle.bin_cov_pairs(M, off, t64, y64, folds, fs, want_Q=True) for fs in [-1] + list(range(nf))]
    return [np.stack([s[i] for s in slabs]).astype(npdt) for i in range(3)]


def _ref_scores(M, hs, nf, C, G, Q, mask=None):
    P = int(np.prod(M))
    C, G, Q = (a.astype(np.float64) for a in (C, G, Q))
    ref = np.zeros((len(hs), nf))
    for i, hb in enumerate(hs):
        for f in range(nf):
            b, _ = oracle.smooth_cov_raw(M, hb, C[0] - C[f + 1], G[0] - G[f + 1])
            Ghat = oracle.assemble_cov(b.reshape(P, P), np.zeros(P), mask)
            ref[i, f] = oracle.cv_score(Q[f + 1], G[f + 1], C[f + 1], Ghat)
    return ref


@pytest.mark.parametrize("dt,grids,ns,hs,nf", [
    ("f32", [(7, 6), (9, 8), (5, 5)], [30, 14, 40], [0.2, 0.35, 0.6], 3),
    ("f64", [(4, 5, 4), (3, 4, 5)], [24, 11], [0.3, 0.55], 4),
    ("f32", [(40,), (23,)], [20, 35], [0.05, 0.12, 0.3], 5),
])
@pytest.mark.parametrize("eng", ["queue", "passes"])
def test_cv_batched_uneven_datasets(torch, F, h, dt, grids, ns, hs, nf, eng):
    with engine(F, h, F.FPCA_ENGINE_QUEUE if eng == "queue" else F.FPCA_ENGINE_PASSES):
        _cv_uneven(torch, F, h, dt, grids, ns, hs, nf, eng)


def _cv_uneven(torch, F, h, dt, grids, ns, hs, nf, eng):
    _say(f"cv uneven datasets {dt} grids={grids} n={ns} h={hs} folds={nf} engine={eng}")
    rng = np.random.default_rng(900 + len(grids[0]))
    npdt = np.float64 if dt == "f64" else np.float32
    data, host = [], []
    for a, (M, n) in enumerate(zip(grids, ns)):
        C, G, Q = _dataset(rng, M, n, nf, npdt, seed=9 + a)
        host.append((M, C, G, Q))
        D = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
        data.append((F.Grid(M), D(C), D(G), D(Q)))
    dtc = F.FPCA_F64 if dt == "f64" else F.FPCA_F32
    scores = F.fpca_cv_batched(h, dtc, data, nf, hs)
    assert scores.shape == (len(grids), len(hs), nf)
    for a, (M, C, G, Q) in enumerate(host):
        ref = _ref_scores(M, hs, nf, C, G, Q)
        np.testing.assert_allclose(scores[a], ref, rtol=1e-9 if dt == "f64" else 1e-5)
    # the same call again is captured into a graph, then replayed: same bits
    for _ in range(2):
        again = F.fpca_cv_batched(h, dtc, data, nf, hs)
        assert np.array_equal(again, scores)


def test_cv_batched_masked_d3_many_jobs_and_select(torch, F, h):
    """d = 3 disk x time mask, 6 bandwidths x 5 folds = 30 jobs over 3
    intermediate slots; the refined bandwidth from the GPU scores equals the
    one from the oracle's scores."""
    M = (5, 5, 4)
    nf = 5
    hs = np.geomspace(0.25, 0.7, 6)
    rng = np.random.default_rng(950)
    mask = disk_time_mask(M)
    C, G, Q = _dataset(rng, M, 30, nf, np.float32, seed=4)
    D = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    _say(f"cv masked d=3 M={M} jobs={len(hs) * nf}")
    with engine(F, h, F.FPCA_ENGINE_QUEUE):  # slot reuse across jobs is the queue kernel's
        scores = F.fpca_cv_batched(h, F.FPCA_F32, [(F.Grid(M, D(mask)), D(C), D(G), D(Q))], nf, hs)[0]
    ref = _ref_scores(M, hs, nf, C, G, Q, mask)
    np.testing.assert_allclose(scores, ref, rtol=1e-5)
    h_gpu = F.fpca_cv_select(hs, scores.sum(1))[0]
    h_ref = F.fpca_cv_select(hs, ref.sum(1))[0]
    assert abs(h_gpu - h_ref) <= 1e-4 * h_ref

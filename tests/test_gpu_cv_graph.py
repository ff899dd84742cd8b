"""Batched CV through its captured graph: the first call per shape runs
eagerly, the second captures, later calls replay. Every replay (with other
inputs and eager work in between) must reproduce an eager run bit for bit --
the CV kernels use no atomics and fixed reduction orders."""
import numpy as np
import pytest

import oracle
from fpca_synth import fold_assignment
from tests._util import rand_irregular

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


def _slabs(torch, seed, M, nf):
    rng = np.random.default_rng(seed)
    n = 24
    off, t, y = rand_irregular(rng, len(M), n, 2, 12, np.float32)
    folds = fold_assignment(n, nf, seed=seed)
    t64, y64 = t.astype(np.float64), y.astype(np.float64)
    sl = [oracle.bin_cov_pairs(M, off, t64, y64, folds, fs, want_Q=True) for fs in [-1] + list(range(nf))]
    return [torch.from_numpy(np.stack([s[i] for s in sl]).astype(np.float32)).cuda() for i in range(3)]


@pytest.mark.parametrize("M,hs", [((9, 8), [0.2, 0.3, 0.45]), ((4, 4, 5), [0.35, 0.6])])
def test_cv_graph_replays_match_eager(torch, F, M, hs):
    print(f"cv graph M={M}", flush=True)
    nf = 3
    A = _slabs(torch, 1, M, nf)
    Bs = _slabs(torch, 2, M, nf)
    g = F.Grid(M)
    # eager references from fresh handles (first call per handle is eager)
    refs = {}
    for name, X in (("A", A), ("B", Bs)):
        he = F.Handle(0)
        F.fpca_set_engine(he, F.FPCA_ENGINE_QUEUE)  # graphs are the queue kernel's
        refs[name] = F.fpca_cv_batched(he, F.FPCA_F32, [(g, *X)], nf, hs)[0]
        he.close()
    h = F.Handle(0)
    F.fpca_set_engine(h, F.FPCA_ENGINE_QUEUE)
    seq = ["A", "B", "A", "B", "B", "A"]  # eager, capture, replays
    for i, name in enumerate(seq):
        X = A if name == "A" else Bs
        got = F.fpca_cv_batched(h, F.FPCA_F32, [(g, *X)], nf, hs)[0]
        assert np.array_equal(got, refs[name]), (i, name, got, refs[name])
        # unrelated eager work on the same stream between replays
        tmp = torch.empty(int(np.prod(M)), dtype=torch.float32, device="cuda:0")
        F.fpca_smooth_mean(h, F.Grid(M), F.FPCA_F32, X[0][0, 0].contiguous(), X[1][0, 0].contiguous(),
                           F.FPCA_K_EPANECHNIKOV, hs[0], tmp)
        torch.cuda.synchronize()
    h.close()

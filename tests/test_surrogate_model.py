"""The committed bandwidth-surrogate model: loadable without pickle, the
parameter count of the 32-128-128-1 network, finite parameters, and a
finite prediction inside the labelled bandwidth range (up to one unit of
log h) for the features of a small held-out dataset of the training family
(FP64 features and forward pass of the reference network)."""
import numpy as np

import oracle
from oracle import mlp as ref
from fpca_synth import make_surrogate_dataset
from paper_1510_04439_amd.surrogate import H_GRID, MODEL_PATH


def test_model_file():
    z = np.load(MODEL_PATH, allow_pickle=False)
    assert z["params"].shape == (ref.NPARAM,)
    assert np.all(np.isfinite(z["params"]))
    assert z["feat_mean"].shape == (ref.NF,) and z["feat_sd"].shape == (ref.NF,)
    assert np.all(z["feat_sd"] > 0)
    assert H_GRID[0] <= float(z["h_lo"]) < float(z["h_hi"]) <= H_GRID[-1]


def test_model_prediction_in_range():
    z = np.load(MODEL_PATH, allow_pickle=False)
    ds = make_surrogate_dataset(304, "test")  # n = 310 curves, about 1M pairs
    M = ds.M_cov
    t64, y64 = ds.t.astype(np.float64), ds.y.astype(np.float64)
    c, s, _, _ = oracle.bin_mean(M, ds.offsets, t64, y64)
    _, s2, _, _ = oracle.bin_mean(M, ds.offsets, t64, y64 ** 2)
    C, G, Q = oracle.bin_cov_pairs(M, ds.offsets, t64, y64, want_Q=True)
    f = ref.features(M, ds.offsets, c, s, s2, C, G, Q)
    X = ((f - z["feat_mean"]) / z["feat_sd"])[None, :]
    out, _ = ref.forward(z["params"].astype(np.float64), X)
    lh = float(out[0])
    assert np.isfinite(lh)
    assert np.log(H_GRID[0]) - 1.0 <= lh <= np.log(H_GRID[-1]) + 1.0

"""Helpers shared by the test modules (no method arithmetic here)."""
import contextlib

import numpy as np


def normwise_rel(x, ref, mask=None):
    """||x - ref||_inf / ||ref||_inf over the selected entries."""
    x = np.asarray(x, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    if mask is not None:
        m = np.asarray(mask).reshape(-1).astype(bool)
        x, ref = x[m], ref[m]
    if ref.size == 0:
        return 0.0
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


def status_agreement(st_gpu, st_ref, minpiv_ref=None):
    """Statuses must agree except where the oracle's smallest pivot lies within
    a factor 10 of the 1e-10 threshold (the decision is taken from FP32 moments
    on the GPU and FP64 moments in the oracle). Returns (n_disagree, n_band)."""
    g = np.asarray(st_gpu).reshape(-1)
    r = np.asarray(st_ref).reshape(-1)
    dis = g != r
    if minpiv_ref is not None:
        mp = np.asarray(minpiv_ref).reshape(-1)
        band = (mp > 1e-11) & (mp < 1e-9)
        return int((dis & ~band).sum()), int((dis & band).sum())
    return int(dis.sum()), 0


def rand_irregular(rng, d, n, Nlo, Nhi, dtype=np.float32):
    Ni = rng.integers(Nlo, Nhi + 1, size=n)
    off = np.concatenate([[0], np.cumsum(Ni)]).astype(np.int64)
    t = rng.random((int(off[-1]), d)).astype(dtype)
    y = rng.standard_normal(int(off[-1])).astype(dtype)
    return off, t, y


@contextlib.contextmanager
def engine(F, h, e):
    """Runs the block with the handle's covariance engine set to e (then AUTO)."""
    F.fpca_set_engine(h, e)
    try:
        yield
    finally:
        F.fpca_set_engine(h, F.FPCA_ENGINE_AUTO)

"""CPU pins of the oracle's bandwidth search (Section 3.3): the trust-region
method with a quadratic regression model, and the binned leave-one-out
criterion it minimizes.

- On a criterion that is exactly quadratic in log h the regression model is
  exact, so the search lands on the known minimizer (d = 1, 2, 3).
- A minimizer outside the bandwidth box is replaced by the box boundary.
- With a small deterministic ripple on the quadratic (a noisy criterion) the
  result stays within the ripple's reach of the minimizer.
- When every pair-bin holds exactly one pair located on its node, the binned
  leave-one-out criterion equals brute-force leave-one-observation-out CV of
  the unbinned local-linear fit (numpy lstsq on the weighted design).
"""
import numpy as np
import pytest

import oracle
from oracle import bw_search as B


def _quad(xstar, A, ripple=0.0):
    def fb(hs):
        out = []
        for h in hs:
            x = np.log(h)
            v = float((x - xstar) @ A @ (x - xstar)) + 5.0
            out.append(v + ripple * float(np.sum(np.sin(40.0 * x))))
        return out
    return fb


@pytest.mark.parametrize("d", [1, 2, 3])
def test_exact_quadratic_recovers_minimizer(d):
    rng = np.random.default_rng(d)
    xstar = np.log(rng.uniform(0.08, 0.3, d))
    Rm = np.linalg.qr(rng.standard_normal((d, d)))[0]
    A = Rm @ np.diag(rng.uniform(0.5, 4.0, d)) @ Rm.T
    h, v, n, tr = B.trust_region_search(_quad(xstar, A), d, [0.02] * d, [0.8] * d, [0.4] * d, max_evals=60)
    assert np.max(np.abs(np.log(h) - xstar)) < 1e-6, (np.log(h), xstar, n)
    assert abs(v - 5.0) < 1e-10
    assert n <= 60


def test_box_boundary():
    xstar = np.log(np.array([0.5, 0.1]))
    h, v, n, _ = B.trust_region_search(_quad(xstar, np.diag([1.0, 2.0])), 2, [0.05, 0.05], [0.3, 0.3],
                                       [0.1, 0.2], max_evals=60)
    assert abs(np.log(h[0]) - np.log(0.3)) < 1e-9
    assert abs(np.log(h[1]) - np.log(0.1)) < 1e-4


def test_noisy_quadratic_within_ripple():
    xstar = np.log(np.array([0.15]))
    h, v, n, _ = B.trust_region_search(_quad(xstar, np.array([[3.0]]), ripple=2e-3), 1, [0.02], [0.8], [0.5],
                                       max_evals=40)
    assert abs(np.log(h[0]) - xstar[0]) < 0.05


def test_binned_loo_equals_brute_force_on_nodes():
    M = (9,)  # nodes m/8: exact in binary, so each observation sits on one node
    rng = np.random.default_rng(5)
    nodes = np.arange(9) / 8.0
    pairs = [(a, b) for a in range(9) for b in range(a + 1, 9)]
    rng.shuffle(pairs)
    pairs = pairs[:26]
    off = np.arange(0, 2 * len(pairs) + 1, 2, dtype=np.int64)
    t = np.array([[nodes[a], nodes[b]] for a, b in pairs]).reshape(-1, 1)
    y = rng.standard_normal(t.shape[0])
    C, G, Q = oracle.bin_cov_pairs(M, off, t, y, want_Q=True)
    h = 0.45
    got = B.loo_cv_score(M, [h], C, G, Q)
    # brute force over the ordered pairs (j != l) of every curve, weight 1/2
    loc, val = [], []
    for i, (a, b) in enumerate(pairs):
        ya, yb = y[2 * i], y[2 * i + 1]
        loc += [(nodes[a], nodes[b]), (nodes[b], nodes[a])]
        val += [ya * yb, ya * yb]
    loc, val = np.array(loc), np.array(val)
    w = 0.5
    ref = 0.0
    for k in range(len(val)):
        keep = np.arange(len(val)) != k
        u = (loc[keep] - loc[k]) / h
        K = np.prod(np.clip(1.0 - u * u, 0.0, None), axis=1)
        sw = np.sqrt(w * K)
        X = np.column_stack([np.ones(keep.sum()), u])
        beta = np.linalg.lstsq(X * sw[:, None], val[keep] * sw, rcond=None)[0]
        ref += w * (val[k] - beta[0]) ** 2
    assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)

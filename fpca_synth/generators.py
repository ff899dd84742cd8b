"""Seeded draws from the paper's data model (Section 2, eqs. 2.1-2.2).

Every workload is synthetic. Shapes, sizes and distributions follow the five
benchmark configurations of this project (d=1 FP64 curves; d=2 irregular
surfaces; d=2 dense common-grid Gaussian-process fields; d=3 spatio-temporal
samples on a disk x time domain; a family of d=2 datasets for the bandwidth
surrogate). The paper's own simulations (Section 3, Simulations I and II) are
closed-form models of the same kind.

Grid convention used throughout: M_k nodes per coordinate at m/(M_k-1),
m = 0..M_k-1, flattened with the last coordinate fastest.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

SQRT2 = np.sqrt(2.0)


def fourier_1d(a: int, x: np.ndarray) -> np.ndarray:
    """Orthonormal Fourier functions on [0,1]: 1: sqrt2 sin 2pi x, 2: sqrt2 cos 2pi x,
    3: sqrt2 sin 4pi x, 4: sqrt2 cos 4pi x."""
    x = np.asarray(x, dtype=np.float64)
    if a == 1:
        return SQRT2 * np.sin(2 * np.pi * x)
    if a == 2:
        return SQRT2 * np.cos(2 * np.pi * x)
    if a == 3:
        return SQRT2 * np.sin(4 * np.pi * x)
    if a == 4:
        return SQRT2 * np.cos(4 * np.pi * x)
    raise ValueError(a)


def grid_nodes(M: int) -> np.ndarray:
    return np.arange(M, dtype=np.float64) / (M - 1)


def grid_points(M: Sequence[int]) -> np.ndarray:
    """All nodes of a tensor grid, shape (prod M, d), last coordinate fastest."""
    axes = [grid_nodes(m) for m in M]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in mesh], axis=1)


def fold_assignment(n: int, n_folds: int, seed: int = 11) -> np.ndarray:
    """Curve i goes to fold pi(i) mod n_folds, pi a seeded permutation."""
    perm = np.random.default_rng(seed).permutation(n)
    return (perm % n_folds).astype(np.int32)


def disk_time_mask(M: Sequence[int]) -> np.ndarray:
    """Indicator of the d=3 domain {(x,y,tau): (x-1/2)^2+(y-1/2)^2 <= 1/4} x [0,1] on the grid."""
    pts = grid_points(M)
    inside = (pts[:, 0] - 0.5) ** 2 + (pts[:, 1] - 0.5) ** 2 <= 0.25 + 1e-12
    return inside.astype(np.uint8)


@dataclass
class Dataset:
    """One synthetic workload.

    Irregular design: `offsets` (n+1, int64) delimit curve i's observations
    `t[offsets[i]:offsets[i+1]]` (N x d) and `y[...]` (N). Common-grid design:
    `y` is an n x P matrix of values at the P nodes of `M_cov` (t is None).
    """
    name: str
    d: int
    design: str                      # "irregular" | "common"
    n: int
    offsets: Optional[np.ndarray]
    t: Optional[np.ndarray]
    y: np.ndarray
    M_mean: tuple
    M_cov: tuple
    h_mean: float
    h_cov: float
    dtype: str                       # "f64" | "f32"
    k: int = 3
    oversample: int = 10
    power_iters: int = 2
    rp_seed: int = 7
    mask: Optional[np.ndarray] = None        # uint8 over the covariance marginal grid
    folds: Optional[np.ndarray] = None       # int32 per curve
    n_folds: int = 0
    h_grid: Optional[np.ndarray] = None
    lambdas: Optional[np.ndarray] = None     # true eigenvalues
    eigfun: Optional[Callable] = None        # pts (m,d) -> (m,K) true eigenfunctions
    meanfun: Optional[Callable] = None
    extra: dict = field(default_factory=dict)

    @property
    def np_dtype(self):
        return np.float64 if self.dtype == "f64" else np.float32

    @property
    def N(self) -> int:
        return int(self.offsets[-1]) if self.offsets is not None else self.n * int(np.prod(self.M_cov))


def irregular_kl(rng: np.random.Generator, d: int, N_per_curve: np.ndarray,
                 sampler: Callable, meanfun: Callable, eigfun: Callable,
                 lambdas: np.ndarray, noise_sd: float, dtype) -> tuple:
    """Y_ij = mu(t_ij) + sum_l A_il phi_l(t_ij) + eps_ij with A_il ~ N(0, lambda_l)."""
    N_per_curve = np.asarray(N_per_curve, dtype=np.int64)
    n = N_per_curve.shape[0]
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(N_per_curve)
    tot = int(offsets[-1])
    t = sampler(rng, tot)
    t = np.asarray(t, dtype=dtype)
    scores = rng.standard_normal((n, len(lambdas))) * np.sqrt(np.asarray(lambdas))
    curve = np.repeat(np.arange(n), N_per_curve)
    t64 = t.astype(np.float64)
    phi = eigfun(t64)
    y = meanfun(t64) + np.einsum("ik,ik->i", scores[curve], phi) + noise_sd * rng.standard_normal(tot)
    return offsets, t, y.astype(dtype)


def _uniform_box(d):
    def s(rng, m):
        return rng.random((m, d))
    return s


def _tensor_eigfun(index_tuples):
    def f(pts):
        cols = []
        for tup in index_tuples:
            v = np.ones(pts.shape[0])
            for k, a in enumerate(tup):
                v = v * fourier_1d(a, pts[:, k])
            cols.append(v)
        return np.stack(cols, axis=1)
    return f


def make_c1(seed: int = 1001, n: int = 200, N_i: int = 50) -> Dataset:
    """d=1 FP64: n curves of N_i uniform points; mean sin 2pi t; 3 Fourier components,
    lambda = (1, .5, .25); noise sd 0.1; Epanechnikov h = 0.1; mean grid 101, cov 51x51."""
    rng = np.random.default_rng(seed)
    lambdas = np.array([1.0, 0.5, 0.25])
    eig = _tensor_eigfun([(2,), (1,), (4,)])
    mean = lambda p: np.sin(2 * np.pi * p[:, 0])
    off, t, y = irregular_kl(rng, 1, np.full(n, N_i), _uniform_box(1), mean, eig, lambdas, 0.1, np.float64)
    return Dataset("c1", 1, "irregular", n, off, t, y, (101,), (51,), 0.1, 0.1, "f64",
                   k=3, oversample=10, power_iters=2, lambdas=lambdas, eigfun=eig, meanfun=mean)


C2_INDEX = [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1)]


def make_c2(seed: int = 1002, n: int = 1000, N_range=(100, 300), M: int = 32) -> Dataset:
    """d=2 irregular FP32: N_i ~ U{100..300} uniform points; mean sin(2pi s)cos(2pi t);
    6 tensor Fourier components with lambda_k = 2^-k; noise sd 0.2; h = 0.08; 32^2 grid."""
    rng = np.random.default_rng(seed)
    lambdas = 2.0 ** -np.arange(1, 7)
    eig = _tensor_eigfun(C2_INDEX)
    mean = lambda p: np.sin(2 * np.pi * p[:, 0]) * np.cos(2 * np.pi * p[:, 1])
    Ni = rng.integers(N_range[0], N_range[1] + 1, size=n)
    off, t, y = irregular_kl(rng, 2, Ni, _uniform_box(2), mean, eig, lambdas, 0.2, np.float32)
    return Dataset("c2", 2, "irregular", n, off, t, y, (M, M), (M, M), 0.08, 0.08, "f32",
                   k=10, oversample=10, power_iters=2, lambdas=lambdas, eigfun=eig, meanfun=mean)


def matern15(r: np.ndarray, ell: float) -> np.ndarray:
    a = np.sqrt(3.0) * r / ell
    return (1.0 + a) * np.exp(-a)


def make_c3(seed: int = 1003, n: int = 5000, M: int = 64, ell: float = 0.2,
            noise_sd: float = 0.1) -> Dataset:
    """d=2 dense common grid: n zero-mean Gaussian-process fields with Matern nu=1.5
    covariance (length scale 0.2, variance 1) at the M x M nodes, plus N(0, 0.1^2) noise.
    h = 0.1. The P x P kernel matrix is factored by FP64 Cholesky (jitter 1e-10)."""
    rng = np.random.default_rng(seed)
    pts = grid_points((M, M))
    diff = pts[:, None, :] - pts[None, :, :]
    K = matern15(np.sqrt((diff ** 2).sum(-1)), ell)
    del diff
    P = M * M
    L = np.linalg.cholesky(K + 1e-10 * np.eye(P))
    z = rng.standard_normal((n, P)).astype(np.float32)
    y = z @ L.T.astype(np.float32)
    y += (noise_sd * rng.standard_normal((n, P))).astype(np.float32)
    ds = Dataset("c3", 2, "common", n, None, None, np.ascontiguousarray(y, dtype=np.float32),
                 (M, M), (M, M), 0.1, 0.1, "f32", k=20, oversample=10, power_iters=2)
    ds.extra["kernel_matrix"] = K
    return ds


C4_INDEX = [(a, b, c) for a in (1, 2) for b in (1, 2) for c in (1, 2)]


def make_c4(seed: int = 1004, n: int = 800, N_range=(200, 600), M: int = 16,
            n_h: int = 16, n_folds: int = 5) -> Dataset:
    """d=3 on the disk x time domain: N_i ~ U{200..600} points uniform in the domain
    (rejection sampling); 8 tensor Fourier components, lambda_k = 1/k^2; mean sin(2 pi tau);
    noise sd 0.15; grid 16^3; bandwidths geomspace(0.1, 0.5, 16); 5 leave-curves-out folds."""
    rng = np.random.default_rng(seed)
    lambdas = 1.0 / np.arange(1, 9) ** 2
    eig = _tensor_eigfun(C4_INDEX)
    mean = lambda p: np.sin(2 * np.pi * p[:, 2])

    def sampler(r, m):
        out = np.empty((0, 3))
        while out.shape[0] < m:
            cand = r.random((2 * (m - out.shape[0]) + 16, 3))
            keep = (cand[:, 0] - 0.5) ** 2 + (cand[:, 1] - 0.5) ** 2 <= 0.25
            out = np.concatenate([out, cand[keep]], axis=0)
        return out[:m]

    Ni = rng.integers(N_range[0], N_range[1] + 1, size=n)
    off, t, y = irregular_kl(rng, 3, Ni, sampler, mean, eig, lambdas, 0.15, np.float32)
    Ms = (M, M, M)
    return Dataset("c4", 3, "irregular", n, off, t, y, Ms, Ms, 0.2, 0.2, "f32",
                   k=8, oversample=10, power_iters=2, mask=disk_time_mask(Ms),
                   folds=fold_assignment(n, n_folds), n_folds=n_folds,
                   h_grid=np.geomspace(0.1, 0.5, n_h), lambdas=lambdas, eigfun=eig, meanfun=mean)


def make_surrogate_dataset(index: int, split: str = "train", M: int = 32,
                           n_range=(200, 5000), N_bounds=(20, 400), n_scale: float = 1.0) -> Dataset:
    """One d=2 dataset of the surrogate family: n ~ logU(n_range) (times n_scale),
    each dataset draws its own N_i range inside N_bounds, noise sd ~ U[0.05, 0.5],
    lambda_k = k^-a with a ~ U[1, 3], the six tensor Fourier components of the d=2
    irregular workload. Train seeds 50000+i, test seeds 90000+i."""
    seed = (50_000 if split == "train" else 90_000) + index
    rng = np.random.default_rng(seed)
    n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))) * n_scale))
    n = max(n, 8)
    lo, hi = sorted(rng.integers(N_bounds[0], N_bounds[1] + 1, size=2))
    hi = max(hi, lo + 1)
    noise = rng.uniform(0.05, 0.5)
    a = rng.uniform(1.0, 3.0)
    lambdas = np.arange(1, 7, dtype=np.float64) ** (-a)
    eig = _tensor_eigfun(C2_INDEX)
    mean = lambda p: np.sin(2 * np.pi * p[:, 0]) * np.cos(2 * np.pi * p[:, 1])
    Ni = rng.integers(lo, hi + 1, size=n)
    off, t, y = irregular_kl(rng, 2, Ni, _uniform_box(2), mean, eig, lambdas, noise, np.float32)
    ds = Dataset(f"sur-{split}-{index}", 2, "irregular", n, off, t, y, (M, M), (M, M), 0.1, 0.1,
                 "f32", lambdas=lambdas, eigfun=eig, meanfun=mean,
                 folds=fold_assignment(n, 5, seed=seed + 7), n_folds=5)
    ds.extra.update(noise_sd=noise, decay=a, N_lo=int(lo), N_hi=int(hi))
    return ds


def sim2_eigfun(l: int, pts: np.ndarray) -> np.ndarray:
    """Simulation II's l-th component as printed: prod_i sin(2 l pi t_i) / 2
    (not unit norm: its squared L2 norm on [0,1]^3 is (1/8)^3)."""
    return np.prod(np.sin(2 * l * np.pi * pts) / 2.0, axis=1)


def make_sim2(seed: int = 1006, n: int = 100, M: int = 64, noise_sd: float = 0.25,
              dtype=np.float64) -> Dataset:
    """Simulation II's model on a complete M^3 grid: mu(t) = exp(|t - 1/2|^2),
    Y_i = mu + sum_{l=1..4} A_il phi_l + eps with A_il ~ N(0, 4^(3-l)),
    phi_l as printed (see sim2_eigfun) and eps ~ N(0, 1/16); n = 100 curves.
    The covariance's eigenpairs are lambda_l = 4^(3-l) ||phi_l||^2 with
    eigenfunctions phi_l / ||phi_l||. h = 0.1 (6 grid steps at M = 64)."""
    rng = np.random.default_rng(seed)
    pts = grid_points((M, M, M))
    P = pts.shape[0]
    mu = np.exp(((pts - 0.5) ** 2).sum(1))
    A = rng.standard_normal((n, 4)) * np.sqrt(4.0 ** (3 - np.arange(1, 5)))
    Phi = np.stack([sim2_eigfun(l, pts) for l in range(1, 5)])
    y = np.empty((n, P), dtype=dtype)
    for i in range(n):
        y[i] = mu + A[i] @ Phi + noise_sd * rng.standard_normal(P)
    ds = Dataset("sim2", 3, "common", n, None, None, y, (M, M, M), (M, M, M), 0.1, 0.1,
                 "f64" if dtype == np.float64 else "f32", k=4, oversample=12, power_iters=2)
    ds.extra["mu"] = mu
    ds.extra["scores"] = A
    return ds


def make_config(k: int, **kw) -> Dataset:
    return {1: make_c1, 2: make_c2, 3: make_c3, 4: make_c4}[k](**kw)

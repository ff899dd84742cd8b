"""One pass of the hot path through the C ABI: bin -> smooth mean -> bin
covariance -> smooth covariance -> randomized eigendecomposition.

This module only allocates device buffers (torch) and calls the library in
order; all arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _binding as B


@dataclass
class DeviceData:
    grid_mean: B.Grid
    grid_cov: B.Grid
    dtype: int
    n: int
    offsets: Optional[object]
    t: Optional[object]
    y: object
    design: int
    tdtype: object
    folds: Optional[object] = None
    n_folds: int = 0


def to_device(ds, device="cuda:0") -> DeviceData:
    import torch
    tdt = torch.float64 if ds.dtype == "f64" else torch.float32
    dt = B.FPCA_F64 if ds.dtype == "f64" else B.FPCA_F32
    mask = None
    if ds.mask is not None:
        mask = torch.from_numpy(np.ascontiguousarray(ds.mask, np.uint8)).to(device)
    gm = B.Grid(ds.M_mean)
    gc = B.Grid(ds.M_cov, mask)
    y = torch.from_numpy(np.ascontiguousarray(ds.y)).to(device=device, dtype=tdt)
    if ds.design == "common":
        return DeviceData(gm, gc, dt, ds.n, None, None, y, B.FPCA_COMMON_GRID, tdt)
    off = torch.from_numpy(np.ascontiguousarray(ds.offsets, np.int64)).to(device)
    t = torch.from_numpy(np.ascontiguousarray(ds.t)).to(device=device, dtype=tdt)
    folds = None
    if ds.folds is not None:
        folds = torch.from_numpy(np.ascontiguousarray(ds.folds, np.int32)).to(device)
    return DeviceData(gm, gc, dt, ds.n, off, t, y, B.FPCA_IRREGULAR, tdt, folds, ds.n_folds)


@dataclass
class FitBuffers:
    c: object
    s: object
    mu: object
    mu_status: object
    mu_cov: object
    C: object
    G: object
    gamma: object
    status: Optional[object]
    efuns: object
    evals: Optional[np.ndarray] = None
    fve: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)


def alloc(dd: DeviceData, k: int, with_status: bool = True, analytic_C: bool = False) -> FitBuffers:
    import torch
    dev = dd.y.device
    Pm, Pc = dd.grid_mean.P, dd.grid_cov.P
    z = lambda *s, dt=dd.tdtype: torch.empty(*s, dtype=dt, device=dev)
    return FitBuffers(
        c=z(Pm), s=z(Pm), mu=z(Pm), mu_status=torch.empty(Pm, dtype=torch.int8, device=dev),
        mu_cov=z(Pc),
        C=None if analytic_C else z(Pc, Pc), G=z(Pc, Pc), gamma=z(Pc, Pc),
        status=torch.empty(Pc, Pc, dtype=torch.int8, device=dev) if with_status else None,
        efuns=z(k, Pc))


def fit(h: B.Handle, dd: DeviceData, bufs: FitBuffers, h_mean: float, h_cov: float, k: int,
        oversample: int, power_iters: int, seed: int, prec: Optional[int] = None,
        analytic_C: bool = False, do_eig: bool = True, eig_prec: Optional[int] = None) -> FitBuffers:
    """Queues the whole hot path; returns the buffers (eigenvalues on the host).
    prec: the binning products' precision; eig_prec: that of the range
    finder's products (FP64 or FP32 storage precision when None)."""
    if prec is None:
        prec = B.FPCA_PREC_F64 if dd.dtype == B.FPCA_F64 else B.FPCA_PREC_F32
    if eig_prec is None:
        eig_prec = B.FPCA_PREC_F64 if dd.dtype == B.FPCA_F64 else B.FPCA_PREC_F32
    B.fpca_bin(h, dd.grid_mean, B.FPCA_BIN_MEAN, dd.design, dd.dtype, prec, dd.n, dd.offsets, dd.t,
               dd.y, None, 0, bufs.c, bufs.s)
    B.fpca_smooth_mean(h, dd.grid_mean, dd.dtype, bufs.c, bufs.s, B.FPCA_K_EPANECHNIKOV, h_mean,
                       bufs.mu, bufs.mu_status)
    mu_cov = mean_on_cov_grid(dd, bufs)
    if analytic_C:
        C = None
        # common grid: the pair weights are c_uniform (1 - delta) and are not materialized
        W = None if dd.design == B.FPCA_COMMON_GRID else bufs.extra.setdefault("Cscratch",
                                                                             bufs.G.new_empty(bufs.G.shape))
        B.fpca_bin(h, dd.grid_cov, B.FPCA_BIN_COV, dd.design, dd.dtype, prec, dd.n, dd.offsets, dd.t,
                   dd.y, None, 0, W, bufs.G)
    else:
        C = bufs.C
        B.fpca_bin(h, dd.grid_cov, B.FPCA_BIN_COV, dd.design, dd.dtype, prec, dd.n, dd.offsets, dd.t,
                   dd.y, None, 0, C, bufs.G)
    B.fpca_smooth_cov(h, dd.grid_cov, dd.dtype, C, uniform_pair_weight(dd), bufs.G, mu_cov,
                      B.FPCA_K_EPANECHNIKOV, h_cov, bufs.gamma, bufs.status)
    if do_eig:
        bufs.evals, bufs.fve = B.fpca_eig_randomized(h, dd.dtype, eig_prec, dd.grid_cov, bufs.gamma, None,
                                                     k, oversample, power_iters, seed, bufs.efuns)
    return bufs


def uniform_pair_weight(dd: DeviceData) -> float:
    """Pair weight n/(P(P-1)) of a complete common-grid design (0 otherwise)."""
    if dd.design != B.FPCA_COMMON_GRID:
        return 0.0
    P = dd.grid_cov.P
    return dd.n / (P * (P - 1.0))


def mean_on_cov_grid(dd: DeviceData, bufs: FitBuffers):
    """The mean at the covariance marginal grid: the same tensor when the grids
    coincide, every other node when the covariance grid is nested in the mean
    grid (M_mean - 1 = 2 (M_cov - 1) per coordinate)."""
    Mm, Mc = dd.grid_mean.M, dd.grid_cov.M
    if Mm == Mc:
        return bufs.mu
    step = []
    for a, b in zip(Mm, Mc):
        if (a - 1) % (b - 1) != 0:
            raise ValueError("covariance grid must be nested in the mean grid")
        step.append((a - 1) // (b - 1))
    v = bufs.mu.view(*Mm)
    sl = tuple(slice(None, None, s) for s in step)
    bufs.mu_cov.copy_(v[sl].reshape(-1))
    return bufs.mu_cov

"""ctypes binding of libfpca.so: argument marshalling only.

Every array argument is a torch tensor on the handle's device (or None for an
optional argument); host outputs (eigenvalues, FVE) are returned as numpy
arrays. Work is queued on the current torch stream of that device.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpca.so")

FPCA_OK = 0
FPCA_ERR_INVALID_ARG = -1
FPCA_ERR_DOMAIN = -2
FPCA_ERR_UNSUPPORTED = -3
FPCA_ERR_WORKSPACE = -4
FPCA_ERR_DEVICE = -5
FPCA_STATUS_OK, FPCA_STATUS_FALLBACK, FPCA_STATUS_EMPTY = 0, 1, 2
FPCA_BIN_MEAN, FPCA_BIN_COV = 0, 1
FPCA_IRREGULAR, FPCA_COMMON_GRID = 0, 1
FPCA_F64, FPCA_F32 = 0, 1
FPCA_PREC_F64, FPCA_PREC_F32, FPCA_PREC_BF16X3 = 0, 1, 2
FPCA_K_EPANECHNIKOV = 0
FPCA_CONV_DIRECT, FPCA_CONV_FFT, FPCA_CONV_AUTO = 0, 1, 2
FPCA_COVOP_RECOMPUTE, FPCA_COVOP_STORE_BAND = 0, 1
FPCA_ENGINE_AUTO, FPCA_ENGINE_QUEUE, FPCA_ENGINE_PASSES = 0, 1, 2

EXPORTED_SYMBOLS = [
    "fpca_create", "fpca_destroy", "fpca_set_stream", "fpca_sync", "fpca_last_error",
    "fpca_bin", "fpca_bin_common", "fpca_smooth_mean", "fpca_smooth_cov", "fpca_eig_randomized", "fpca_rng_normal",
    "fpca_cv_batched", "fpca_bw_features", "fpca_bw_num_params", "fpca_bw_mlp_forward",
    "fpca_bw_mlp_backward", "fpca_bw_adam_step", "fpca_noise_variance", "fpca_pace_scores",
    "fpca_reconstruct", "fpca_pace_scores_noalloc", "fpca_cv_select", "fpca_cv_loo", "fpca_bw_search",
    "fpca_set_conv", "fpca_covop_create", "fpca_covop_apply", "fpca_covop_destroy", "fpca_eig_covop",
    "fpca_set_engine", "fpca_stream_create_cu_range", "fpca_stream_destroy",
]


class FpcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fpca error {code}: {msg}")
        self.code = code


class _GridC(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("M", ctypes.c_int * 3), ("mask", ctypes.c_void_p)]


class _CvDataC(ctypes.Structure):
    _fields_ = [("grid", _GridC), ("C", ctypes.c_void_p), ("G", ctypes.c_void_p), ("Q", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
    L.fpca_create.argtypes = [ctypes.POINTER(vp), i32]
    L.fpca_destroy.argtypes = [vp]
    L.fpca_set_stream.argtypes = [vp, vp]
    L.fpca_sync.argtypes = [vp]
    L.fpca_set_conv.argtypes = [vp, i32]
    L.fpca_set_engine.argtypes = [vp, i32]
    L.fpca_stream_create_cu_range.argtypes = [i32, i32, i32, ctypes.POINTER(vp)]
    L.fpca_stream_destroy.argtypes = [vp]
    L.fpca_covop_create.argtypes = [vp, ctypes.POINTER(_GridC), i64, vp, vp, ctypes.POINTER(ctypes.c_double), i32,
                                    ctypes.POINTER(vp)]
    L.fpca_covop_apply.argtypes = [vp, i32, vp, vp]
    L.fpca_covop_destroy.argtypes = [vp]
    L.fpca_eig_covop.argtypes = [vp, vp, i32, i32, i32, u64, ctypes.POINTER(ctypes.c_double), vp,
                                 ctypes.POINTER(ctypes.c_double)]
    L.fpca_reconstruct.argtypes = [vp, i32, i64, i64, i32, vp, vp, vp, vp]
    L.fpca_pace_scores.argtypes = [vp, ctypes.POINTER(_GridC), i32, i32, i64, vp, vp, vp, vp, vp, i32,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp]
    L.fpca_pace_scores_noalloc.argtypes = L.fpca_pace_scores.argtypes
    L.fpca_noise_variance.argtypes = [vp, ctypes.POINTER(_GridC), i32, vp, vp, vp, vp,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.fpca_last_error.restype = ctypes.c_char_p
    L.fpca_bin.argtypes = [vp, ctypes.POINTER(_GridC), i32, i32, i32, i32, i64, vp, vp, vp, vp, i32,
                           vp, vp, vp, vp, vp]
    L.fpca_bin_common.argtypes = [vp, ctypes.POINTER(_GridC), i32, i32, i64, vp, vp, vp, vp, vp, vp]
    L.fpca_smooth_mean.argtypes = [vp, ctypes.POINTER(_GridC), i32, vp, vp, i32,
                                   ctypes.POINTER(ctypes.c_double), vp, vp]
    L.fpca_smooth_cov.argtypes = [vp, ctypes.POINTER(_GridC), i32, vp, ctypes.c_double, vp, vp, i32,
                                  ctypes.POINTER(ctypes.c_double), vp, vp]
    L.fpca_eig_randomized.argtypes = [vp, i32, i32, ctypes.POINTER(_GridC), vp, vp, i32, i32, i32, u64,
                                      ctypes.POINTER(ctypes.c_double), vp,
                                      ctypes.POINTER(ctypes.c_double)]
    L.fpca_rng_normal.argtypes = [vp, u64, i64, vp]
    L.fpca_cv_batched.argtypes = [vp, i32, i32, ctypes.POINTER(_CvDataC), i32, i32,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    dp = ctypes.POINTER(ctypes.c_double)
    L.fpca_cv_loo.argtypes = [vp, ctypes.POINTER(_GridC), i32, vp, vp, vp, i32, dp, dp]
    L.fpca_bw_search.argtypes = [vp, ctypes.POINTER(_GridC), i32, vp, vp, vp, dp, dp, dp, i32, dp, dp,
                                 ctypes.POINTER(i32), dp]
    L.fpca_cv_select.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]
    L.fpca_bw_features.argtypes = [vp, ctypes.POINTER(_GridC), i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.fpca_bw_num_params.argtypes = []
    L.fpca_bw_mlp_forward.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.fpca_bw_mlp_backward.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    f32 = ctypes.c_float
    L.fpca_bw_adam_step.argtypes = [vp, i32, f32, f32, f32, f32, f32, vp, vp, vp, vp]
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise FpcaError(rc, load_library().fpca_last_error().decode())


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if not x.is_cuda:
        raise ValueError("device tensor expected")
    if not x.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return x.data_ptr()


class Grid:
    """Regular grid: d coordinates, M[k] nodes at m/(M_k-1); optional uint8 mask tensor."""

    def __init__(self, M: Sequence[int], mask=None):
        self.M = tuple(int(m) for m in M)
        self.d = len(self.M)
        self.mask = mask
        self.P = int(np.prod(self.M))

    def c(self) -> _GridC:
        g = _GridC()
        g.d = self.d
        for k in range(3):
            g.M[k] = self.M[k] if k < self.d else 1
        g.mask = _ptr(self.mask)
        return g


class Handle:
    """fpca_create / fpca_destroy around one device; binds the current torch stream."""

    def __init__(self, device: int = 0):
        import torch
        self.device = device
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.fpca_create(ctypes.byref(h), device))
        self._h = h
        self._torch = torch

    @property
    def ptr(self):
        stream = self._torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().fpca_set_stream(self._h, ctypes.c_void_p(stream)))
        return self._h

    def sync(self):
        _check(load_library().fpca_sync(self.ptr))

    def close(self):
        if self._h:
            load_library().fpca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fpca_stream_create_cu_range(device: int, cu_begin: int, cu_end: int) -> int:
    """A stream on CU mask bits cu_begin..cu_end-1 of `device`; returns the hipStream_t as an int
    (wrap it with torch.cuda.ExternalStream); release with fpca_stream_destroy."""
    st = ctypes.c_void_p()
    _check(load_library().fpca_stream_create_cu_range(int(device), int(cu_begin), int(cu_end), ctypes.byref(st)))
    return int(st.value)


def fpca_stream_destroy(stream: int):
    _check(load_library().fpca_stream_destroy(ctypes.c_void_p(stream)))


def fpca_bin_common(h: Handle, grid: Grid, dtype: int, prec: int, n: int, y, mean_weights, mean_sums,
                    mean_sq_sums, cov_weights, cov_sums):
    g = grid.c()
    _check(load_library().fpca_bin_common(h.ptr, ctypes.byref(g), dtype, prec, int(n), _ptr(y), _ptr(mean_weights),
                                          _ptr(mean_sums), _ptr(mean_sq_sums), _ptr(cov_weights), _ptr(cov_sums)))


def fpca_bin(h: Handle, grid: Grid, kind: int, design: int, dtype: int, prec: int, n: int,
             offsets, t, y, fold_of_curve, n_folds: int, weights, sums, sq_sums=None,
             bin_index=None, cell_count=None):
    g = grid.c()
    _check(load_library().fpca_bin(h.ptr, ctypes.byref(g), kind, design, dtype, prec, int(n),
                                   _ptr(offsets), _ptr(t), _ptr(y), _ptr(fold_of_curve), int(n_folds),
                                   _ptr(weights), _ptr(sums), _ptr(sq_sums), _ptr(bin_index),
                                   _ptr(cell_count)))


def _bw(bandwidth, d):
    arr = (ctypes.c_double * d)(*[float(b) for b in np.broadcast_to(np.asarray(bandwidth, float), (d,))])
    return arr


def fpca_smooth_mean(h: Handle, grid: Grid, dtype: int, weights, sums, kernel: int, bandwidth, mu,
                     status=None):
    g = grid.c()
    _check(load_library().fpca_smooth_mean(h.ptr, ctypes.byref(g), dtype, _ptr(weights), _ptr(sums),
                                           kernel, _bw(bandwidth, grid.d), _ptr(mu), _ptr(status)))


def fpca_smooth_cov(h: Handle, grid: Grid, dtype: int, C, c_uniform: float, G, mu, kernel: int, bandwidth,
                    gamma, status=None):
    g = grid.c()
    _check(load_library().fpca_smooth_cov(h.ptr, ctypes.byref(g), dtype, _ptr(C), float(c_uniform), _ptr(G),
                                          _ptr(mu),
                                          kernel, _bw(bandwidth, grid.d), _ptr(gamma), _ptr(status)))


def fpca_eig_randomized(h: Handle, dtype: int, prec: int, grid: Grid, gamma, quad_w, k: int,
                        oversample: int, power_iters: int, seed: int, efuns):
    """Returns (evals[k], fve[k]) as numpy arrays; eigenfunctions go to `efuns` (k x P tensor,
    i.e. P x k column-major)."""
    g = grid.c()
    ev = (ctypes.c_double * k)()
    fv = (ctypes.c_double * k)()
    _check(load_library().fpca_eig_randomized(h.ptr, dtype, prec, ctypes.byref(g), _ptr(gamma),
                                              _ptr(quad_w), k, oversample, power_iters,
                                              ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ev, _ptr(efuns),
                                              fv))
    return np.array(ev[:]), np.array(fv[:])


def fpca_noise_variance(h: Handle, grid: Grid, dtype: int, b0, mu, gamma, sigma2_t=None):
    """Returns (sigma2, count); writes the per-node values into sigma2_t when given."""
    g = grid.c()
    s2 = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load_library().fpca_noise_variance(h.ptr, ctypes.byref(g), int(dtype), _ptr(b0), _ptr(mu), _ptr(gamma),
                                              _ptr(sigma2_t), ctypes.byref(s2), ctypes.byref(cnt)))
    return s2.value, cnt.value


def fpca_pace_scores(h: Handle, grid: Grid, design: int, dtype: int, n: int, offsets, t, y, mu, efuns, k: int,
                     evals, sigma2: float, scores):
    g = grid.c()
    ev = (ctypes.c_double * k)(*[float(v) for v in np.asarray(evals, np.float64)[:k]])
    _check(load_library().fpca_pace_scores(h.ptr, ctypes.byref(g), int(design), int(dtype), int(n), _ptr(offsets),
                                           _ptr(t), _ptr(y), _ptr(mu), _ptr(efuns), int(k), ev, float(sigma2),
                                           _ptr(scores)))


def fpca_pace_scores_noalloc(h: Handle, grid: Grid, design: int, dtype: int, n: int, offsets, t, y, mu, efuns,
                             k: int, evals, sigma2: float, scores):
    g = grid.c()
    ev = (ctypes.c_double * k)(*[float(v) for v in np.asarray(evals, np.float64)[:k]])
    _check(load_library().fpca_pace_scores_noalloc(h.ptr, ctypes.byref(g), int(design), int(dtype), int(n),
                                                   _ptr(offsets), _ptr(t), _ptr(y), _ptr(mu), _ptr(efuns), int(k),
                                                   ev, float(sigma2), _ptr(scores)))


def fpca_reconstruct(h: Handle, dtype: int, P: int, n: int, k: int, mu, efuns, scores, xhat):
    _check(load_library().fpca_reconstruct(h.ptr, int(dtype), int(P), int(n), int(k), _ptr(mu), _ptr(efuns),
                                           _ptr(scores), _ptr(xhat)))


def fpca_rng_normal(h: Handle, seed: int, count: int, out):
    _check(load_library().fpca_rng_normal(h.ptr, ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), int(count),
                                          _ptr(out)))


def fpca_bw_features(h: Handle, grid: Grid, n: int, offsets, c, s, s2, C, G, Q, feat):
    g = grid.c()
    _check(load_library().fpca_bw_features(h.ptr, ctypes.byref(g), int(n), _ptr(offsets), _ptr(c), _ptr(s),
                                           _ptr(s2), _ptr(C), _ptr(G), _ptr(Q), _ptr(feat)))


def fpca_bw_num_params() -> int:
    return int(load_library().fpca_bw_num_params())


def fpca_bw_mlp_forward(h: Handle, batch: int, feat, feat_mean, feat_sd, params, out, z1=None, z2=None):
    _check(load_library().fpca_bw_mlp_forward(h.ptr, int(batch), _ptr(feat), _ptr(feat_mean), _ptr(feat_sd),
                                              _ptr(params), _ptr(out), _ptr(z1), _ptr(z2)))


def fpca_bw_mlp_backward(h: Handle, batch: int, feat, feat_mean, feat_sd, params, out, target, z1, z2, work,
                         grad):
    _check(load_library().fpca_bw_mlp_backward(h.ptr, int(batch), _ptr(feat), _ptr(feat_mean), _ptr(feat_sd),
                                               _ptr(params), _ptr(out), _ptr(target), _ptr(z1), _ptr(z2),
                                               _ptr(work), _ptr(grad)))


def fpca_bw_adam_step(h: Handle, step: int, lr: float, beta1: float, beta2: float, eps: float,
                      weight_decay: float, params, grad, m, v):
    _check(load_library().fpca_bw_adam_step(h.ptr, int(step), lr, beta1, beta2, eps, weight_decay, _ptr(params),
                                            _ptr(grad), _ptr(m), _ptr(v)))


def _bw_rows(bandwidths, d):
    bw = np.asarray(bandwidths, np.float64)
    if bw.ndim == 1:
        bw = np.repeat(bw[:, None], d, axis=1)
    return np.ascontiguousarray(bw)


def fpca_cv_batched(h: Handle, dtype: int, data, n_folds: int, bandwidths):
    """data: list of (Grid, C, G, Q) per dataset; bandwidths: n_h x d (or n_h
    scalars shared by all coordinates). Returns scores (n_data x n_h x n_folds)."""
    data = list(data)
    d = data[0][0].d
    bw = _bw_rows(bandwidths, d)
    n_h = bw.shape[0]
    arr = (_CvDataC * len(data))()
    for i, (grid, C, G, Q) in enumerate(data):
        arr[i].grid = grid.c()
        arr[i].C, arr[i].G, arr[i].Q = _ptr(C), _ptr(G), _ptr(Q)
    out = np.zeros(len(data) * n_h * n_folds)
    _check(load_library().fpca_cv_batched(h.ptr, int(dtype), len(data), arr, int(n_folds), n_h,
                                          bw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(len(data), n_h, n_folds)


def fpca_cv_select(bandwidths, cv, d: int = 1) -> np.ndarray:
    """Refined CV bandwidth (n_h rows on a ray, cv summed over folds); returns d values."""
    bw = _bw_rows(bandwidths, d)
    cvv = np.ascontiguousarray(np.asarray(cv, np.float64))
    out = np.zeros(d)
    P = ctypes.POINTER(ctypes.c_double)
    _check(load_library().fpca_cv_select(bw.shape[0], d, bw.ctypes.data_as(P), cvv.ctypes.data_as(P),
                                         out.ctypes.data_as(P)))
    return out


def fpca_cv_loo(h: Handle, grid: Grid, dtype: int, C, G, Q, bandwidths) -> np.ndarray:
    """Leave-one-out criteria (n_h) of the bandwidth rows (n_h x d, or n_h scalars)."""
    bw = _bw_rows(bandwidths, grid.d)
    out = np.zeros(bw.shape[0])
    g = grid.c()
    P = ctypes.POINTER(ctypes.c_double)
    _check(load_library().fpca_cv_loo(h.ptr, ctypes.byref(g), int(dtype), _ptr(C), _ptr(G), _ptr(Q), bw.shape[0],
                                      bw.ctypes.data_as(P), out.ctypes.data_as(P)))
    return out


def fpca_bw_search(h: Handle, grid: Grid, dtype: int, C, G, Q, h_lo, h_hi, h_init, max_evals: int = 40):
    """Trust-region bandwidth search; returns (h (d), criterion, evaluations, trace (n x (d+1)))."""
    d = grid.d
    arr = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (d,)))
    lo, hi, h0 = arr(h_lo), arr(h_hi), arr(h_init)
    hout = np.zeros(d)
    cv = np.zeros(1)
    n = ctypes.c_int(0)
    trace = np.zeros((max_evals, d + 1))
    g = grid.c()
    P = ctypes.POINTER(ctypes.c_double)
    _check(load_library().fpca_bw_search(h.ptr, ctypes.byref(g), int(dtype), _ptr(C), _ptr(G), _ptr(Q),
                                         lo.ctypes.data_as(P), hi.ctypes.data_as(P), h0.ctypes.data_as(P),
                                         int(max_evals), hout.ctypes.data_as(P), cv.ctypes.data_as(P),
                                         ctypes.byref(n), trace.ctypes.data_as(P)))
    return hout, float(cv[0]), int(n.value), trace[:min(n.value, max_evals)]


def fpca_set_engine(h: Handle, engine: int):
    """Covariance smoother engine: FPCA_ENGINE_AUTO, FPCA_ENGINE_QUEUE or FPCA_ENGINE_PASSES."""
    _check(load_library().fpca_set_engine(h.ptr, int(engine)))


def fpca_set_conv(h: Handle, mode: int):
    """Pass method of the general smoother: FPCA_CONV_DIRECT, FPCA_CONV_FFT or FPCA_CONV_AUTO."""
    _check(load_library().fpca_set_conv(h.ptr, int(mode)))


class CovOp:
    """fpca_covop_create / fpca_covop_destroy: the smoothed covariance of
    complete common-grid curves Y (n x P, FP64 device) as an operator."""

    def __init__(self, h: Handle, grid: Grid, Y, mu, bandwidth, mode: int = FPCA_COVOP_RECOMPUTE):
        self.h = h
        self.grid = grid
        g = grid.c()
        op = ctypes.c_void_p()
        _check(load_library().fpca_covop_create(h.ptr, ctypes.byref(g), int(Y.shape[0]), _ptr(Y), _ptr(mu),
                                                _bw(bandwidth, grid.d), int(mode), ctypes.byref(op)))
        self._op = op

    def apply(self, X, out):
        """out = Gamma_hat X for X, out: P x r row-major FP64 device tensors."""
        self.h.ptr  # binds the current stream to the handle
        _check(load_library().fpca_covop_apply(self._op, int(X.shape[1]), _ptr(X), _ptr(out)))

    def eig(self, quad_w, k: int, oversample: int, power_iters: int, seed: int, efuns):
        """fpca_eig_covop; returns (evals[k], fve[k]); efuns: k x P FP64 tensor."""
        self.h.ptr
        ev = (ctypes.c_double * k)()
        fv = (ctypes.c_double * k)()
        _check(load_library().fpca_eig_covop(self._op, _ptr(quad_w), k, oversample, power_iters,
                                             ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ev, _ptr(efuns), fv))
        return np.array(ev[:]), np.array(fv[:])

    def close(self):
        if self._op:
            load_library().fpca_covop_destroy(self._op)
            self._op = None

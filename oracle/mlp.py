"""FP64 reference of the bandwidth surrogate (test infrastructure only).

The feature vector and the network follow the definitions stated in
include/fpca.h for fpca_bw_features and fpca_bw_mlp_*: 32 summary statistics
of the binned arrays; MLP 32 -> 128 GELU -> 128 GELU -> 1 with the exact GELU
z Phi(z); loss mean (out - target)^2; Adam (Kingma & Ba 2015) with decoupled
weight decay.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NF, NH, NLAG = 32, 128, 8
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X):
    """X: standardized features (B x 32). Returns out (B,) and the cache."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    out = h2 @ p["W3"] + p["b3"][0]
    return out, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, y):
    """Mean squared error and its gradient by back-propagation."""
    p = unpack(theta)
    out, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    r = out - y
    loss = float(np.mean(r * r))
    dout = 2.0 * r / B
    gW3 = h2.T @ dout
    gb3 = np.array([dout.sum()])
    dz2 = (dout[:, None] * p["W3"][None, :]) * gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
    return loss, grad


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def features(M, offsets, c, s, s2, C, G, Q=None):
    """The 32 summary features (the list in include/fpca.h, in that order)."""
    M = tuple(M)
    d = len(M)
    P = int(np.prod(M))
    C = np.asarray(C, np.float64).reshape(P, P)
    G = np.asarray(G, np.float64).reshape(P, P)
    c, s = np.asarray(c, np.float64), np.asarray(s, np.float64)
    Ni = np.diff(np.asarray(offsets, np.int64)).astype(np.float64)
    n = len(Ni)
    tiny = 1e-30
    f = np.zeros(NF)
    meanN = Ni.mean()
    f[0] = math.log(n)
    f[1] = math.log(max(meanN, 1.0))
    f[2] = math.log(max((Ni * (Ni - 1)).sum(), 1.0))
    f[3] = math.sqrt(max((Ni * Ni).mean() - meanN ** 2, 0.0)) / max(meanN, tiny)
    f[4] = math.log(P)
    f[5] = c.sum() ** 2 / max(P * (c * c).sum(), tiny)
    f[6] = (C > 0).sum() / (P * P)
    EY2 = (np.asarray(s2, np.float64).sum() if s2 is not None else 0.0) / max(c.sum(), tiny)
    EY = s.sum() / max(c.sum(), tiny)
    g0 = np.trace(G) / max(np.trace(C), tiny)
    f[7] = math.log(max(EY2, tiny))
    f[8] = EY * EY / max(EY2, tiny)
    f[9] = math.log(max(abs(g0), tiny))
    f[10] = (EY2 - g0) / max(EY2, tiny)
    if Q is not None:
        Q = np.asarray(Q, np.float64).reshape(P, P)
        gbar = G.sum() / max(C.sum(), tiny)
        qbar = Q.sum() / max(C.sum(), tiny)
        f[11] = math.log(max(qbar - gbar * gbar, tiny))
    coords = np.stack(np.unravel_index(np.arange(P), M), axis=1)
    diff = np.abs(coords[:, None, :] - coords[None, :, :])
    gs = g0 if abs(g0) > tiny else tiny
    lags = []
    for k in (0, d - 1):
        others = [j for j in range(d) if j != k]
        same = np.all(diff[:, :, others] == 0, axis=2) if others else np.ones((P, P), bool)
        g = np.zeros(NLAG)
        for l in range(1, NLAG + 1):
            sel = same & (diff[:, :, k] == l)
            g[l - 1] = G[sel].sum() / max(C[sel].sum(), tiny)
        lags.append(g)
    f[12:20] = lags[0] / gs
    f[20:28] = lags[1] / gs
    f[28] = (lags[0][1] - 2 * lags[0][0] + g0) / gs
    f[29] = (lags[1][1] - 2 * lags[1][0] + g0) / gs
    f[30] = math.log(max(C.sum() / (P * P), tiny))
    f[31] = math.log(1.0 / (M[0] - 1))
    return f

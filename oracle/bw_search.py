"""Oracle of the paper's bandwidth search (Section 3.3): leave-one-observation-
out cross-validation of the covariance smoother, minimized over continuous
bandwidths by a derivative-free trust-region method whose local model is a
quadratic REGRESSION on the sampled criterion (the paper replaces the
interpolation step of the trust-region interpolation method by a regression
because the empirical criterion is noisy).

TEST INFRASTRUCTURE ONLY (see the package header). FP64 throughout.

Reading of the binned criterion: on binned data, leaving one observation out
is read as leaving its bin out: at node x the local-linear fit is computed
with x's own bin removed (its weight and sum leave S0 and T0; u = 0 there, so
no other moment changes), and the held-in data are scored through their bins:
  CV(h) = sum_x [ Q(x) - 2 G(x) b_{-x}(x) + C(x) b_{-x}(x)^2 ]
(= sum over pairs of w (Y_ij Y_il - b_{-x})^2 spread over the pair's bins;
b_{-x} is 0 where the reduced window is empty and outside the domain mask).
When every bin holds one pair located on its node, this is exactly the
leave-one-observation-out criterion.

The search works on x = log h (one coordinate per grid coordinate, shared by
the s- and t-coordinates). All constants of the algorithm are listed in
`trust_region_search`.
"""
from __future__ import annotations

import numpy as np


def loo_cv_score(M, h, C, G, Q, mask=None):
    """The binned leave-one-out criterion above for bandwidth vector h (d)."""
    from . import num_moments, smooth, wls_from_moments
    M = tuple(int(m) for m in M)
    d = len(M)
    D = 2 * d
    P = int(np.prod(M))
    hh = np.broadcast_to(np.asarray(h, np.float64), (d,))
    C = np.asarray(C, np.float64).reshape(P * P)
    G = np.asarray(G, np.float64).reshape(P * P)
    Q = np.asarray(Q, np.float64).reshape(P * P)
    _, _, mom, _ = smooth(M + M, np.concatenate([hh, hh]), C, G, want_moments=True)
    mom = np.array(mom, np.float64)
    nc = 1 + D + D * (D + 1) // 2
    mom[:, 0] -= C  # the node's own bin leaves S0 ...
    mom[:, nc] -= G  # ... and T0
    b, _, _ = wls_from_moments(D, mom)
    b = np.where(np.isnan(b), 0.0, b)
    if mask is not None:
        mk = np.asarray(mask).astype(bool).reshape(P)
        out = ~(mk[:, None] & mk[None, :]).reshape(P * P)
        b[out] = 0.0
    assert num_moments(D) == mom.shape[1]
    return float(np.sum(Q - 2.0 * G * b + C * b * b))


def _tr_step(g, H):
    """argmin g.z + z.H.z/2 over |z| <= 1: the Newton point if H is positive
    definite and it lies inside, else the boundary point (H + mu I)^{-1}
    (-g) with |.| = 1 found by 200 bisection steps on mu (and the
    eigenvector of the smallest eigenvalue added in the hard case)."""
    lam, V = np.linalg.eigh(H)
    gam = V.T @ g
    if lam[0] > 0.0:
        zn = -V @ (gam / lam)
        if np.linalg.norm(zn) <= 1.0:
            return zn
    mu_lo = max(0.0, -lam[0])
    phi = lambda mu: float(np.sum(gam * gam / (lam + mu) ** 2))
    tiny = 1e-14 * max(1.0, abs(lam).max())
    if lam[0] + mu_lo <= tiny and abs(gam[0]) <= 1e-14 * max(1.0, np.linalg.norm(g)):
        # hard case: g has no component along the flattest direction
        others = lam + mu_lo > tiny
        z = np.zeros_like(g)
        z[others] = -gam[others] / (lam[others] + mu_lo)
        t2 = 1.0 - float(np.sum(z * z))
        z[0] = np.sqrt(max(t2, 0.0))
        return V @ z
    lo = mu_lo
    hi = mu_lo + np.linalg.norm(gam) + 1e-12
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if lam[0] + mid <= 0.0 or phi(mid) > 1.0:
            lo = mid
        else:
            hi = mid
    return -V @ (gam / (lam + hi))


def _quad_basis(z):
    d = z.shape[1]
    cols = [np.ones(len(z))] + [z[:, k] for k in range(d)]
    for k in range(d):
        for l in range(k, d):
            cols.append(z[:, k] * z[:, l])
    return np.stack(cols, axis=1)


def _fit(Z, f):
    """Least-squares quadratic (normal equations with a 1e-10 relative ridge,
    Cholesky solve); returns (c0, g, H) of c0 + g.z + z.H.z/2."""
    A = _quad_basis(Z)
    N = A.T @ A
    N = N + 1e-10 * np.trace(N) / N.shape[0] * np.eye(N.shape[0])
    L = np.linalg.cholesky(N)
    c = np.linalg.solve(L.T, np.linalg.solve(L, A.T @ f))
    d = Z.shape[1]
    g = c[1:1 + d].copy()
    H = np.zeros((d, d))
    i = 1 + d
    for k in range(d):
        for l in range(k, d):
            if k == l:
                H[k, k] = 2.0 * c[i]
            else:
                H[k, l] = H[l, k] = c[i]
            i += 1
    return c[0], g, H


def trust_region_search(fbatch, d, h_lo, h_hi, h_init, max_evals=40):
    """Minimize the criterion over log h in the box [log h_lo, log h_hi].

    fbatch(list of h vectors) -> list of criterion values (one batch per call).
    Constants: initial radius 0.25 x the widest box side (clamped to
    [0.05, 1]); minimum radius 0.01; maximum 1; acceptance eta1 = 0.1,
    expansion eta2 = 0.75 when the step reaches 0.9 of the radius; regression
    on the points within 2 radii (max norm) of the centre, else the p + 1
    nearest (p = (d+1)(d+2)/2); after a rejected step one geometry point
    centre + radius e_k (k cycling; minus if already sampled) is evaluated with
    the next candidate. Returns (h, value, evaluations, trace of (h, value))."""
    lo = np.log(np.broadcast_to(np.asarray(h_lo, np.float64), (d,)))
    hi = np.log(np.broadcast_to(np.asarray(h_hi, np.float64), (d,)))
    x0 = np.clip(np.log(np.broadcast_to(np.asarray(h_init, np.float64), (d,))), lo, hi)
    delta = float(np.clip(0.25 * np.max(hi - lo), 0.05, 1.0))
    dmin, dmax, eta1, eta2 = 0.01, 1.0, 0.1, 0.75
    p = (d + 1) * (d + 2) // 2
    X, F = [], []

    def evaluate(pts):
        pts = [np.clip(np.asarray(q, np.float64), lo, hi) for q in pts]
        vals = fbatch([np.exp(q) for q in pts])
        for q, v in zip(pts, vals):
            X.append(q)
            F.append(float(v))
        return pts, [float(v) for v in vals]

    def seen(q):
        return any(np.array_equal(q, r) for r in X)

    # initial design around x0
    E = np.eye(d)
    design = [x0.copy()]
    for k in range(d):
        design += [x0 + delta * E[k], x0 - delta * E[k]]
    for k in range(d):
        design += [x0 + 0.5 * delta * E[k], x0 - 0.5 * delta * E[k]]
    for k in range(d):
        for l in range(k + 1, d):
            design.append(x0 + 0.5 * delta * (E[k] + E[l]))
    uniq = []
    for q in design:
        q = np.clip(q, lo, hi)
        if not any(np.array_equal(q, r) for r in uniq):
            uniq.append(q)
    evaluate(uniq)
    b = int(np.argmin(F))
    xc, fc = X[b].copy(), F[b]
    it = 0
    failed = False
    while len(X) < max_evals and delta >= dmin:
        XA = np.array(X)
        dist = np.max(np.abs(XA - xc), axis=1)
        sel = np.nonzero(dist <= 2.0 * delta)[0]
        if len(sel) < p + 1:
            e2 = np.linalg.norm(XA - xc, axis=1)
            sel = np.argsort(e2, kind="stable")[:p + 1]
        Z = (XA[sel] - xc) / delta
        c0, g, H = _fit(Z, np.array(F)[sel])
        z = _tr_step(g, H)
        xp = np.clip(xc + delta * z, lo, hi)
        if np.linalg.norm(xp - xc) <= 1e-6:
            delta *= 0.5
            it += 1
            failed = True
            continue
        batch = [xp]
        if failed:
            k = it % d
            xg = np.clip(xc + delta * E[k], lo, hi)
            if seen(xg):
                xg = np.clip(xc - delta * E[k], lo, hi)
            if not seen(xg) and not np.array_equal(xg, xp):
                batch.append(xg)
        pts, vals = evaluate(batch)
        zs = (pts[0] - xc) / delta
        pred = -(float(g @ zs) + 0.5 * float(zs @ H @ zs))
        rho = (fc - vals[0]) / pred if pred > 0.0 else -1.0
        if rho >= eta1 and vals[0] < fc:
            xc, fc = pts[0].copy(), vals[0]
            if rho >= eta2 and np.linalg.norm(zs) >= 0.9:
                delta = min(2.0 * delta, dmax)
            failed = False
        else:
            delta *= 0.5
            failed = True
        if len(vals) > 1 and vals[1] < fc:
            xc, fc = pts[1].copy(), vals[1]
        it += 1
    b = int(np.argmin(F))
    return np.exp(X[b]), F[b], len(X), [(np.exp(q), v) for q, v in zip(X, F)]

"""Bandwidth surrogate for the covariance smoother: label datasets with the
library's batched cross-validation, train the MLP with the library's forward,
backward and Adam kernels, and select h for new data (batched CV is the
fallback when the prediction leaves the trained range).

Every arithmetic step runs in the HIP library; this module orders the calls,
keeps host copies of labels and features, and saves/loads the trained model
(npz, loaded with allow_pickle=False).

CLI (runs on the GPU):
  python -m paper_1510_04439_amd.surrogate --n-train 2000 --n-test 300 \
      --out gpurun_out/bw_surrogate.npz --report gpurun_out/bw_surrogate.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "data", "bw_surrogate.npz")
H_GRID = np.geomspace(0.05, 0.28, 16)  # covariance bandwidths on the 32 x 32 grid
N_FOLDS = 5


def log(msg):
    print(f"[surrogate] {msg}", flush=True)


@dataclass
class Binned:
    grid: B.Grid
    n: int
    offsets: object
    c: object
    s: object
    s2: object
    C: object   # (N_FOLDS+1) x P x P
    G: object
    Q: object


def bin_dataset(h: B.Handle, ds, n_folds: int = N_FOLDS) -> Binned:
    """Mean binning (with the sums of Y^2) and covariance binning with folds."""
    import torch
    dev = "cuda:0"
    grid = B.Grid(ds.M_cov)
    P = grid.P
    off = torch.from_numpy(np.ascontiguousarray(ds.offsets, np.int64)).to(dev)
    t = torch.from_numpy(np.ascontiguousarray(ds.t, np.float32)).to(dev)
    y = torch.from_numpy(np.ascontiguousarray(ds.y, np.float32)).to(dev)
    folds = torch.from_numpy(np.ascontiguousarray(ds.folds, np.int32)).to(dev)
    f32 = dict(dtype=torch.float32, device=dev)
    c, s, s2 = (torch.empty(P, **f32) for _ in range(3))
    B.fpca_bin(h, grid, B.FPCA_BIN_MEAN, B.FPCA_IRREGULAR, B.FPCA_F32, B.FPCA_PREC_F32, ds.n, off, t, y, None, 0,
               c, s, s2)
    C, G, Q = (torch.empty(n_folds + 1, P, P, **f32) for _ in range(3))
    B.fpca_bin(h, grid, B.FPCA_BIN_COV, B.FPCA_IRREGULAR, B.FPCA_F32, B.FPCA_PREC_F32, ds.n, off, t, y, folds,
               n_folds, C, G, Q)
    return Binned(grid, ds.n, off, c, s, s2, C, G, Q)


def features(h: B.Handle, bd: Binned, out=None):
    import torch
    if out is None:
        out = torch.empty(32, dtype=torch.float32, device="cuda:0")
    B.fpca_bw_features(h, bd.grid, bd.n, bd.offsets, bd.c, bd.s, bd.s2, bd.C[0], bd.G[0], bd.Q[0], out)
    return out


def cv_scores(h: B.Handle, bd: Binned, hs) -> np.ndarray:
    """CV(h) summed over folds for each bandwidth in hs."""
    sc = B.fpca_cv_batched(h, B.FPCA_F32, [(bd.grid, bd.C, bd.G, bd.Q)], N_FOLDS, np.asarray(hs, np.float64))
    return sc[0].sum(axis=1)


def refine_argmin(hs, scores) -> float:
    """Grid argmin of the CV curve, refined by the vertex of the parabola
    through the three neighbouring points in log h (fpca_cv_select)."""
    return float(B.fpca_cv_select(np.asarray(hs, np.float64), np.asarray(scores, np.float64), 1)[0])


class Surrogate:
    """The trained network (device tensors) and its input standardization."""

    def __init__(self, params, fmu, fsd, h_lo, h_hi):
        import torch
        dev = "cuda:0"
        self.params = torch.as_tensor(np.asarray(params, np.float32), device=dev)
        self.fmu = torch.as_tensor(np.asarray(fmu, np.float32), device=dev)
        self.fsd = torch.as_tensor(np.asarray(fsd, np.float32), device=dev)
        self.h_lo, self.h_hi = float(h_lo), float(h_hi)
        self._out = torch.empty(1, dtype=torch.float32, device=dev)

    @staticmethod
    def load(path: str = MODEL_PATH) -> "Surrogate":
        z = np.load(path, allow_pickle=False)
        return Surrogate(z["params"], z["feat_mean"], z["feat_sd"], float(z["h_lo"]), float(z["h_hi"]))

    def save(self, path: str, extra: Optional[dict] = None):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        arrs = dict(params=self.params.cpu().numpy(), feat_mean=self.fmu.cpu().numpy(),
                    feat_sd=self.fsd.cpu().numpy(), h_lo=np.float64(self.h_lo), h_hi=np.float64(self.h_hi))
        if extra:
            arrs.update({k: np.asarray(v) for k, v in extra.items()})
        np.savez(path, **arrs)

    def predict_log_h(self, h: B.Handle, feat, batch: int = 1):
        out = self._out if batch == 1 else feat.new_empty(batch)
        B.fpca_bw_mlp_forward(h, batch, feat, self.fmu, self.fsd, self.params, out)
        return out

    def select(self, h: B.Handle, bd: Binned, feat=None):
        """Returns (h_selected, used_fallback)."""
        if feat is None:
            feat = features(h, bd)
        lh = float(self.predict_log_h(h, feat).item())
        hv = math.exp(lh) if math.isfinite(lh) else float("nan")
        if not (0.9 * self.h_lo <= hv <= 1.1 * self.h_hi):
            sc = cv_scores(h, bd, H_GRID)
            return refine_argmin(H_GRID, sc), True
        return min(max(hv, self.h_lo), self.h_hi), False


def train(h: B.Handle, feats: np.ndarray, targets: np.ndarray, steps: int = 4000, lr: float = 2e-3,
          wd: float = 1e-4, seed: int = 0) -> Surrogate:
    """Full-batch Adam on mean (out - log h_CV)^2 with the library's kernels."""
    import torch
    dev = "cuda:0"
    N = feats.shape[0]
    fmu = feats.mean(0)
    fsd = feats.std(0)
    fsd = np.where(fsd > 1e-6, fsd, 1.0)
    rng = np.random.default_rng(seed)
    npar = B.fpca_bw_num_params()
    theta = np.zeros(npar, np.float32)
    # He-style initialization of the weights, zero biases
    o = 0
    for fan_in, fan_out in ((32, 128), (128, 128), (128, 1)):
        w = rng.standard_normal(fan_in * fan_out) * math.sqrt(2.0 / fan_in)
        theta[o:o + fan_in * fan_out] = w
        o += fan_in * fan_out + fan_out
    theta[-1] = float(np.mean(targets))
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    prm, ft, mu_t, sd_t, tg = T(theta), T(feats), T(fmu), T(fsd), T(targets)
    out = torch.empty(N, dtype=torch.float32, device=dev)
    z1 = torch.empty(N, 128, dtype=torch.float32, device=dev)
    z2 = torch.empty_like(z1)
    work = torch.empty(N * 257, dtype=torch.float32, device=dev)
    grad = torch.empty(npar, dtype=torch.float32, device=dev)
    m = torch.zeros(npar, dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    for step in range(1, steps + 1):
        B.fpca_bw_mlp_forward(h, N, ft, mu_t, sd_t, prm, out, z1, z2)
        B.fpca_bw_mlp_backward(h, N, ft, mu_t, sd_t, prm, out, tg, z1, z2, work, grad)
        B.fpca_bw_adam_step(h, step, lr, 0.9, 0.999, 1e-8, wd, prm, grad, m, v)
        if step % 500 == 0 or step == 1:
            o_h = out.cpu().numpy()
            log(f"step {step}: train MSE on log h = {np.mean((o_h - targets) ** 2):.5f}")
    s = Surrogate(prm.cpu().numpy(), fmu, fsd, H_GRID[0], H_GRID[-1])
    return s


def label_many(h: B.Handle, split: str, count: int, n_scale: float, start: int = 0):
    """Features, CV scores on H_GRID and refined labels for datasets start..start+count-1."""
    from fpca_synth import make_surrogate_dataset
    feats, labels, scores, qtot, meta = [], [], [], [], []
    t0 = time.time()
    for i in range(start, start + count):
        ds = make_surrogate_dataset(i, split, n_scale=n_scale)
        bd = bin_dataset(h, ds)
        f = features(h, bd).cpu().numpy()
        sc = cv_scores(h, bd, H_GRID)
        feats.append(f)
        scores.append(sc)
        labels.append(refine_argmin(H_GRID, sc))
        qtot.append(float(bd.Q[1:].sum(dtype=__import__("torch").float64).item()))
        meta.append((ds.n, ds.extra["noise_sd"], ds.extra["decay"], ds.extra["N_lo"], ds.extra["N_hi"]))
        if (i - start + 1) % 100 == 0:
            log(f"{split}: labelled {i - start + 1}/{count} datasets ({time.time() - t0:.0f} s)")
    return (np.array(feats), np.array(labels), np.array(scores), np.array(qtot), np.array(meta))


def hdep_loss(score, s_min, q):
    """Loss of a selected bandwidth on the h-dependent part of the CV score:
    (CV(h) - min_grid CV) / |min_grid CV - q|, with q the h-independent sum of
    the held-out squared products (0 at the grid optimum, > 0 when worse)."""
    return (score - s_min) / abs(s_min - q)


def best_constant_h(scores: np.ndarray, qtot: np.ndarray) -> float:
    """The bandwidth of H_GRID with the smallest mean h-dependent loss over
    labelled (training) datasets: the best selector that ignores the data."""
    smin = scores.min(axis=1)
    loss = (scores - smin[:, None]) / np.abs(smin - qtot)[:, None]
    return float(H_GRID[int(np.argmin(loss.mean(axis=0)))])


def evaluate(h: B.Handle, model: Surrogate, split: str, count: int, n_scale: float, start: int = 0,
             h_const: Optional[float] = None):
    """Held-out comparison of surrogate selection against batched CV: CV-score
    ratio CV(h_sur)/min_grid CV, the loss on the h-dependent part (hdep_loss)
    for the surrogate and for a constant bandwidth, |log h_sur - log h_CV| and
    the times of both selectors (after the shared binning)."""
    import torch
    from fpca_synth import make_surrogate_dataset
    rows = []
    for i in range(start, start + count):
        ds = make_surrogate_dataset(i, split, n_scale=n_scale)
        bd = bin_dataset(h, ds)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hs, fb = model.select(h, bd)
        torch.cuda.synchronize()
        t_sur = time.perf_counter() - t0
        t0 = time.perf_counter()
        sc = cv_scores(h, bd, H_GRID)
        h_cv = refine_argmin(H_GRID, sc)
        t_cv = time.perf_counter() - t0
        s_sur = float(cv_scores(h, bd, [hs])[0])
        s_min = float(sc.min())
        q = float(bd.Q[1:].sum(dtype=torch.float64).item())
        row = dict(n=ds.n, h_sur=hs, h_cv=h_cv, fallback=fb, ratio=s_sur / s_min,
                   loss=hdep_loss(s_sur, s_min, q), dlogh=abs(math.log(hs) - math.log(h_cv)),
                   t_sur=t_sur, t_cv=t_cv)
        if h_const is not None:
            s_c = float(sc[int(np.argmin(np.abs(H_GRID - h_const)))])
            row.update(const_ratio=s_c / s_min, const_loss=hdep_loss(s_c, s_min, q))
        rows.append(row)
        if (i - start + 1) % 50 == 0:
            log(f"evaluated {i - start + 1}/{count}")
    return rows


def summarize(rows):
    r = np.array([x["ratio"] for x in rows])
    e = np.array([x["loss"] for x in rows])
    d = np.array([x["dlogh"] for x in rows])
    ts = np.array([x["t_sur"] for x in rows])
    tc = np.array([x["t_cv"] for x in rows])
    out = dict(count=len(rows), ratio_mean=float(r.mean()), ratio_p95=float(np.percentile(r, 95)),
               ratio_max=float(r.max()),
               hdep_loss_mean=float(e.mean()), hdep_loss_p95=float(np.percentile(e, 95)),
               hdep_loss_max=float(e.max()),
               dlogh_mean=float(d.mean()), fallback_rate=float(np.mean([x["fallback"] for x in rows])),
               t_sur_ms_median=float(np.median(ts) * 1e3), t_cv_ms_median=float(np.median(tc) * 1e3),
               speedup_median=float(np.median(tc / ts)))
    if rows and "const_loss" in rows[0]:
        c = np.array([x["const_loss"] for x in rows])
        cr = np.array([x["const_ratio"] for x in rows])
        out.update(const_hdep_loss_mean=float(c.mean()), const_hdep_loss_p95=float(np.percentile(c, 95)),
                   const_hdep_loss_max=float(c.max()), const_ratio_max=float(cr.max()))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--train-start", type=int, default=0, help="index of the first training dataset")
    ap.add_argument("--n-test", type=int, default=300)
    ap.add_argument("--n-scale", type=float, default=1.0)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--labels-out", default=None, help="save the training labels (npz) and stop")
    ap.add_argument("--labels-in", default=None,
                    help="comma-separated label files from --labels-out to train on (no labelling)")
    ap.add_argument("--model-in", default=None, help="evaluate this trained model (no labelling or training)")
    ap.add_argument("--n-const", type=int, default=500,
                    help="training datasets labelled to choose the constant-bandwidth baseline")
    ap.add_argument("--out", default="gpurun_out/bw_surrogate.npz")
    ap.add_argument("--report", default="gpurun_out/bw_surrogate.json")
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available()
    h = B.Handle(0)
    if args.model_in:
        model = Surrogate.load(args.model_in)
        _, _, sc_c, q_c, _ = label_many(h, "train", args.n_const, args.n_scale, start=0)
        h_const = best_constant_h(sc_c, q_c)
        log(f"constant-bandwidth baseline from {args.n_const} training datasets: h = {h_const:.4f}")
        rows = evaluate(h, model, "test", args.n_test, args.n_scale, h_const=h_const)
        summ = summarize(rows)
        summ.update(model=os.path.basename(args.model_in), h_grid=H_GRID.tolist(), h_const=h_const,
                    n_const=args.n_const)
        with open(args.report, "w") as fh:
            json.dump(dict(summary=summ, rows=rows), fh)
        log(json.dumps(summ))
        h.close()
        return
    if args.labels_in:
        parts = [np.load(f) for f in args.labels_in.split(",")]
        ftr = np.concatenate([z["feats"] for z in parts])
        ltr = np.concatenate([z["labels"] for z in parts])
        log(f"loaded {len(ltr)} labelled training datasets")
    else:
        log(f"labelling {args.n_train} training datasets from index {args.train_start}")
        ftr, ltr, str_, qtr, mtr = label_many(h, "train", args.n_train, args.n_scale, start=args.train_start)
        if args.labels_out:
            np.savez(args.labels_out, feats=ftr, labels=ltr, scores=str_, qtot=qtr, meta=mtr,
                     start=args.train_start, n_scale=args.n_scale)
            log(f"saved {args.labels_out}")
            h.close()
            return
    log("training")
    model = train(h, ftr, np.log(ltr), steps=args.steps)
    model.save(args.out)
    log(f"saved {args.out}; evaluating on {args.n_test} held-out datasets")
    rows = evaluate(h, model, "test", args.n_test, args.n_scale)
    summ = summarize(rows)
    summ.update(n_train=len(ltr), n_scale=args.n_scale, steps=args.steps, h_grid=H_GRID.tolist(),
                label_log_h_sd=float(np.std(np.log(ltr))))
    with open(args.report, "w") as fh:
        json.dump(dict(summary=summ, rows=rows), fh)
    log(json.dumps(summ))
    h.close()


if __name__ == "__main__":
    main()

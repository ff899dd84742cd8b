"""Benchmark of the multi-dimensional FPCA hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): d = 2 dense
common-grid data, n = 5000 Gaussian-process fields (Matern nu = 1.5, length
scale 0.2) on a 64 x 64 grid plus noise; covariance smoothed on the 64^4 =
16,777,216-node grid (h = 0.1, FP32 moments, FP64 per-node solve);
randomized eigendecomposition with k = 20, oversampling 10, 2 power
iterations.

One step = the whole hot path on that input, resident in HBM:
  bin (mean) -> smooth mean -> bin (covariance Gram product) -> smooth
  covariance -> randomized eigendecomposition.
value = 64^4 covariance nodes / step time (grid points per second).

Prints one JSON line (see the keys below). The CPU baseline is the FP64
oracle's direct-window smoother timed on a bounded random sample of the same
64^4 nodes on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFS = 2500.0  # dense BF16 matrix peak of one MI355X
FP64_PEAK_TFS = 78.6  # FP64 vector peak of one MI355X


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "c3_64x64_smooth_cov_hbm_traffic.md")
SMOOTHER_SOURCES = ("paper_1510_04439_amd/csrc/smooth_fused.hip", "paper_1510_04439_amd/csrc/wls.hpp")


def measured_traffic():
    """HBM bytes per fpca_smooth_cov call from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when the
    smoother's sources changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m_t = re.search(r"^traffic_bytes_per_call: (\d+)$", text, re.M)
    m_h = re.search(r"^source_sha256: ([0-9a-f]{64})$", text, re.M)
    if not (m_t and m_h):
        return None
    h = hashlib.sha256()
    for f in SMOOTHER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return int(m_t.group(1)) if h.hexdigest() == m_h.group(1) else None


def cpu_baseline(ds, G_host: np.ndarray, budget_s: float = 15.0):
    """The oracle (never tuned for this) on a bounded sample of the covariance
    nodes: direct-window FP64 local-linear smoother of the raw surface."""
    import oracle
    P = int(np.prod(ds.M_cov))
    C = np.full((P, P), 1.0)
    np.fill_diagonal(C, 0.0)
    rng = np.random.default_rng(5)
    m = 64
    t_used = 0.0
    done = 0
    while t_used < budget_s and done < 200_000:
        nodes = rng.integers(0, P * P, m)
        t0 = time.perf_counter()
        oracle.smooth_cov_raw(ds.M_cov, ds.h_cov, C, G_host, nodes)
        dt = time.perf_counter() - t0
        t_used += dt
        done += m
        if dt < budget_s / 8:
            m *= 2
    return {"value": done / t_used, "unit": "smoothed cov grid pts/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{done} random nodes of the 64^4 covariance grid, direct-window FP64 smoother "
                      f"of the raw surface (binning and eigendecomposition not included), {t_used:.1f} s"}


def hselect_timing(h, torch, n_datasets: int = 5):
    """Bandwidth selection on held-out d=2 irregular datasets of the surrogate
    family (32x32 grid, 16 bandwidths x 5 folds): the trained surrogate
    (features + MLP) against batched CV, both after the shared binning."""
    from paper_1510_04439_amd import surrogate as S
    from fpca_synth import make_surrogate_dataset
    if not os.path.exists(S.MODEL_PATH):
        return None
    log("bandwidth selection: surrogate vs batched CV")
    model = S.Surrogate.load()
    rows = []
    for i in range(n_datasets):
        ds = make_surrogate_dataset(i, "test")
        bd = S.bin_dataset(h, ds)
        S.cv_scores(h, bd, S.H_GRID[:1])  # warm the smoother's scratch
        model.select(h, bd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hs, fb = model.select(h, bd)
        torch.cuda.synchronize()
        t_sur = time.perf_counter() - t0
        t0 = time.perf_counter()
        sc = S.cv_scores(h, bd, S.H_GRID)
        t_cv = time.perf_counter() - t0
        s_sur = float(S.cv_scores(h, bd, [hs])[0])
        rows.append((t_sur, t_cv, s_sur / float(sc.min()), fb))
    t_sur = float(np.median([r[0] for r in rows]))
    t_cv = float(np.median([r[1] for r in rows]))
    return {"surrogate_ms": t_sur * 1e3, "batched_cv_ms": t_cv * 1e3, "speedup": t_cv / t_sur,
            "cv_score_ratio_max": float(max(r[2] for r in rows)), "fallbacks": int(sum(r[3] for r in rows)),
            "datasets": n_datasets, "jobs_per_cv": len(S.H_GRID) * S.N_FOLDS}


def cv_d3_timing(h, torch, F):
    """Batched CV on the d=3 disk x time workload: n=800 curves, 16^3 grid with
    the domain mask, covariance on 16^6 = 16.8M nodes (7x7 per-node systems),
    16 bandwidths x 5 leave-curves-out folds (80 smoother jobs)."""
    from fpca_synth import make_c4
    log("batched CV, d=3 (16 bandwidths x 5 folds on 16^6 nodes)")
    ds = make_c4()
    P = int(np.prod(ds.M_cov))
    dev = "cuda:0"
    off = torch.from_numpy(ds.offsets).to(dev)
    t = torch.from_numpy(ds.t).to(dev)
    y = torch.from_numpy(ds.y).to(dev)
    folds = torch.from_numpy(ds.folds).to(dev)
    mask = torch.from_numpy(ds.mask).to(dev)
    grid = F.Grid(ds.M_cov, mask)
    C, G, Q = (torch.empty(ds.n_folds + 1, P, P, dtype=torch.float32, device=dev) for _ in range(3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fpca_bin(h, grid, F.FPCA_BIN_COV, F.FPCA_IRREGULAR, F.FPCA_F32, F.FPCA_PREC_F32, ds.n, off, t, y, folds,
               ds.n_folds, C, G, Q)
    torch.cuda.synchronize()
    t_bin = time.perf_counter() - t0
    data = [(grid, C, G, Q)]
    t0 = time.perf_counter()
    F.fpca_cv_batched(h, F.FPCA_F32, data, ds.n_folds, ds.h_grid)  # tile-shape tuning, then an eager run
    t_first = time.perf_counter() - t0
    F.fpca_cv_batched(h, F.FPCA_F32, data, ds.n_folds, ds.h_grid)  # captured into a graph
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        sc = F.fpca_cv_batched(h, F.FPCA_F32, data, ds.n_folds, ds.h_grid)[0]  # graph replay
        times.append(time.perf_counter() - t0)
    t_cv = float(np.median(times))
    tot = sc.sum(1)
    return {"bin_ms": t_bin * 1e3, "cv_ms": t_cv * 1e3, "first_call_ms": t_first * 1e3, "jobs": int(sc.size),
            "nodes_per_job": P * P, "h_best": float(ds.h_grid[int(np.argmin(tot))]),
            "h_select": float(F.fpca_cv_select(ds.h_grid, tot)[0]),
            "node_solves_per_s": sc.size * P * P / t_cv}


def fits_timing(h, torch, F):
    """The whole hot path (bin mean, smooth mean, bin pairs, smooth covariance,
    randomized eig) on the other two FPCA workloads: d=1 FP64 curves (mean grid
    101, covariance 51 x 51) and d=2 irregular FP32 surfaces (32^2 grid,
    covariance 32^4 nodes); median of 5 fits after a warm-up."""
    from fpca_synth import make_c1, make_c2
    from paper_1510_04439_amd import pipeline as PL
    log("end-to-end fits, d=1 and d=2 irregular")
    res = {}
    for name, ds in (("d1_fp64_101_51", make_c1()), ("d2_irregular_32x32", make_c2())):
        dd = PL.to_device(ds)
        bufs = PL.alloc(dd, ds.k)
        args = (ds.h_mean, ds.h_cov, ds.k, ds.oversample, ds.power_iters, ds.rp_seed)
        PL.fit(h, dd, bufs, *args)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            PL.fit(h, dd, bufs, *args)  # returns after the eigenvalues reached the host
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        P = int(np.prod(ds.M_cov))
        res[name] = {"fit_ms": float(np.median(ts)) * 1e3, "observations": int(len(ds.y)) if ds.t is not None else int(ds.y.size),
                     "curves": ds.n, "cov_nodes": P * P, "evals_top3": [float(v) for v in bufs.evals[:3]]}
    return res


def f2_timing(h, torch, F):
    """Simulation II's shape (d=3, 64^3 grid, n=100 complete curves, h=0.1):
    the smoothed covariance on 64^6 = 6.9e10 nodes (275 GB in FP32) is never
    stored; the randomized eigendecomposition takes its products through the
    covariance operator. The band part is recomputed in every product
    (FPCA_COVOP_RECOMPUTE) and, as the alternative, kept as band blocks."""
    from fpca_synth import make_sim2, sim2_eigfun, grid_points
    log("covariance operator, d=3 64^3 (Simulation II shape)")
    M, hb, k, over, q = 64, 0.1, 4, 12, 2
    ds = make_sim2(M=M)
    P = M ** 3
    dev = "cuda:0"
    g = F.Grid((M, M, M))
    Y = torch.from_numpy(ds.y).to(dev)
    c = torch.empty(P, dtype=torch.float64, device=dev)
    s = torch.empty_like(c)
    mu = torch.empty_like(c)
    F.fpca_bin(h, g, F.FPCA_BIN_MEAN, F.FPCA_COMMON_GRID, F.FPCA_F64, F.FPCA_PREC_F64, ds.n, None, None, Y, None, 0,
               c, s)
    F.fpca_smooth_mean(h, g, F.FPCA_F64, c, s, F.FPCA_K_EPANECHNIKOV, hb, mu)
    h.sync()
    R = int(np.floor(hb * (M - 1)))
    band_1d = sum(min(x + 2 * R, M - 1) - max(x - 2 * R, 0) + 1 for x in range(M))
    band_pairs = band_1d ** 3
    r = k + over
    X = torch.randn(P, r, dtype=torch.float64, device=dev)
    out = torch.empty(P, r, dtype=torch.float64, device=dev)
    res = {"workload": "d=3 complete curves on 64^3, n=100, h=0.1 (13 taps per coordinate), k=4, r=16, q=2",
           "cov_nodes": P * P, "band_pairs": band_pairs}

    def timed(fn, reps=1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    pts = grid_points((M, M, M))
    w = 1.0 / (M - 1) ** 3

    def quality(ev, ef):
        phi = ef.cpu().numpy()
        ise = []
        for l in range(1, 5):
            tru = sim2_eigfun(l, pts)
            tru = tru / np.sqrt(w * (tru ** 2).sum())
            e = phi[l - 1]
            sg = np.sign((e * tru).sum())
            ise.append(float(w * ((sg * e - tru) ** 2).sum()))
        return {"evals": [float(v) for v in ev], "ise_phi": ise}

    op = F.CovOp(h, g, Y, mu, hb, F.FPCA_COVOP_RECOMPUTE)
    try:
        op.apply(X, out)
        t_apply = timed(lambda: op.apply(X, out), 2)
        ef = torch.empty(k, P, dtype=torch.float64, device=dev)
        evh = {}
        t_eig = timed(lambda: evh.update(v=op.eig(None, k, over, q, 7, ef)))
        res["recompute"] = {"apply_ms": t_apply, "eig_ms": t_eig, **quality(evh["v"][0], ef)}
    finally:
        op.close()
    flops = band_pairs * 2.0 * 7 * ds.n
    res["roofline"] = {"bound": "fp64", "kernel": "k_band<3> (one product, r=16)",
                       "alg_flops_per_band_pair": 2 * 7 * ds.n, "achieved": flops / (t_apply * 1e-3) / 1e12,
                       "peak": 78.6, "unit": "TFLOP/s", "frac": flops / (t_apply * 1e-3) / 1e12 / 78.6}
    free, _ = torch.cuda.mem_get_info()
    if free > (64 << 30):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = F.CovOp(h, g, Y, mu, hb, F.FPCA_COVOP_STORE_BAND)
        torch.cuda.synchronize()
        t_create = (time.perf_counter() - t0) * 1e3
        try:
            op.apply(X, out)
            t_apply2 = timed(lambda: op.apply(X, out), 3)
            ef = torch.empty(k, P, dtype=torch.float64, device=dev)
            evh = {}
            t_eig2 = timed(lambda: evh.update(v=op.eig(None, k, over, q, 7, ef)))
            res["stored_band"] = {"create_ms": t_create, "apply_ms": t_apply2, "eig_ms": t_eig2,
                                  **quality(evh["v"][0], ef)}
        finally:
            op.close()
    res["lambda_true"] = [4.0 ** (3 - l) / 512 for l in range(1, 5)]
    return res


def f1_timing(h, torch, F, dd, ds, b):
    """Noise variance (eq. 2.6), PACE scores (eq. 2.7) and the reconstruction on
    the grid for the benchmark workload, from one step's smoothed mean,
    covariance and eigenpairs (not part of the timed step)."""
    log("noise variance, PACE scores and reconstruction")
    P, n, k = dd.grid_cov.P, dd.n, ds.k
    z = lambda *sh: torch.empty(*sh, dtype=dd.tdtype, device="cuda:0")
    c2, s2, sq, b0 = z(P), z(P), z(P), z(P)
    scores, xhat = z(n * k), z(n * P)
    res = {}

    def legs(ev=None):
        cur = torch.cuda.current_stream()
        if ev: ev[0].record(cur)
        F.fpca_bin(h, dd.grid_cov, F.FPCA_BIN_MEAN, dd.design, dd.dtype, F.FPCA_PREC_F32, n, None, None, dd.y,
                   None, 0, c2, s2, sq)
        F.fpca_smooth_mean(h, dd.grid_cov, dd.dtype, c2, sq, F.FPCA_K_EPANECHNIKOV, ds.h_mean, b0)
        if ev: ev[1].record(cur)
        res["sigma2"], _ = F.fpca_noise_variance(h, dd.grid_cov, dd.dtype, b0, b.mu, b.gamma, None)
        if ev: ev[2].record(cur)
        F.fpca_pace_scores(h, dd.grid_cov, F.FPCA_COMMON_GRID, dd.dtype, n, None, None, dd.y, b.mu, b.efuns, k,
                           b.evals, res["sigma2"], scores)
        if ev: ev[3].record(cur)
        F.fpca_reconstruct(h, dd.dtype, P, n, k, b.mu, b.efuns, scores, xhat)
        if ev: ev[4].record(cur)

    legs()
    reps = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(3)]
    for ev in reps:
        legs(ev)
    torch.cuda.synchronize()
    med = lambda a, c: float(np.median([ev[a].elapsed_time(ev[c]) for ev in reps]))
    rc_ms = med(3, 4)
    rc_bytes = 4.0 * (n * P + P * (k + 1) + n * k)
    pace_ms = med(2, 3)
    # every curve of this workload is complete: the kernel forms Phi^T (Y - mu)
    # per curve (2 n P k flop) against one shared factor, streaming Y once
    pace_flop = 2.0 * n * P * k
    pace_bytes = 4.0 * (n * P + P * (k + 1) + n * k)
    return {"sigma2": res["sigma2"], "k": k,
            "ms": {"bin_sq+smooth_b0": med(0, 1), "noise_variance": med(1, 2), "pace_scores": pace_ms,
                   "reconstruct": rc_ms},
            "pace_roofline": {"bound": "hbm", "alg_bytes": pace_bytes,
                              "achieved": pace_bytes / (pace_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": pace_bytes / (pace_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                              "alg_flop": pace_flop, "flop_frac_fp64": pace_flop / (pace_ms / 1e3) / 1e12 / FP64_PEAK_TFS},
            "reconstruct_roofline": {"bound": "hbm", "alg_bytes": rc_bytes,
                                     "achieved": rc_bytes / (rc_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": rc_bytes / (rc_ms / 1e3) / 1e9 / HBM_PEAK_GBS}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cv-d3", action="store_true", help="skip the d=3 batched-CV timing")
    ap.add_argument("--no-hselect", action="store_true", help="skip the surrogate-versus-CV timing")
    ap.add_argument("--no-f1", action="store_true", help="skip the noise-variance, PACE and reconstruction timing")
    ap.add_argument("--no-f2", action="store_true", help="skip the covariance-operator (64^3) timing")
    ap.add_argument("--no-fits", action="store_true", help="skip the d=1 and d=2 irregular end-to-end fits")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--eig-cus", type=int, default=0,
                    help="CUs of the pipelined steps' eigendecomposition streams (0: a quarter of the chip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the reference for HBM byte counters)")
    ap.add_argument("--gram-prec", choices=["bf16x3", "f32"], default="bf16x3",
                    help="precision of the binning Gram product (bf16 hi/lo x3 with FP32 accumulation, or FP32)")
    ap.add_argument("--panel-prec", choices=["bf16x3", "f32"], default="bf16x3",
                    help="precision of the range finder's products of the covariance with the basis")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)
        return
    import paper_1510_04439_amd as F
    from paper_1510_04439_amd import pipeline as PL
    from fpca_synth import make_c3

    assert torch.cuda.is_available()
    log("generating the 64x64 common-grid workload")
    ds = make_c3(n=args.n)
    assert tuple(ds.M_mean) == tuple(ds.M_cov), "the one-pass binning needs the mean on the covariance grid"
    P = int(np.prod(ds.M_cov))
    nodes = P * P
    dd = PL.to_device(ds)
    # two handles (own scratch), two buffer sets and two streams (default
    # priority): the timed steps alternate between them so that the binning
    # and smoothing of step i+1 run beside the eigendecomposition of step i
    hs = [F.Handle(0), F.Handle(0)]
    h = hs[0]
    bl = [PL.alloc(dd, ds.k, with_status=True, analytic_C=True) for _ in range(2)]
    bufs = bl[0]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    # The pipelined steps split the chip: binning and smoothing on the lower
    # three quarters of the CU mask, the latency-bound eigendecomposition on
    # the top quarter (64 of 256 CUs, 8 per XCD: 0.88 against 0.95 ms per step
    # unsplit; 32 or 96 CUs for it measured 1.25 and 0.97 ms). Plain streams
    # when the runtime refuses the masks.
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    eig_cus = args.eig_cus if args.eig_cus > 0 else max(32, (ncu // 4) // 32 * 32)
    raw_streams = []
    try:
        for lo, hi in ((0, ncu - eig_cus), (0, ncu - eig_cus), (ncu - eig_cus, ncu), (ncu - eig_cus, ncu)):
            raw_streams.append(F.fpca_stream_create_cu_range(0, lo, hi))
        s_stage = [torch.cuda.ExternalStream(r) for r in raw_streams[:2]]
        s_eig = [torch.cuda.ExternalStream(r) for r in raw_streams[2:]]
        split = f"binning and smoothing on CUs [0, {ncu - eig_cus}), eigendecomposition on [{ncu - eig_cus}, {ncu})"
    except F.FpcaError:
        for r in raw_streams:
            F.fpca_stream_destroy(r)
        raw_streams = []
        s_stage = s_eig = streams
        split = "one stream per step slot (CU masks refused)"
    step_done = [torch.cuda.Event(), torch.cuda.Event()]
    gram_prec = F.FPCA_PREC_BF16X3 if args.gram_prec == "bf16x3" else F.FPCA_PREC_F32
    panel_prec = F.FPCA_PREC_BF16X3 if args.panel_prec == "bf16x3" else F.FPCA_PREC_F32

    def stages(slot, ev=None):
        """Binning and smoothing of one step on slot's handle, buffers and (current) stream;
        `ev`: timing events (created outside the timed loop) or None."""
        hh, b = hs[slot], bl[slot]
        cur = torch.cuda.current_stream()
        if ev: ev[0].record(cur)
        # both binnings in one pass over the curves (the mean's grid is the covariance's)
        F.fpca_bin_common(hh, dd.grid_cov, dd.dtype, gram_prec, dd.n, dd.y, b.c, b.s, None, None, b.G)
        if ev: ev[1].record(cur)
        F.fpca_smooth_mean(hh, dd.grid_mean, dd.dtype, b.c, b.s, F.FPCA_K_EPANECHNIKOV, ds.h_mean,
                           b.mu, b.mu_status)
        if ev: ev[2].record(cur)
        F.fpca_smooth_cov(hh, dd.grid_cov, dd.dtype, None, PL.uniform_pair_weight(dd), b.G, b.mu,
                          F.FPCA_K_EPANECHNIKOV, ds.h_cov, b.gamma, b.status)
        if ev: ev[3].record(cur)

    def eig(slot, ev=None):
        hh, b = hs[slot], bl[slot]
        b.evals, b.fve = F.fpca_eig_randomized(hh, dd.dtype, panel_prec, dd.grid_cov, b.gamma, None, ds.k,
                                               ds.oversample, ds.power_iters, ds.rp_seed, b.efuns)
        if ev: ev[4].record(torch.cuda.current_stream())

    def run(nsteps):
        """nsteps pipelined steps: step i+1's binning and smoothing are queued before step i's
        eigendecomposition, on the other slot's handle, buffers and streams; a step's
        eigendecomposition waits for its own smoothing (an event between the two streams)."""
        def stage_part(slot):
            with torch.cuda.stream(s_stage[slot]):
                stages(slot)
                step_done[slot].record(s_stage[slot])
        stage_part(0)
        for i in range(nsteps):
            if i + 1 < nsteps:
                stage_part((i + 1) % 2)
            with torch.cuda.stream(s_eig[i % 2]):
                s_eig[i % 2].wait_event(step_done[i % 2])
                eig(i % 2)  # returns after this step's eigenvalues reached the host

    log("warmup")
    with torch.cuda.stream(streams[0]):
        for _ in range(max(args.warmup, 1)):
            stages(0)
            eig(0)
    torch.cuda.synchronize()
    # per-step latency and stage times: the same steps one after another on one stream
    log("sequential steps (latency and stage times)")
    nseq = min(args.steps, 10)
    recs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(nseq)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    with torch.cuda.stream(streams[0]):
        for i in range(nseq):
            stages(0, recs[i])
            eig(0, recs[i])
    torch.cuda.synchronize()
    latency_ms = (time.perf_counter() - t1) * 1e3 / nseq
    log("timed steps")
    run(2 * max(args.warmup, 1))  # pipelined warm-up (both slots, the streams of the pipeline)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for hh in hs:
        hh.sync()
    stages_ = {"bin_mean+bin_cov": [], "smooth_mean": [], "smooth_cov": [], "eig": []}
    for ev in recs:
        stages_["bin_mean+bin_cov"].append(ev[0].elapsed_time(ev[1]))
        stages_["smooth_mean"].append(ev[1].elapsed_time(ev[2]))
        stages_["smooth_cov"].append(ev[2].elapsed_time(ev[3]))
        stages_["eig"].append(ev[3].elapsed_time(ev[4]))
    stage_ms = {k: float(np.median(v)) for k, v in stages_.items()}
    ms_per_step = wall * 1e3 / args.steps
    value = nodes / (ms_per_step / 1e3)
    sc_ms = stage_ms["smooth_cov"]
    # the Gram product Y^T Y of the covariance binning: the symmetric product
    # has P (P + 1) / 2 distinct entries of 2 n flop each; the kernel runs
    # three BF16 products on every 128 x 128 tile on or above the diagonal
    Pc = int(np.prod(ds.M_cov))
    gram_flops = 1.0 * args.n * Pc * (Pc + 1)
    nt = (Pc + 127) // 128
    gram_mfma_flops = 3.0 * 2.0 * args.n * 128 * 128 * nt * (nt + 1) / 2
    alg_bytes = 12.0 * nodes  # read C and G, write gamma: 4 B each per node
    alg_bytes_min = 8.0 * nodes  # C is analytic on the complete grid: read G, write gamma
    achieved = alg_bytes / (sc_ms / 1e3) / 1e9
    out = {
        "metric": "smoothed cov grid pts/s (d=2, 64^4) + HBM GB/s frac; h-select time vs batched CV",
        "value": value,
        "unit": "smoothed cov grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 per-node solve and Rayleigh-Ritz)",
        "data": "synthetic",
        "config": {"workload": "d=2 common grid 64x64, n=%d Matern-1.5 GP fields, cov 64^4 nodes, h=0.1, "
                               "randomized eig k=20 p=10 q=2" % args.n,
                   "n": args.n, "grid": [64, 64], "cov_nodes": nodes, "h": ds.h_cov,
                   "gram_prec": args.gram_prec, "panel_prec": args.panel_prec},
        "stages_ms": stage_ms,
        "latency_ms_per_step": latency_ms,
        "pipelining": "steps alternate over two handles and buffer sets; step i+1's binning and smoothing run "
                      "beside step i's eigendecomposition, " + split + " (stages_ms and latency from sequential "
                      "steps on one unrestricted stream)",
        "smooth_cov_pts_per_s": nodes / (sc_ms / 1e3),
        "roofline": {"bound": "hbm", "kernel": "fpca_smooth_cov (k_tables, k_stage_t, k_stage_s)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "alg_bytes_per_node": 12,
                     "frac_at_8_bytes_per_node": alg_bytes_min / (sc_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "roofline_gram": {"bound": "mfma",
                          "kernel": "fpca_bin_common (k_split_t with the mean's column sums, k_syrk_bf16x3, "
                                    "k_syrk_fixup, k_colsum_finish)",
                          "achieved": gram_flops / (stage_ms["bin_mean+bin_cov"] / 1e3) / 1e12,
                          "peak": BF16_PEAK_TFS, "unit": "TFLOP/s",
                          "frac": gram_flops / (stage_ms["bin_mean+bin_cov"] / 1e3) / 1e12 / BF16_PEAK_TFS,
                          "alg_flops": gram_flops, "mfma_flops": gram_mfma_flops,
                          "mfma_issue_frac": gram_mfma_flops / (stage_ms["bin_mean+bin_cov"] / 1e3) / 1e12
                          / BF16_PEAK_TFS},
        "evals_top3": [float(v) for v in bufs.evals[:3]],
    }
    out["f1"] = None if args.no_f1 else f1_timing(h, torch, F, dd, ds, bufs)
    out["hselect"] = None if args.no_hselect else hselect_timing(h, torch)
    if not args.no_cv_d3:
        out["cv_d3"] = cv_d3_timing(h, torch, F)
    out["f2"] = None if args.no_f2 else f2_timing(h, torch, F)
    out["fits"] = None if args.no_fits else fits_timing(h, torch, F)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        G_host = bufs.G.cpu().numpy().astype(np.float64)
        out["cpu_baseline"] = cpu_baseline(ds, G_host, args.cpu_budget)
    torch.cuda.synchronize()
    for r in raw_streams:
        F.fpca_stream_destroy(r)
    for hh in hs:
        hh.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

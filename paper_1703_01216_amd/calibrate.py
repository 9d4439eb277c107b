"""Fine-tuning of the alpha predictor for one geometry, on the GPU.

    from paper_1703_01216_amd import calibrate
    cal = calibrate.fine_tune(ctx, Fs, deltas)      # ctx holds the trained network
    opts = fr3d.default_opts(use_predictor=1, seed_slope=cal["seed_slope"], seed_snap_lo=cal["seed_snap_lo"],
                             seed_slope_ratio=cal["seed_slope_ratio"])

The predictor is trained on a mix of grids, source sets and heights of Y
(the training workload); on one fixed geometry its seeds carry an error that
depends on the data's spectrum.  Given instances of that geometry (other
draws than the ones to be solved), this continues the network's training on
them with the library's own kernels (BF16 matrix-core forward and backward,
Adam), so the seed becomes the network's, with no other model beside it:

* labels: each instance's root t* = log10 alpha with |r/delta - 1| <=
  label_tol, found by the library's learned search from the network's seed
  (instances without a root in the range are labelled at the range end, as
  in training);
* the network is fine-tuned on the first part of the instances (full batch,
  `steps` Adam steps at learning rate `lr`, fresh moments);
* the rest are held out: the standard deviation of the fine-tuned seed's
  error on them sets seed_snap_lo = SNAP_SIGMAS sigma (a seed closer than that
  to the lower end of the range starts the search at that end, where an
  instance whose root lies below the range ends after one evaluation);
* seed_slope, the slope of ln r per decade of alpha that the first secant
  step assumes, is the median over the instances of the one-sided
  difference (ln r(t* + h) - ln delta)/h at the root;
* seed_slope_ratio, the factor from the slope of the whole-box residual
  (which each seed evaluation forms exactly) to that of the residual on Y,
  is the median over the instances of the ratio of the two one-sided
  differences at the root (the whole-box residual from the library's
  diagnostics).

Everything runs through the library's calls; the host only forms medians
and standard deviations of the values they return.
"""
from __future__ import annotations

import math
import time

SNAP_SIGMAS = 2.0


def split(m, hold):
    """Indices of the fitted and held-out instances: the last round(hold m)
    (at least one) are held out."""
    k = max(1, min(m - 1, int(round(hold * m))))
    return list(range(m - k)), list(range(m - k, m))


def median(v):
    v = sorted(v)
    if not v:
        raise ValueError("median of nothing")
    k = len(v) // 2
    return v[k] if len(v) % 2 else 0.5 * (v[k - 1] + v[k])


def std(v):
    mu = sum(v) / len(v)
    return math.sqrt(sum((x - mu) ** 2 for x in v) / len(v))


def fine_tune(ctx, Fs, deltas, lr=1e-3, steps=100, hold=0.25, h=0.05, label_tol=1e-5, lo=-8.0, hi=0.0,
              start_slope=0.05):
    import numpy as np
    import torch

    t_start = time.perf_counter()
    m = len(Fs)
    fit_idx, held_idx = split(m, hold)
    zs = [torch.empty_like(F) for F in Fs]
    feat = torch.empty((m, 65), dtype=torch.float32, device=Fs[0].device)
    ctx.predictor_set_calibration(None)
    reps = ctx.solve_batch(Fs, deltas, zs, feat=feat, use_predictor=1, tol=label_tol, accept_lo=1 - label_tol,
                           accept_hi=1 + label_tol, seed_slope=start_slope, max_steps=60,
                           log10_alpha_lo=lo, log10_alpha_hi=hi)
    t = [min(max(math.log10(r["alpha"]), lo), hi) for r in reps]
    root = [(r["flags"] & 7) == 0 for r in reps]
    label_evals = sum(r["n_evals"] for r in reps)
    # slope of ln r at the root, one-sided over h decades
    slopes, ratios = [], []
    z = zs[0]
    ctx.set_diagnostics(True)
    try:
        for i in range(m):
            if not root[i] or t[i] + h > hi:
                continue
            ctx.set_data(Fs[i], deltas[i])
            r1 = ctx.solve_alpha(10.0 ** (t[i] + h), z)
            r0 = ctx.solve_alpha(10.0 ** t[i], z)
            s = (math.log(r1["residual"]) - math.log(deltas[i])) / h
            sf = (math.log(r1["residual_full_box"]) - math.log(r0["residual_full_box"])) / h
            if s > 0:
                slopes.append(s)
                if sf > 0:
                    ratios.append(s / sf)
    finally:
        ctx.set_diagnostics(False)
    # fine-tune on the fitted part (fresh Adam moments)
    params, norm = ctx.predictor_get()
    ctx.predictor_set(params, norm)
    X = feat[fit_idx].contiguous()
    tt = torch.tensor(np.array([t[i] for i in fit_idx], dtype=np.float32), device=feat.device)
    for _ in range(steps):
        ctx.predictor_train_step(X, tt, lr)
    # held-out error of the fine-tuned seed
    y = torch.empty(len(held_idx), dtype=torch.float32, device=feat.device)
    ctx.predictor_forward(feat[held_idx].contiguous(), y)
    yh = y.cpu().numpy().astype(np.float64)
    err = [min(max(float(yh[k]), lo), hi) - t[i] for k, i in enumerate(held_idx) if root[i]]
    sigma = std(err) if len(err) >= 2 else 0.0
    torch.cuda.synchronize()
    return dict(seed_slope=median(slopes), seed_snap_lo=SNAP_SIGMAS * sigma,
                seed_slope_ratio=median(ratios) if ratios else 0.0,
                slope_ratio_spread=(std(ratios) / median(ratios)) if len(ratios) >= 2 else 0.0,
                instances=m, fitted=len(fit_idx),
                held_out=len(held_idx), held_out_err_std_decades=sigma,
                held_out_err_mean_decades=(sum(err) / len(err)) if err else 0.0,
                slope_instances=len(slopes), label_evals=label_evals, lr=lr, steps=steps,
                seconds=time.perf_counter() - t_start)

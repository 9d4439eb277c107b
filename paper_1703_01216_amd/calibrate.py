"""Calibration of the learned seed for one geometry.

    from paper_1703_01216_amd import calibrate
    cal = calibrate.seed_calibration(ctx, Fs, deltas)
    ctx.predictor_set_calibration(cal["coef"])
    opts = fr3d.default_opts(use_predictor=1, seed_slope=cal["seed_slope"], seed_slope_x=cal["seed_slope_x"],
                             seed_snap_lo=cal["seed_snap_lo"])

The predictor is trained on a mix of grids, source sets and heights of Y; on
one fixed geometry its seeds carry an error that depends on the data's
spectrum, and the secant refinement of the seeded search wants the slope of
ln r at the root.  Given calibration instances of that geometry (other
draws than the ones to be solved), this fits

    t* - t_net  ~  c_0 + sum_k c_k x_k          (ridge regression, lambda = 1 on
                                                 standardised features),
    log10 s*    ~  log10 slope + slope_x x_64    (least squares),

with t* = log10 alpha of the plain rule to |r/delta - 1| <= 1e-6, s* the
slope d ln r / d log10 alpha at t* (central difference over +-h decades),
t_net the network's output and x the 65 raw features (x_64 = log10(delta/
||F||)); instances without a root in the range are skipped.  coef holds
c_0 and the c_k for the raw features (the library's
fr3d_predictor_set_calibration).  seed_snap_lo = SNAP_SIGMAS times the
standard deviation of the shift's residual: a calibrated seed closer than
that to the lower end of the range is about as likely to have its root
below the range (the network was trained with such instances labelled at
the range end), so the search starts at the end, where such an instance
ends after one evaluation.  Everything runs through the library's calls.
"""
from __future__ import annotations

import math

RIDGE = 1.0
SNAP_SIGMAS = 2.0


def seed_calibration(ctx, Fs, deltas, h=0.05, lo=-8.0, hi=0.0):
    import numpy as np
    import torch

    X, dt, ls = [], [], []
    z = torch.empty_like(Fs[0])
    y = torch.empty(1, dtype=torch.float32, device=Fs[0].device)
    ctx.predictor_set_calibration(None)
    for F, d in zip(Fs, deltas):
        ctx.set_data(F, d)
        feat, _ = ctx.get_features()
        ctx.predictor_forward(feat.view(1, 65).contiguous(), y)
        t_net = float(y[0])
        rep = ctx.solve_discrepancy(z, tol=1e-6, max_steps=60, log10_alpha_lo=lo, log10_alpha_hi=hi)
        if rep["flags"] != 0:
            continue
        t = math.log10(rep["alpha"])
        rp = ctx.solve_alpha(10.0 ** (t + h), z)["residual"]
        rm = ctx.solve_alpha(10.0 ** (t - h), z)["residual"]
        s = (math.log(rp) - math.log(rm)) / (2 * h)
        if s > 0:
            X.append(feat.double().cpu().numpy())
            dt.append(t - t_net)
            ls.append(math.log10(s))
    if len(X) < 3:
        raise RuntimeError("too few calibration instances with a root in the range")
    return fit(np.array(X), np.array(dt), np.array(ls))


def fit(X, dt, ls, ridge=RIDGE):
    """The least-squares fits on calibration rows: X [m][65] raw features,
    dt = t* - t_net, ls = log10 s*.  Returns the raw-feature coefficients of
    the seed shift (ridge on standardised features; constant features get
    no weight) and the power law of the slope in x_64."""
    import numpy as np

    X, dt, ls = np.asarray(X, dtype=np.float64), np.asarray(dt, dtype=np.float64), np.asarray(ls, dtype=np.float64)
    mu, sd = X.mean(0), X.std(0)
    live = sd > 1e-9
    Z = np.zeros_like(X)
    Z[:, live] = (X[:, live] - mu[live]) / sd[live]
    A = np.c_[np.ones(len(X)), Z]
    reg = ridge * np.eye(A.shape[1])
    reg[0, 0] = 0.0
    w = np.linalg.solve(A.T @ A + reg, A.T @ dt)
    coef = np.zeros(X.shape[1] + 1)
    coef[1:][live] = w[1:][live] / sd[live]
    coef[0] = w[0] - float(np.sum(coef[1:][live] * mu[live]))
    B = np.c_[np.ones(len(X)), X[:, 64]]
    sl = np.linalg.lstsq(B, ls, rcond=None)[0]
    res = float(np.std(dt - A @ w))
    return dict(coef=coef.tolist(), seed_slope=float(10.0 ** sl[0]), seed_slope_x=float(sl[1]),
                seed_snap_lo=SNAP_SIGMAS * res, instances=len(X), shift_residual_decades=res,
                slope_residual_log10=float(np.std(ls - B @ sl)))

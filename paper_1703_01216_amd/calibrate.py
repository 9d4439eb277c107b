"""Calibration of the learned seed for one geometry.

    from paper_1703_01216_amd import calibrate
    opts_fields = calibrate.seed_calibration(ctx, Fs, deltas)

The predictor is trained on a mix of grids, source sets and heights of Y; on
one fixed geometry its seeds carry a bias that depends on the noise level,
and the secant refinement of the seeded search wants the slope of ln r at
the root.  Given calibration instances of that geometry (other draws than
the ones to be solved), this fits by least squares

    t* - t_net  ~  shift + shift_x x_64,      log10 s*  ~  log10 slope + slope_x x_64,

with t* = log10 alpha of the plain rule to |r/delta - 1| <= 1e-6, s* the
slope d ln r / d log10 alpha at t* (central difference over +-h decades),
t_net the network's output and x_64 = log10(delta/||F||) the noise feature;
instances without a root in the range are skipped.  The result holds the
fr3d_dp_opts fields seed_shift, seed_shift_x, seed_slope, seed_slope_x.
Everything runs through the library's calls.
"""
from __future__ import annotations

import math


def seed_calibration(ctx, Fs, deltas, h=0.05, lo=-8.0, hi=0.0):
    import numpy as np
    import torch

    rows = []
    z = torch.empty_like(Fs[0])
    y = torch.empty(1, dtype=torch.float32, device=Fs[0].device)
    for F, d in zip(Fs, deltas):
        ctx.set_data(F, d)
        feat, _ = ctx.get_features()
        ctx.predictor_forward(feat.view(1, 65).contiguous(), y)
        t_net, x64 = float(y[0]), float(feat[64])
        rep = ctx.solve_discrepancy(z, tol=1e-6, max_steps=60, log10_alpha_lo=lo, log10_alpha_hi=hi)
        if rep["flags"] != 0:
            continue
        t = math.log10(rep["alpha"])
        rp = ctx.solve_alpha(10.0 ** (t + h), z)["residual"]
        rm = ctx.solve_alpha(10.0 ** (t - h), z)["residual"]
        s = (math.log(rp) - math.log(rm)) / (2 * h)
        if s > 0:
            rows.append((x64, t - t_net, math.log10(s)))
    if len(rows) < 3:
        raise RuntimeError("too few calibration instances with a root in the range")
    r = np.array(rows)
    A = np.c_[np.ones(len(r)), r[:, 0]]
    sh = np.linalg.lstsq(A, r[:, 1], rcond=None)[0]
    sl = np.linalg.lstsq(A, r[:, 2], rcond=None)[0]
    return dict(seed_shift=float(sh[0]), seed_shift_x=float(sh[1]), seed_slope=float(10.0 ** sl[0]),
                seed_slope_x=float(sl[1]), instances=len(rows),
                shift_residual_decades=float(np.std(r[:, 1] - A @ sh)),
                slope_residual_log10=float(np.std(r[:, 2] - A @ sl)))

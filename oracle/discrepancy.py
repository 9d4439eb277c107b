"""Choice of alpha by the discrepancy principle (Sec. 4, after Algorithm 1:
Tikhonov with the discrepancy principle or its generalisation keeps the
regularity conditions (12)-(13)).

Oracle (test infrastructure only).

Reading used (the paper cites the rule but does not write it out):

    rho(t) = r(10^t)^2 - (tau delta + h_op ||zeta(10^t)||)^2 - mu^2,
    target T(t) = sqrt((tau delta + h_op ||zeta||)^2 + mu^2),

tau = 1, h_op = mu = 0 is Morozov's principle.  r is the residual on Y.

Plain search (bisection in t = log10 alpha):
  evaluate t = hi;  |r/T - 1| <= tol -> stop, alpha = 10^hi;  rho < 0 -> stop, NOROOT_HIGH
  evaluate t = lo;  |r/T - 1| <= tol -> stop, alpha = 10^lo;  rho > 0 -> stop, NOROOT_LOW
  up to max_steps times: m = (lo + hi)/2, evaluate;
      |r/T - 1| <= tol -> stop, alpha = 10^m
      rho(m) < 0 -> lo = m, else hi = m
  otherwise alpha = 10^hi, MAXITER (re-evaluated there if hi was not the last point).

Seeded search (a predicted t0 from the alpha predictor):
  evaluate t0 (clipped to [lo, hi]); accept if acc_lo <= r/T <= acc_hi;
  otherwise step one decade at a time away from t0 in the direction rho
  points to (up if rho < 0), accepting any point inside the window, until
  rho changes sign (bracket found) or the range end is reached (NOROOT_*);
  then the plain bisection inside the bracket, whose ends are already known.
  PRED_FALLBACK is set whenever the first point is not accepted.
"""
from __future__ import annotations

import math

NOROOT_HIGH = 1
NOROOT_LOW = 2
MAXITER = 4
NAN_INPUT = 8
PRED_FALLBACK = 16


class _Counter:
    def __init__(self, evaluate, delta, tau, h_op, mu):
        self.evaluate = evaluate
        self.delta, self.tau, self.h_op, self.mu = delta, tau, h_op, mu
        self.n = 0
        self.last_t = None
        self.trace = []

    def __call__(self, t):
        r, zn = self.evaluate(10.0 ** t)
        self.n += 1
        self.last_t = t
        tgt2 = (self.tau * self.delta + self.h_op * zn) ** 2 + self.mu ** 2
        rho = r * r - tgt2
        ratio = r / math.sqrt(tgt2) if tgt2 > 0 else math.inf
        self.trace.append((t, r, zn, rho))
        return rho, ratio, r, zn


def _bisect(ev, a, b, max_steps, tol, flags):
    for _ in range(max_steps):
        m = 0.5 * (a + b)
        rho, ratio, r, zn = ev(m)
        if abs(ratio - 1.0) <= tol:
            return m, flags
        if rho < 0:
            a = m
        else:
            b = m
    if ev.last_t != b:
        ev(b)
    return b, flags | MAXITER


def bisection(evaluate, delta, lo=-8.0, hi=0.0, max_steps=40, tol=1e-3, tau=1.0, h_op=0.0, mu=0.0):
    """Plain search. ``evaluate(alpha_rel) -> (r_norm, zeta_norm)``.
    Returns dict(alpha, t, flags, n_evals, trace)."""
    ev = _Counter(evaluate, delta, tau, h_op, mu)
    rho, ratio, r, zn = ev(hi)
    if abs(ratio - 1.0) <= tol:
        return dict(alpha=10.0 ** hi, t=hi, flags=0, n_evals=ev.n, trace=ev.trace)
    if rho < 0:
        return dict(alpha=10.0 ** hi, t=hi, flags=NOROOT_HIGH, n_evals=ev.n, trace=ev.trace)
    rho, ratio, r, zn = ev(lo)
    if abs(ratio - 1.0) <= tol:
        return dict(alpha=10.0 ** lo, t=lo, flags=0, n_evals=ev.n, trace=ev.trace)
    if rho > 0:
        return dict(alpha=10.0 ** lo, t=lo, flags=NOROOT_LOW, n_evals=ev.n, trace=ev.trace)
    t, flags = _bisect(ev, lo, hi, max_steps, tol, 0)
    return dict(alpha=10.0 ** t, t=t, flags=flags, n_evals=ev.n, trace=ev.trace)


def seeded(evaluate, delta, t0, lo=-8.0, hi=0.0, max_steps=40, tol=1e-3, acc_lo=0.9, acc_hi=1.1,
           tau=1.0, h_op=0.0, mu=0.0):
    """Seeded search from a predicted log10 alpha ``t0``."""
    ev = _Counter(evaluate, delta, tau, h_op, mu)
    t = min(max(float(t0), lo), hi)
    rho, ratio, r, zn = ev(t)
    if acc_lo <= ratio <= acc_hi:
        return dict(alpha=10.0 ** t, t=t, flags=0, n_evals=ev.n, trace=ev.trace)
    flags = PRED_FALLBACK
    if rho < 0:          # residual below target: alpha too small, move up
        a = t
        while True:
            if a >= hi:
                return dict(alpha=10.0 ** hi, t=hi, flags=flags | NOROOT_HIGH, n_evals=ev.n, trace=ev.trace)
            tn = min(a + 1.0, hi)
            rho, ratio, r, zn = ev(tn)
            if acc_lo <= ratio <= acc_hi:
                return dict(alpha=10.0 ** tn, t=tn, flags=flags, n_evals=ev.n, trace=ev.trace)
            if rho >= 0:
                b = tn
                break
            a = tn
    else:                # residual above target: alpha too large, move down
        b = t
        while True:
            if b <= lo:
                return dict(alpha=10.0 ** lo, t=lo, flags=flags | NOROOT_LOW, n_evals=ev.n, trace=ev.trace)
            tn = max(b - 1.0, lo)
            rho, ratio, r, zn = ev(tn)
            if acc_lo <= ratio <= acc_hi:
                return dict(alpha=10.0 ** tn, t=tn, flags=flags, n_evals=ev.n, trace=ev.trace)
            if rho <= 0:
                a = tn
                break
            b = tn
    t, flags = _bisect(ev, a, b, max_steps, tol, flags)
    return dict(alpha=10.0 ** t, t=t, flags=flags, n_evals=ev.n, trace=ev.trace)

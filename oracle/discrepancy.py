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

Seeded search (a predicted t0 from the alpha predictor; not in the paper):
  a point is accepted when acc_lo <= r/T <= acc_hi or |r/T - 1| <= tol.
  Evaluate t0 (clipped to [lo, hi]).  Otherwise walk away from it in the
  direction rho points to (up if rho < 0) with steps walk, 2 walk, 4 walk, ...
  (clipped to the range; NOROOT_* when a range end is reached without a sign
  change) until rho changes sign, then regula falsi on g = r/T - 1 inside the
  bracket with the Illinois modification (the function value kept at an end
  that survives two steps in a row is halved), at most max_steps points;
  otherwise alpha = 10^b, MAXITER.  PRED_FALLBACK is set whenever the first
  point is not accepted.
  Secant refinement (``seeded_secant``): after the seed, steps on
  g = ln(r/T): the first with an assumed slope of g per decade, later ones
  through the last two points, regula falsi (Illinois) whenever a step would
  leave a known bracket; range ends and the step limit as above.  With a
  slope ratio c > 0 the assumed slope becomes c times the whole-box
  residual's slope d ln ||r_box|| / d log10 alpha at the seed, when that is
  positive (the residual on Y is a part of the whole-box one and its slope
  follows it closely on one geometry).

K-candidate search (K alphas per step, log-spaced in the current bracket; not
in the paper -- the batched form of the same rule):
  step 1 evaluates t_j = lo + j (hi - lo)/(K - 1), j = 0..K-1 (both range ends);
  later steps evaluate the K interior points t_j = a + (j + 1)(b - a)/(K + 1).
  After a step: the candidate with the smallest |r/T - 1| among those with
  |r/T - 1| <= tol (the lowest index on ties) is accepted.  Otherwise, in
  step 1, rho(hi) < 0 -> NOROOT_HIGH at hi and rho(lo) > 0 -> NOROOT_LOW at lo;
  then b is the first point (in increasing t, the old b last) with rho >= 0 and
  a the point before it (the old a first).  After max_steps steps the answer
  is b, MAXITER.  The answer is evaluated once more on its own (it is where
  zeta is written), so n_evals = K * steps + 1.
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


def _start(t0, lo, hi, snap):
    """First point of a seeded search: the seed clipped to [lo, hi]; a seed
    less than ``snap`` decades above lo starts at lo (for such a seed the
    root is often below the range, and then the point at lo ends the search
    at once)."""
    t = min(max(float(t0), lo), hi)
    return lo if t < lo + snap else t


def seeded(evaluate, delta, t0, lo=-8.0, hi=0.0, max_steps=40, tol=1e-3, acc_lo=0.9, acc_hi=1.1,
           tau=1.0, h_op=0.0, mu=0.0, walk=0.25, snap=0.0):
    """Seeded search from a predicted log10 alpha ``t0`` (first point as in
    ``_start``)."""
    ev = _Counter(evaluate, delta, tau, h_op, mu)

    def ok(ratio):
        return acc_lo <= ratio <= acc_hi or abs(ratio - 1.0) <= tol

    def out(t, flags):
        return dict(alpha=10.0 ** t, t=t, flags=flags, n_evals=ev.n, trace=ev.trace)

    t = _start(t0, lo, hi, snap)
    rho, ratio, r, zn = ev(t)
    if ok(ratio):
        return out(t, 0)
    flags = PRED_FALLBACK
    step = walk
    while True:                                   # walk to a sign change
        up = rho < 0                              # residual below target: alpha too small
        if up and t >= hi:
            return out(hi, flags | NOROOT_HIGH)
        if not up and t <= lo:
            return out(lo, flags | NOROOT_LOW)
        tn = min(t + step, hi) if up else max(t - step, lo)
        rn, ration, _, _ = ev(tn)
        if ok(ration):
            return out(tn, flags)
        if (up and rn >= 0) or (not up and rn <= 0):
            if up:
                a, ga, b, gb = t, ratio - 1.0, tn, ration - 1.0
            else:
                a, ga, b, gb = tn, ration - 1.0, t, ratio - 1.0
            break
        t, rho, ratio = tn, rn, ration
        step *= 2.0
    side = 0
    for _ in range(max_steps):                    # Illinois regula falsi, g(a) < 0 < g(b)
        m = b - gb * (b - a) / (gb - ga)
        rm, ratiom, _, _ = ev(m)
        if ok(ratiom):
            return out(m, flags)
        if rm < 0:
            a, ga = m, ratiom - 1.0
            if side == -1:
                gb *= 0.5
            side = -1
        else:
            b, gb = m, ratiom - 1.0
            if side == 1:
                ga *= 0.5
            side = 1
    if ev.last_t != b:
        ev(b)
    return out(b, flags | MAXITER)


def seeded_secant(evaluate, delta, t0, lo=-8.0, hi=0.0, max_steps=40, tol=1e-3, acc_lo=0.9, acc_hi=1.1,
                  tau=1.0, h_op=0.0, mu=0.0, slope=0.03, snap=0.0, slope_at=None, slope_ratio=0.0):
    """Seeded search refined by secant steps on g(t) = ln(r / T) (a proposal
    for the learned path; the paper has no predictor).  From the seed the
    first step is Newton's with the assumed slope ``slope`` of g per decade
    of alpha; later steps take the slope through the last two points (the
    assumed one when that is not positive).  Once points on both sides of
    the target are known, a step that leaves the bracket is replaced by the
    regula falsi point, with the Illinois halving of an end kept twice.
    A point at hi below the target ends with NOROOT_HIGH, one at lo above it
    with NOROOT_LOW; after max_steps steps the answer is the upper bracket
    end (MAXITER), evaluated if it was not the last point.  The first point
    is the seed as in ``_start``.  With ``slope_ratio`` > 0 and
    ``slope_at(t)`` (the whole-box residual's slope at t) positive at the
    seed, the assumed slope is ``slope_ratio * slope_at(seed)`` instead."""
    ev = _Counter(evaluate, delta, tau, h_op, mu)

    def ok(ratio):
        return acc_lo <= ratio <= acc_hi or abs(ratio - 1.0) <= tol

    def out(t, flags):
        return dict(alpha=10.0 ** t, t=t, flags=flags, n_evals=ev.n, trace=ev.trace)

    def lg(ratio):
        # ln(r / T), kept finite
        return min(max(math.log(ratio), -50.0), 50.0) if ratio > 0 else -50.0

    t = _start(t0, lo, hi, snap)
    rho, ratio, _, _ = ev(t)
    if ok(ratio):
        return out(t, 0)
    flags = PRED_FALLBACK
    if slope_ratio > 0 and slope_at is not None:
        sf = slope_at(t)
        if sf > 0:
            slope = slope_ratio * sf
    g = lg(ratio)
    a = b = ga = gb = None
    side = 0
    prev = None
    steps = 0
    while True:
        if rho < 0:                               # below the target: alpha too small
            if t >= hi:
                return out(hi, flags | NOROOT_HIGH)
            if a is not None and b is not None:
                if side == -1:
                    gb *= 0.5
                side = -1
            a, ga = t, g
        else:
            if t <= lo:
                return out(lo, flags | NOROOT_LOW)
            if a is not None and b is not None:
                if side == 1:
                    ga *= 0.5
                side = 1
            b, gb = t, g
        if steps >= max_steps:
            tb = b if b is not None else t
            if ev.last_t != tb:
                ev(tb)
            return out(tb, flags | MAXITER)
        s = (g - prev[1]) / (t - prev[0]) if prev is not None and t != prev[0] else 0.0
        if not s > 0:
            s = slope
        tn = t - g / s
        if a is not None and b is not None and not a < tn < b:
            tn = a - ga * (b - a) / (gb - ga)
        tn = min(max(tn, lo), hi)
        prev = (t, g)
        t = tn
        rho, ratio, _, _ = ev(t)
        steps += 1
        if ok(ratio):
            return out(t, flags)
        g = lg(ratio)


def kary(evaluate, delta, K=16, lo=-8.0, hi=0.0, max_steps=40, tol=1e-3, tau=1.0, h_op=0.0, mu=0.0):
    """K-candidate search (module docstring).  Returns dict(alpha, t, flags,
    n_evals, trace, steps)."""
    if K < 2:
        raise ValueError("K >= 2")
    ev = _Counter(evaluate, delta, tau, h_op, mu)

    def finish(t, flags, steps):
        ev(t)
        return dict(alpha=10.0 ** t, t=t, flags=flags, n_evals=ev.n, trace=ev.trace, steps=steps)

    a = b = None
    for step in range(max_steps):
        if step == 0:
            ts = [lo + j * (hi - lo) / (K - 1) for j in range(K)]
        else:
            ts = [a + (j + 1) * (b - a) / (K + 1) for j in range(K)]
        res = [ev(t) for t in ts]
        best = None
        for j, (rho, ratio, r, zn) in enumerate(res):
            d = abs(ratio - 1.0)
            if d <= tol and (best is None or d < best[0]):
                best = (d, j)
        if best is not None:
            return finish(ts[best[1]], 0, step + 1)
        rhos = [x[0] for x in res]
        if step == 0:
            if rhos[-1] < 0:
                return finish(hi, NOROOT_HIGH, 1)
            if rhos[0] > 0:
                return finish(lo, NOROOT_LOW, 1)
            pts, signs = ts, rhos
        else:
            pts = [a] + ts + [b]
            signs = [-1.0] + rhos + [0.0]          # rho(a) < 0 <= rho(b)
        jb = next(j for j, v in enumerate(signs) if v >= 0)
        a, b = pts[jb - 1], pts[jb]
    return finish(b, MAXITER, max_steps)

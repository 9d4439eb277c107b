// Device-resident control block of the alpha search.  a_scale converts the
// caller's alpha to the filter's: 1 (L2 units) or max |k^|^2 (relative).
//
// The regularisation parameter is chosen by the discrepancy principle
// (Sec. 4, after Algorithm 1: Tikhonov's method with the discrepancy
// principle or its generalisation).  With t = log10 alpha and r the residual
// on Y, rho(t) = r^2 - (tau delta + h_op ||zeta||)^2 - mu^2.
//
// The search runs on the device: the inverse transform of each evaluation
// reads alpha from this block and the last workgroup of the final pass, once
// the two FP64 norms are complete, advances the state machine below and
// writes the next alpha.  Once the search is done, `active` drops to 0 and
// every later pass kernel of that search returns at once, so the host can
// enqueue evaluations ahead without reading anything back.
//
// Plain search: every evaluated point with |r/T - 1| <= tol is accepted.
// Evaluate hi; rho < 0 -> done NOROOT_HIGH.  Evaluate lo; rho > 0 -> done
// NOROOT_LOW.  Then bisect: m = (a+b)/2, accept when
// |r/T - 1| <= tol, else a = m if rho < 0 else b = m; after max_steps the
// answer is b (MAXITER), re-evaluated there if b was not the last point.
// Seeded search: a point is accepted when acc_lo <= r/T <= acc_hi or
// |r/T - 1| <= tol.  Evaluate the predicted t0; otherwise walk toward the
// sign change with steps walk, 2 walk, 4 walk, ... (NOROOT at a range end),
// then regula falsi on g = r/T - 1 inside the bracket with the Illinois
// modification (the value kept at an end that survives two steps is halved).
// Secant refinement (slope > 0): after the seed, steps on g = ln(r/T), the
// first with the assumed slope of g per decade, later ones through the last
// two points (the assumed slope when that is not positive); a step that
// would leave a known bracket becomes the regula falsi point (Illinois);
// NOROOT at a range end, MAXITER after max_steps steps (answer b).  With a
// slope ratio c > 0 the first step assumes c times the whole-box residual's
// slope d ln ||C u - E_Y F|| / d log10 alpha at the seed (closed form by
// Parseval, summed by the seed's own z pass) when that is positive.
// K-candidate search: each step evaluates K alphas at once (the pass kernels
// take the candidate from the grid), step 1 at K points from lo to hi, later
// steps at the K interior points of the bracket (spaced (b - a)/(K + 1)).
// The candidate closest to the target among those within tol is accepted;
// otherwise (step 1) NOROOT_HIGH / NOROOT_LOW as in the plain search, and the
// bracket becomes [point before, first point with rho >= 0].  After max_steps
// steps the answer is b (MAXITER).  The answer is then evaluated once more
// on its own, which writes zeta and the final norms.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fr3d {

enum : int32_t {
  ST_IDLE = 0,
  ST_FIXED = 1,   // one evaluation at a given alpha
  ST_HI = 2,      // evaluating the upper range end
  ST_LO = 3,      // evaluating the lower range end
  ST_BISECT = 4,  // evaluating a bisection midpoint
  ST_FINAL = 5,   // re-evaluating b after the step limit
  ST_SEED = 6,    // evaluating the predicted point
  ST_WALK = 7,    // walking from the seed toward the sign change
  ST_FALSI = 8,   // regula falsi inside the bracket
  ST_DONE = 9,
  ST_KARY = 10,   // evaluating K candidates
  ST_KFINAL = 11, // evaluating the answer of the K-candidate search
  ST_SECANT = 12, // secant refinement of the seeded search
};

constexpr int KMAX = 16;  // candidates per step of the K-candidate search

enum : int32_t { F_NOROOT_HIGH = 1, F_NOROOT_LOW = 2, F_MAXITER = 4, F_NAN = 8, F_PRED_FALLBACK = 16 };

struct Ctrl {
  // first: every pass kernel of an evaluation reads these 16 bytes as one
  // load at its start (ctrl_head)
  int32_t state, active;
  double alpha_abs;  // 10^t * a_scale, read by the filter
  // settings
  double a_scale, delta, tau, h_op, mu, tol, acc_lo, acc_hi, lo, hi, walk;
  int32_t max_steps;
  // state
  int32_t n_evals, flags, steps;
  double t;          // log10 of the alpha being evaluated (caller units)
  double a, b;       // bracket
  double r2, z2;     // norms of the last evaluation
  double r2_full;    // full-box ||r||^2 of the last evaluation (diagnostics; < 0: not formed)
  double target;     // T of the last evaluation
  double ga, gb;     // r/T - 1 at the bracket ends (seeded search)
  double prev_t, prev_g, wstep;
  int32_t side, up;
  double slope;      // assumed d ln(r/T) / d log10 alpha of the secant refinement (0: walk)
  double slope_x;    // secant slope 10^(slope_x x_64) with the noise feature x_64 of the data
  double snap;       // a seed below lo + snap starts at lo
  double slope_ratio;  // > 0: the first secant step's slope is slope_ratio x slope_full
  double slope_full; // d ln r_full / d log10 alpha at the last evaluation (< 0: not formed)
  int32_t have;      // secant refinement: bit 0 a known, bit 1 b known, bit 2 previous point known
  // K-candidate search
  int32_t kc, kmax, pend;   // candidates this step, K, flags of the answer
  double ct[KMAX];          // log10 alpha of each candidate
  double ca[KMAX];          // filter alpha of each candidate
  void* kw1;                // K-candidate workspaces of the search: K slices of W1,
  void* kw2;                // K slices of W2 and K arrays of norm partials (the
  double2* knorm;           // K-candidate kernels take them from here)
  void* out;                // zeta of the search (device, nz*ny*nx), written by the x pass
};

static_assert(offsetof(Ctrl, state) == 0 && offsetof(Ctrl, active) == 4 && offsetof(Ctrl, alpha_abs) == 8,
              "ctrl_head reads the first 16 bytes");

// state, active and alpha_abs in one 16-byte load
__device__ __forceinline__ void ctrl_head(const Ctrl* c, int32_t& state, int32_t& active, double& alpha_abs) {
  int4 v;
  __builtin_memcpy(&v, c, sizeof(v));
  state = v.x;
  active = v.y;
  alpha_abs = __hiloint2double(v.w, v.z);
}

__device__ __forceinline__ void ctrl_set_t(Ctrl* c, double t) {
  c->t = t;
  c->alpha_abs = pow(10.0, t) * c->a_scale;
}

__device__ __forceinline__ void ctrl_finish(Ctrl* c, int32_t flags) {
  c->flags |= flags;
  c->state = ST_DONE;
  c->active = 0;
}

// Candidates of the next step of the K-candidate search (steps done so far
// in c->steps; bracket [a, b] after the first step).
__device__ inline void ctrl_kary_points(Ctrl* c) {
  const int K = c->kmax;
  for (int j = 0; j < K; ++j) {
    const double t = c->steps == 0 ? c->lo + j * (c->hi - c->lo) / (K - 1) : c->a + (j + 1) * (c->b - c->a) / (K + 1);
    c->ct[j] = t;
    c->ca[j] = pow(10.0, t) * c->a_scale;
  }
  c->kc = K;
}

__device__ inline void ctrl_kary_answer(Ctrl* c, double t, int32_t flags) {
  c->pend = flags;
  c->kc = 0;
  c->state = ST_KFINAL;
  ctrl_set_t(c, t);
}

// Advance after a K-candidate step with ||r||^2 = r2[j], ||zeta||^2 = z2[j].
__device__ inline void ctrl_advance_k(Ctrl* c, const double* r2, const double* z2) {
  const int K = c->kc;
  c->n_evals += K;
  double rho[KMAX];
  int best = -1;
  double bd = 0.0;
  for (int j = 0; j < K; ++j) {
    if (!isfinite(r2[j]) || !isfinite(z2[j])) {
      c->r2 = r2[j];
      c->z2 = z2[j];
      c->t = c->ct[j];
      ctrl_finish(c, F_NAN);
      return;
    }
    const double r = sqrt(r2[j]), zn = sqrt(z2[j]);
    const double g = c->tau * c->delta + c->h_op * zn;
    const double tgt2 = g * g + c->mu * c->mu;
    rho[j] = r2[j] - tgt2;
    const double ratio = tgt2 > 0 ? r / sqrt(tgt2) : INFINITY;
    const double d = fabs(ratio - 1.0);
    if (d <= c->tol && (best < 0 || d < bd)) { best = j; bd = d; }
  }
  const int step = c->steps;
  c->steps = step + 1;
  if (best >= 0) { ctrl_kary_answer(c, c->ct[best], 0); return; }
  int jb = 0;
  if (step == 0) {
    if (rho[K - 1] < 0) { ctrl_kary_answer(c, c->hi, F_NOROOT_HIGH); return; }
    if (rho[0] > 0) { ctrl_kary_answer(c, c->lo, F_NOROOT_LOW); return; }
    while (rho[jb] < 0) ++jb;  // jb >= 1: rho(lo) <= 0 and rho(lo) = 0 was accepted
    c->a = c->ct[jb - 1];
    c->b = c->ct[jb];
  } else {
    while (jb < K && rho[jb] < 0) ++jb;
    const double na = jb == 0 ? c->a : c->ct[jb - 1];
    const double nb = jb == K ? c->b : c->ct[jb];
    c->a = na;
    c->b = nb;
  }
  if (c->steps >= c->max_steps) { ctrl_kary_answer(c, c->b, F_MAXITER); return; }
  ctrl_kary_points(c);
}

// One step of the secant refinement after an evaluation at c->t that was not
// accepted (rho and r/T of that evaluation).
__device__ inline void ctrl_secant(Ctrl* c, double rho, double ratio) {
  const double g = ratio > 0 ? fmin(fmax(log(ratio), -50.0), 50.0) : -50.0;
  if (rho < 0) {
    if (c->t >= c->hi) { ctrl_finish(c, F_NOROOT_HIGH); return; }
    if ((c->have & 3) == 3) {
      if (c->side == -1) c->gb *= 0.5;
      c->side = -1;
    }
    c->a = c->t; c->ga = g; c->have |= 1;
  } else {
    if (c->t <= c->lo) { ctrl_finish(c, F_NOROOT_LOW); return; }
    if ((c->have & 3) == 3) {
      if (c->side == 1) c->ga *= 0.5;
      c->side = 1;
    }
    c->b = c->t; c->gb = g; c->have |= 2;
  }
  if (c->steps >= c->max_steps) {
    const double tb = (c->have & 2) ? c->b : c->t;
    if (tb == c->t) { ctrl_finish(c, F_MAXITER); return; }
    c->state = ST_FINAL;
    ctrl_set_t(c, tb);
    return;
  }
  double s = 0.0;
  if ((c->have & 4) && c->t != c->prev_t) s = (g - c->prev_g) / (c->t - c->prev_t);
  if (!(s > 0)) s = c->slope;
  double tn = c->t - g / s;
  if ((c->have & 3) == 3 && !(c->a < tn && tn < c->b)) tn = c->a - c->ga * (c->b - c->a) / (c->gb - c->ga);
  tn = fmin(fmax(tn, c->lo), c->hi);
  c->prev_t = c->t;
  c->prev_g = g;
  c->have |= 4;
  c->steps += 1;
  c->state = ST_SECANT;
  ctrl_set_t(c, tn);
}

// Whether the evaluation now running forms the full-box slope: the seed of
// a secant search with slope_ratio > 0.
__device__ __forceinline__ bool ctrl_wants_slope(const Ctrl* c) { return c->state == ST_SEED && c->slope_ratio > 0; }

// Advance after an evaluation at c->t with ||r||^2 = r2 and ||zeta||^2 = z2
// (sfull: the full-box slope, or < 0 when not formed).
__device__ inline void ctrl_advance(Ctrl* c, double r2, double z2, double sfull = -1.0) {
  c->r2 = r2;
  c->z2 = z2;
  c->slope_full = sfull;
  c->n_evals += 1;
  const double r = sqrt(r2), zn = sqrt(z2);
  const double g = c->tau * c->delta + c->h_op * zn;
  const double tgt2 = g * g + c->mu * c->mu;
  const double rho = r2 - tgt2;
  const double tgt = sqrt(tgt2);
  c->target = tgt;
  const double ratio = tgt2 > 0 ? r / tgt : INFINITY;
  if (!isfinite(r2) || !isfinite(z2)) { ctrl_finish(c, F_NAN); return; }
  const bool in_window = ratio >= c->acc_lo && ratio <= c->acc_hi;
  switch (c->state) {
    case ST_FIXED:
      ctrl_finish(c, 0);
      return;
    case ST_HI:
      if (fabs(ratio - 1.0) <= c->tol) { ctrl_finish(c, 0); return; }
      if (rho < 0) { ctrl_finish(c, F_NOROOT_HIGH); return; }
      c->state = ST_LO;
      ctrl_set_t(c, c->lo);
      return;
    case ST_LO:
      if (fabs(ratio - 1.0) <= c->tol) { ctrl_finish(c, 0); return; }
      if (rho > 0) { ctrl_finish(c, F_NOROOT_LOW); return; }
      c->a = c->lo; c->b = c->hi; c->steps = 0;
      c->state = ST_BISECT;
      ctrl_set_t(c, 0.5 * (c->a + c->b));
      return;
    case ST_BISECT:
      if (fabs(ratio - 1.0) <= c->tol) { ctrl_finish(c, 0); return; }
      if (rho < 0) c->a = c->t; else c->b = c->t;
      c->steps += 1;
      if (c->steps >= c->max_steps) {
        if (c->t == c->b) { ctrl_finish(c, F_MAXITER); return; }
        c->state = ST_FINAL;
        ctrl_set_t(c, c->b);
        return;
      }
      ctrl_set_t(c, 0.5 * (c->a + c->b));
      return;
    case ST_FINAL:
      ctrl_finish(c, F_MAXITER);
      return;
    case ST_KFINAL:
      ctrl_finish(c, c->pend);
      return;
    case ST_SEED:
    case ST_WALK: {
      const double g = ratio - 1.0;
      if (in_window || fabs(g) <= c->tol) { ctrl_finish(c, 0); return; }
      if (c->state == ST_SEED && c->slope > 0) {
        c->flags |= F_PRED_FALLBACK;
        c->have = 0;
        c->side = 0;
        c->steps = 0;
        if (c->slope_ratio > 0 && c->slope_full > 0) c->slope = c->slope_ratio * c->slope_full;
        ctrl_secant(c, rho, ratio);
        return;
      }
      if (c->state == ST_SEED) {
        c->flags |= F_PRED_FALLBACK;
        c->wstep = c->walk;
      } else {
        const bool changed = c->up ? rho >= 0 : rho <= 0;
        if (changed) {
          if (c->up) { c->a = c->prev_t; c->ga = c->prev_g; c->b = c->t; c->gb = g; }
          else { c->a = c->t; c->ga = g; c->b = c->prev_t; c->gb = c->prev_g; }
          c->side = 0;
          c->steps = 0;
          c->state = ST_FALSI;
          ctrl_set_t(c, c->b - c->gb * (c->b - c->a) / (c->gb - c->ga));
          return;
        }
        c->wstep *= 2.0;
      }
      c->up = rho < 0;
      if (c->up && c->t >= c->hi) { ctrl_finish(c, F_NOROOT_HIGH); return; }
      if (!c->up && c->t <= c->lo) { ctrl_finish(c, F_NOROOT_LOW); return; }
      c->prev_t = c->t;
      c->prev_g = g;
      c->state = ST_WALK;
      ctrl_set_t(c, c->up ? fmin(c->t + c->wstep, c->hi) : fmax(c->t - c->wstep, c->lo));
      return;
    }
    case ST_SECANT:
      if (in_window || fabs(ratio - 1.0) <= c->tol) { ctrl_finish(c, 0); return; }
      ctrl_secant(c, rho, ratio);
      return;
    case ST_FALSI: {
      const double g = ratio - 1.0;
      if (in_window || fabs(g) <= c->tol) { ctrl_finish(c, 0); return; }
      if (rho < 0) {
        c->a = c->t; c->ga = g;
        if (c->side == -1) c->gb *= 0.5;
        c->side = -1;
      } else {
        c->b = c->t; c->gb = g;
        if (c->side == 1) c->ga *= 0.5;
        c->side = 1;
      }
      c->steps += 1;
      if (c->steps >= c->max_steps) {
        if (c->t == c->b) { ctrl_finish(c, F_MAXITER); return; }
        c->state = ST_FINAL;
        ctrl_set_t(c, c->b);
        return;
      }
      ctrl_set_t(c, c->b - c->gb * (c->b - c->a) / (c->gb - c->ga));
      return;
    }
    default:
      ctrl_finish(c, 0);
      return;
  }
}

}  // namespace fr3d

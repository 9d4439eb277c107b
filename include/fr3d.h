/*
 * fr3d -- regularised FFT solve of the layered 3D Fredholm equation of the
 * first kind for the inverse coefficient problem of the wave equation
 * (Leonov & Bakushinsky, arXiv 1703.01216), on AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 3, Eq. (8)): find zeta on the layer R from data F on the
 * layer Y, where
 *     (A zeta)(y) = sum over cells r of R  h^3 K(x_y - x_r) zeta(r),
 *     K(x,y,z) = d/dz 1/|x| = -z / (x^2+y^2+z^2)^(3/2),
 * and F approximates A zeta with ||F - A zeta|| <= delta (Sec. 3, before
 * Eq. (11)).  The solve follows Algorithm 1 (Sec. 4) with the transform taken
 * over all three axes of the zero-padded P^3 = (2n)^3 box: Tikhonov's
 * estimate of the circulant-embedded operator
 *     zeta^ = conj(k^) f^ / (|k^|^2 + alpha),
 * the inverse transform restricted to R, alpha chosen by the discrepancy
 * principle on Y (Sec. 4, after Algorithm 1), and step 4:
 *     xi = zeta / V0,   c = (1/c0^2 - xi)^(-1/2)   (xi = 1/c0^2 - 1/c^2, Sec. 2).
 *
 * Conventions for every call:
 *   - Arrays are C order [z][y][x] (x fastest), cell (i,j,k) of R has centre
 *     ((i+.5)h, (j+.5)h, (k+.5)h); cell (i,j,k) of Y has centre
 *     ((i+.5)h, (j+.5)h, (D+k+.5)h).
 *   - Pointers with the suffix _dev are device pointers owned by the caller;
 *     they must stay valid until the context's stream has reached the work
 *     that uses them.  Element type is float for precision 32 and double for
 *     precision 64 unless stated.
 *   - All GPU work is enqueued on the stream given to fr3d_create.  Calls that
 *     return host values (reports, deltas, counts) synchronise that stream.
 *   - Every call returns an fr3d_status; no exception crosses the boundary.
 *     On failure fr3d_last_error(ctx) holds a message.  One context per host
 *     thread.
 */
#ifndef FR3D_H
#define FR3D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr3d_ctx fr3d_ctx;  /* opaque, owned by the library */

typedef enum {
  FR3D_OK = 0,
  FR3D_E_INVALID = 1, /* bad argument: null pointer, size, alpha <= 0, delta < 0, non-finite */
  FR3D_E_STATE = 2,   /* call out of order: no kernel loaded, no data set */
  FR3D_E_NOMEM = 3,   /* device allocation failed */
  FR3D_E_DEVICE = 4   /* HIP runtime error, or no usable gfx950 device */
} fr3d_status;

/* Report flags (non-fatal outcomes of a solve). */
#define FR3D_NOROOT_HIGH 1   /* residual below the target even at the largest alpha */
#define FR3D_NOROOT_LOW 2    /* residual above the target even at the smallest alpha */
#define FR3D_MAXITER 4       /* step limit reached; alpha is the upper bracket end */
#define FR3D_NAN_INPUT 8     /* a norm came out non-finite */
#define FR3D_PRED_FALLBACK 16 /* predicted alpha rejected; the search continued */
#define FR3D_CG_LIMIT 32      /* exact-operator solve: CG stopped at max_iter before its tolerance */
#define FR3D_UNFINISHED 64    /* _dev solve: the search had not ended after the enqueued evaluations */

/* Geometry of R and Y (Sec. 3: both are horizontal layers with the same
 * lateral footprint; Sec. 5: uniform grids, midpoint quadrature weight = the
 * cell volume h^2 hz). */
typedef struct {
  int32_t nx, ny, nz; /* cells per axis of R (= of Y); each 2n must be 2^a 3^b, n >= 2 */
  double h;           /* lateral cell edge (> 0); also the vertical one unless hz > 0 */
  double D;           /* z-offset of Y above R in vertical cells, >= nz; <= 0 selects the default */
  int32_t kind;       /* 0: K = dz(1/|x|) (Eq. (6), (8)); 1: K = 1/|x| (Eq. (5)) */
  int32_t q;          /* source parameter: -1 = single-kernel default gap nz + ceil(nz/4);
                         q >= 0: gap (q+1) ceil(nz/8) (each q gives its own kernel) */
  int32_t precision;  /* 32: FP32 complex transforms and filtering, FP64 kernel spectrum,
                         norms and alpha search; 64: all FP64 */
  int32_t alpha_relative; /* 0: alpha is the parameter of the Tikhonov functional
                         ||A zeta - F||^2 + alpha ||zeta||^2 in the L2 norms of Sec. 3
                         (the cell-volume weights of both terms cancel); 1: alpha is
                         relative, alpha_abs = alpha max|k^|^2 */
  double hz;          /* vertical cell edge; <= 0: hz = h (thin layers of Sec. 6 use hz < h) */
} fr3d_geom;

/* Options of the discrepancy search (Sec. 4: Tikhonov with the discrepancy
 * principle or its generalisation).  rho(t) = r(10^t)^2 - (tau delta +
 * h_op ||zeta||)^2 - mu^2 with r the residual on Y; t = log10 alpha. */
typedef struct {
  double log10_alpha_lo, log10_alpha_hi; /* search range, default -8, 0 */
  int32_t max_steps;                     /* bisection steps, default 40 */
  double tol;                            /* accept |r/T - 1| <= tol, default 1e-3 */
  double accept_lo, accept_hi;           /* window for predicted points, default 0.9, 1.1 */
  double tau, h_op, mu;                  /* generalised principle, default 1, 0, 0 */
  int32_t use_predictor;                 /* 1: seed the search with the alpha predictor */
  double seed_walk;                      /* first walk step from the seed in decades, default 0.25 */
  int32_t candidates;                    /* K = 2..16: K-candidate search (K alphas per step); 0: off */
  double seed_slope;                     /* > 0: secant refinement after the seed with this assumed
                                            d ln(r/T) / d log10 alpha; 0 (default): the walk */
  double seed_slope_x;                   /* with seed_slope > 0: the slope is seed_slope
                                            10^(seed_slope_x x_64), clamped to [1e-4, 1e3] (x_64 =
                                            log10(delta/||F||), the noise feature); default 0 */
  double seed_snap_lo;                   /* >= 0: a seed below log10_alpha_lo + seed_snap_lo (decades)
                                            starts the search at log10_alpha_lo; default 0 (off) */
  double seed_slope_ratio;               /* > 0 (3D form, Tikhonov filter, secant refinement): the first
                                            step's slope is seed_slope_ratio times the slope of the
                                            full-box residual d ln ||C u - E_Y F|| / d log10 alpha at the
                                            seed, formed exactly by the seed's evaluation; seed_slope
                                            when that is not positive; default 0 (off) */
} fr3d_dp_opts;

typedef struct {
  double alpha;             /* alpha of the returned estimate (geom.alpha_relative units) */
  double residual;          /* ||r||_Y at alpha */
  double zeta_norm;         /* ||zeta||_R at alpha */
  double delta;             /* noise level used */
  double target;            /* (tau delta + h_op ||zeta||)^2 + mu^2, square-rooted */
  int32_t n_evals;          /* number of alpha evaluations (inverse transforms) */
  int32_t flags;            /* FR3D_* report flags */
  int64_t n_clamped;        /* cells clamped by the recovery of c (batch with recovery), else -1 */
  double residual_full_box; /* with diagnostics on (fr3d_set_diagnostics), the residual of the
                               regularised model on the whole padded box, ||C u - E_Y F|| =
                               (sum |r^|^2 / (Px Py Pz))^(1/2) by Parseval, at alpha (3D form, single
                               evaluations); otherwise -1 */
} fr3d_report;

/* Defaults of fr3d_dp_opts. */
void fr3d_dp_opts_default(fr3d_dp_opts* opts);

/* Create a context on HIP device `device` enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  FR3D_E_DEVICE if the device is not
 * present or is not gfx950.  *out is NULL on failure. */
fr3d_status fr3d_create(fr3d_ctx** out, int32_t device, void* hip_stream);
/* Free every device buffer of the context (synchronises its stream). */
fr3d_status fr3d_destroy(fr3d_ctx* ctx);
/* Change the stream later work is enqueued on. */
fr3d_status fr3d_set_stream(fr3d_ctx* ctx, void* hip_stream);
/* Number of lanes (1..64) the batch solver uses.  Lane 0 runs on the
 * context's stream; each further lane owns a stream (default priority) and its
 * own data spectrum, workspaces and search state (about 1.3 P^3 complex values
 * each); all lanes share the kernel spectrum.  Lanes once created stay
 * allocated; a smaller count only leaves the extra ones idle. */
fr3d_status fr3d_set_lanes(fr3d_ctx* ctx, int32_t lanes);

/* Sample K at every wrapped cell offset of the P^3 box (zero in the slot no
 * pair of cells reaches), take its FP64 3D DFT and keep the octant
 * kx,ky,kz <= P/2 of k^ (k^ is even in kx and ky and Hermitian in kz).
 * Algorithm 1 step 1 (Sec. 4) for the kernel, with the midpoint quadrature of
 * Sec. 5.  Allocates the context's workspaces for this geometry; drops data
 * set earlier. */
fr3d_status fr3d_load_kernel(fr3d_ctx* ctx, const fr3d_geom* geom);

/* The same with the caller's kernel table instead of the sampled kernel of
 * Sec. 3 (the circulant embedding of Sec. 5 with any kernel that is real
 * and even in x and y): k_dev (device, FP64, read during the call only)
 * holds the wrapped samples k[c][b][a], Pz x Py x Px with a fastest, that is
 * the weight of the pair of cells whose offset is (a, b, c) modulo P, as in
 * (A zeta)[y] = sum_r k[(y - r) mod P] zeta[r], including the cell volume.
 * geom gives nx, ny, nz, precision and alpha_relative (kind is not used; h,
 * hz, D and q only place the point sources of fr3d_source_potential).
 * Samples that are not finite, all zero or not even in x and y (relative
 * deviation above 1e-12) give FR3D_E_INVALID and leave no kernel loaded. */
fr3d_status fr3d_load_kernel_samples(fr3d_ctx* ctx, const fr3d_geom* geom, const double* k_dev);

/* Algorithm 1 as run in Sec. 5: load the geometry for the lateral 2D
 * transform and per-frequency dense z-systems of Eq. (14) instead of the 3D
 * embedding.  Lateral axes are zero-padded to 2n (the exact discrete lateral
 * convolution); z is not embedded: for every lateral frequency the real
 * nz x nz matrix A[i][j] = k~(kx, ky; i - j) couples R's layer j with Y's
 * layer i, k~ being the lateral transform of the kernel samples at the z
 * offset (D + i - j) h (K is even in x and y, so A is real and shared by
 * ky and Py - ky).  Each A is factorised once here (one-sided Jacobi SVD in
 * FP64).  Afterwards set_data, solve_alpha, solve_discrepancy (plain and
 * K-candidate searches), solve_batch / solve_group, recover_c,
 * apply_operator (F^ = A zeta^ per frequency) and the filters of
 * fr3d_set_filter work on this form; one alpha for all frequencies, the
 * discrepancy on Y's whole footprint.  Not available in this form:
 * predictor features (use_predictor, get_features, batch features) and the
 * 3D octant (FR3D_E_STATE).  get_data_spectrum returns the lateral spectrum,
 * complex T [Px/2+1][nz][Py].  Limits: 1 <= nz <= 60, 2 nx and 2 ny
 * compiled lengths; nz needs no transform length.  geom as for
 * fr3d_load_kernel (alpha_relative scales by the largest s^2). */
fr3d_status fr3d_load_layered(fr3d_ctx* ctx, const fr3d_geom* geom);

/* Set the data F on Y (nz*ny*nx values, device) and the noise level delta >= 0
 * (absolute, ||F - A zeta|| <= delta).  Runs the zero-padded forward
 * transform (Algorithm 1 step 1 for the data) and the predictor features'
 * energy reduction.  F is not retained. */
fr3d_status fr3d_set_data(fr3d_ctx* ctx, const void* F_dev, double delta);

/* One alpha evaluation at alpha > 0 (units set by geom.alpha_relative):
 * Algorithm 1 steps 2-3 with Tikhonov's filter.  Writes zeta on R
 * (nz*ny*nx, device) and fills *rep (synchronises). */
fr3d_status fr3d_solve_alpha(fr3d_ctx* ctx, double alpha, void* zeta_dev, fr3d_report* rep);

/* Choose alpha by the discrepancy principle and write zeta at that alpha.
 * opts NULL = defaults.  Plain rule: evaluate the range ends (hi first), then
 * bisect in log10 alpha; any point with |r/T - 1| <= tol is accepted.  With
 * use_predictor: start from the predicted alpha (clipped to the range; lo
 * itself when it is within seed_snap_lo decades above lo; accepted inside
 * [accept_lo, accept_hi] or within tol), walk toward the sign change with doubling steps
 * from seed_walk decades, then Illinois regula falsi on r/T - 1 inside the
 * bracket; with seed_slope > 0 instead secant steps on ln(r/T), the first
 * with the slope seed_slope per decade, later ones through the last two
 * points, regula falsi (Illinois) when a step would leave a known bracket.  With candidates = K (2..16, not with use_predictor, max_steps >= 1):
 * each step evaluates K alphas in one set of launches, the first step at K
 * points from lo to hi, later steps at the K interior points of the current
 * bracket (log-spaced); the candidate closest to the target within tol is
 * accepted, else the bracket narrows to the two points around the sign change
 * of rho (NOROOT_* as above after the first step, MAXITER after max_steps
 * steps with the answer b); the answer is evaluated once more on its own to
 * write zeta (n_evals = K steps + 1).  Fills *rep (synchronises). */
fr3d_status fr3d_solve_discrepancy(fr3d_ctx* ctx, const fr3d_dp_opts* opts, void* zeta_dev,
                                   fr3d_report* rep);

/* fr3d_solve_alpha and fr3d_solve_discrepancy (Algorithm 1 steps 2-3 and
 * the discrepancy principle of Sec. 4) without a host
 * synchronisation, for callers that chain a solve behind other device work
 * or capture it into a HIP graph (stream capture on the context's stream,
 * fr3d_set_stream): the search's first point, every evaluation the search
 * may need (its bound: 1 for a fixed alpha; 2 + max_steps + 1 for the plain
 * rule; 1 + max_steps + 1 seeded with seed_slope > 0; seed + walk +
 * max_steps + 1 seeded otherwise; max_steps K-candidate steps) and a final
 * kernel that writes the report to rep_dev are enqueued on the context's
 * stream, and the call returns.  Evaluations enqueued after the search has
 * ended return at once (a few microseconds per pass launch), so a small
 * max_steps keeps that idle tail short.  rep_dev: device memory for one
 * fr3d_report, owned by the caller; zeta_dev and rep_dev must stay valid
 * until the stream reaches them.  The report equals the synchronous call's
 * (n_clamped = -1); FR3D_UNFINISHED is set if the search had not ended.  The
 * evaluations are plain kernel launches (fr3d_set_graphs does not apply), no
 * memory is allocated or set by the host except the K-candidate workspaces on
 * a context's first K-candidate search (run one before capturing such
 * searches).  A captured solve replays with the delta, options and pointers
 * of its capture.  Errors found on the host are returned: FR3D_E_INVALID
 * (null zeta_dev or rep_dev, bad options, alpha), FR3D_E_STATE (no kernel or
 * data, timing on: fr3d_set_timing records host-side events). */
fr3d_status fr3d_solve_alpha_dev(fr3d_ctx* ctx, double alpha, void* zeta_dev, fr3d_report* rep_dev);
fr3d_status fr3d_solve_discrepancy_dev(fr3d_ctx* ctx, const fr3d_dp_opts* opts, void* zeta_dev,
                                       fr3d_report* rep_dev);

/* Solve n instances on the lanes: for item i, set the data F_devs[i] with
 * noise level deltas[i], choose alpha by the discrepancy principle (opts,
 * NULL = defaults) writing zeta_devs[i], and, if c_devs is not NULL, recover
 * c into c_devs[i] from V0_dev and c0; feat_dev, if not NULL, receives each
 * item's 65 predictor features (float [n][65], device).  Instances run concurrently, one per
 * lane; each lane advances one evaluation at a time and the host polls the
 * lanes, so no evaluation is launched after its search has ended.  The
 * caller's stream is ordered before and after the whole batch.  reps[i]
 * receives each item's report (n_clamped when c is recovered).  Returns when
 * every search has finished (recoveries may still be in flight on the
 * context's stream). */
fr3d_status fr3d_solve_batch(fr3d_ctx* ctx, int32_t n, const void* const* F_devs, const double* deltas,
                             void* const* zeta_devs, const fr3d_dp_opts* opts, const void* V0_dev, double c0,
                             void* const* c_devs, float* feat_dev, fr3d_report* reps);

/* The same solve for items of different geometries (Sec. 6 model: grid sizes
 * and source sets differ between surveys): item i runs on ctxs[i], a context
 * whose kernel is loaded for that item's grid (nz*ny*nx of that context),
 * with V0s[i] its V0 when c_devs is not NULL.  Every lane of every distinct
 * context is scheduled together, so instances of all geometries are in
 * flight at once.  With use_predictor each context uses its own loaded
 * predictor.  A context must not appear in two concurrent calls.  Errors are
 * reported on ctxs[0] (fr3d_last_error).  n = 0 returns FR3D_OK. */
fr3d_status fr3d_solve_group(int32_t n, fr3d_ctx* const* ctxs, const void* const* F_devs, const double* deltas,
                             void* const* zeta_devs, const fr3d_dp_opts* opts, const void* const* V0_devs,
                             double c0, void* const* c_devs, fr3d_report* reps);

/* Algorithm 1 step 4: xi = zeta / V0 and c = (1/c0^2 - xi)^(-1/2) on R; where
 * 1/c0^2 - xi < 1e-6/c0^2 the argument is clamped and the cell counted in
 * *n_clamped (synchronises).  c0 > 0.  zeta, V0, c: nz*ny*nx device arrays. */
fr3d_status fr3d_recover_c(fr3d_ctx* ctx, const void* zeta_dev, const void* V0_dev, double c0,
                           void* c_dev, int64_t* n_clamped);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * recovery of fr3d_recover_c without a context, without any allocation and
 * without a host synchronisation.  c = (1/c0^2 - zeta/V0)^(-1/2) over n
 * cells with the same clamp as fr3d_recover_c (identical c, identical
 * count); precision 32 (float arrays) or 64 (double arrays); zeta_dev,
 * V0_dev, c_dev: n device values each, any layout (elementwise), owned by
 * the caller; n_clamped_dev: one device int64 that receives the number of
 * clamped cells, or NULL to skip the count.  Work is enqueued on hip_stream
 * (a hipStream_t, NULL = the null stream) of the current device.
 * Workspace: the per-workgroup partial counts live in a static device array
 * of 2048 doubles (16 KiB), one per device, held until the process ends;
 * every call on a device shares it, so calls that overlap on one device
 * (concurrent streams or host threads) race -- serialise them.  Nothing in
 * it needs clearing (each call writes every partial it reads).
 * FR3D_E_INVALID: precision not 32 or 64, n < 0 or n > FR3D_NOALLOC_MAX_CELLS,
 * a null array with n > 0, c0 not finite and > 0.  FR3D_E_DEVICE: the
 * current device is not a gfx950, its workspace address could not be
 * obtained, or a launch failed.  n = 0 writes a count of 0. */
#define FR3D_NOALLOC_MAX_CELLS (((int64_t)1) << 40)
fr3d_status fr3d_recover_c_noalloc(int32_t precision, int64_t n, const void* zeta_dev, const void* V0_dev, double c0,
                                   void* c_dev, int64_t* n_clamped_dev, void* hip_stream);

/* V0 on R's cell centres for the geometry's ten point sources (Sec. 6):
 * V0(x) = -(A0/4 pi) sum_l 1/|x - x_l|.  The sources form the model example's
 * cross (lateral centre and +-0.4 n along x and y) at heights nz + G/4 and
 * nz + 3G/4 with G = D - nz.  Writes nz*ny*nx values. */
fr3d_status fr3d_source_potential(fr3d_ctx* ctx, double A0, void* V0_dev);

/* Algorithm 1 step 2 read per lateral frequency (per-frequency systems only,
 * after fr3d_load_layered and fr3d_set_data): every system gets its own
 * alpha by the plain discrepancy rule of fr3d_solve_discrepancy (upper end,
 * lower end, bisection in log10 alpha over opts' range, any point within
 * opts.tol accepted) applied to its own residual ||A x^ - f^|| against
 * tau delta, in unnormalised lateral-DFT units (white noise of norm delta on
 * Y has expected energy delta^2 at every frequency); then one lateral
 * inverse writes zeta on R.  alpha_dev (double [Px/2+1][Py]) and flags_dev
 * (int32 [Px/2+1][Py]), if not NULL, receive each frequency's alpha (in
 * the search's units, relative to s_max when the geometry says so) and
 * flags.  rep: alpha = 10^(mean log10 alpha over all Px Py frequencies),
 * residual = ||r||_Y and zeta_norm of the result, flags = OR of the
 * per-frequency flags, n_evals = 1.  use_predictor, candidates and a
 * nonzero h_op or mu are rejected (FR3D_E_INVALID); a context without the per-frequency systems or
 * data gives FR3D_E_STATE; synchronises. */
fr3d_status fr3d_solve_per_frequency(fr3d_ctx* ctx, const fr3d_dp_opts* opts, void* zeta_dev, double* alpha_dev,
                                     int32_t* flags_dev, fr3d_report* rep);

/* Tikhonov's method for the exact discrete operator A: L2(R) -> L2(Y) (the
 * quadrature of Eq. (8); Sec. 3's regularised normal solution, nothing on a
 * padded box): zeta = argmin ||A zeta - F||^2_Y + alpha ||zeta||^2_R, by
 * conjugate gradients on (A^T A + alpha I) zeta = A^T F from zero; every
 * product with A and A^T runs through the context's transforms (A^T with
 * the conjugate kernel spectrum).  Stops when the normal-equation residual
 * is <= tol ||A^T F|| (checked every 16 steps) or after max_iter steps
 * (flag FR3D_CG_LIMIT).  F: data on Y, zeta: out, nz*ny*nx device arrays;
 * alpha in the units of geom.alpha_relative.  rep: alpha, residual =
 * ||A zeta - F||_Y, zeta_norm, n_evals = CG steps.  Overwrites the context's
 * data spectrum (set_data again before the other solves); synchronises. */
fr3d_status fr3d_solve_exact(fr3d_ctx* ctx, const void* F_dev, double alpha, void* zeta_dev, int32_t max_iter,
                             double tol, fr3d_report* rep);

/* The same with alpha chosen by the plain discrepancy rule of
 * fr3d_solve_discrepancy (bisection in log10 alpha, range ends first, any
 * point within tol accepted; use_predictor and candidates are rejected),
 * each point a CG solve from zero; n_evals counts alpha points, flags add
 * FR3D_CG_LIMIT if any solve hit max_iter. */
fr3d_status fr3d_solve_exact_discrepancy(fr3d_ctx* ctx, const void* F_dev, double delta, const fr3d_dp_opts* opts,
                                         void* zeta_dev, int32_t max_iter, double tol, fr3d_report* rep);

/* Apply the forward operator: F = A zeta on Y (Eq. (8) by midpoint
 * quadrature), through the same padded transforms and the loaded kernel
 * spectrum.  zeta on R, F on Y, both nz*ny*nx device arrays; may alias. */
fr3d_status fr3d_apply_operator(fr3d_ctx* ctx, const void* zeta_dev, void* F_dev);

/* F += e * (delta_rel ||F|| / ||e||) with FP64 norms; *delta (host) receives
 * ||added noise|| (synchronises).  F, e: nz*ny*nx device arrays. */
fr3d_status fr3d_add_noise(fr3d_ctx* ctx, void* F_dev, const void* e_dev, double delta_rel,
                           double* delta);

/* Inspection of the context's spectra (for checks).  Layouts:
 *   octant: double2 [Px/2+1][Pz/2+1][Py/2+1]  (k^ at kx, kz, ky)
 *   data spectrum: complex T [Px/2+1][Pz][Py] (f^ at kx, kz, ky; kx <= Px/2)
 *   features: float[65] = log10(E_b/mean E + 1e-30), b < 64, then log10(delta/||F||)
 *   energy: double[64] E_b = sum of |f^|^2 over the full spectrum's points of level b,
 *     the level of a point being the number of thresholds s_max 10^((j - 64)/4),
 *     j = 1..63, that its |k^|^2 reaches (quarter decades below s_max; the
 *     Tikhonov filter acts on a point through |k^|^2 alone). */
fr3d_status fr3d_get_octant(fr3d_ctx* ctx, void* out_dev, int64_t bytes);
fr3d_status fr3d_get_data_spectrum(fr3d_ctx* ctx, void* out_dev, int64_t bytes);
fr3d_status fr3d_get_features(fr3d_ctx* ctx, float* feat_dev, double* energy_dev);
/* |k^|max^2 of the loaded kernel (host). */
fr3d_status fr3d_get_smax(fr3d_ctx* ctx, double* smax);

/* Singular values of the per-frequency systems (Sec. 5, Eq. (14); Fig. 6
 * shows their decay), after fr3d_load_layered: out (device, double,
 * [Px/2+1][Py/2+1][nz]) receives for each distinct system (kx, |ky|) its
 * nz singular values in descending order.  bytes is out's capacity; a
 * smaller buffer gives FR3D_E_INVALID, a 3D context FR3D_E_STATE.
 * Asynchronous on lane 0's stream. */
fr3d_status fr3d_get_singular_values(fr3d_ctx* ctx, double* out, int64_t bytes);

/* The alpha predictor (not part of the paper): a perceptron 65 -> 128 ->
 * 128 -> 1 with exact-erf GELU, bfloat16 matrix-core products with FP32
 * accumulation, FP32 master weights and Adam.  Input: the 65 features of a
 * data set (fr3d_get_features), standardised by norm = (mu[65], sigma[65],
 * t_mu, t_sigma); output log10 alpha = t_mu + t_sigma y.  Parameters (FP32,
 * host arrays): W1[128][65], b1[128], W2[128][128], b2[128], w3[128], b3 --
 * 25089 values.  With fr3d_dp_opts.use_predictor the network's prediction
 * for the set data is the first point of the search. */
fr3d_status fr3d_predictor_set(fr3d_ctx* ctx, const float* params, int64_t n_params, const float* norm);
fr3d_status fr3d_predictor_get(fr3d_ctx* ctx, float* params, float* norm);
/* y_dev[b] = predicted log10 alpha for raw features X_dev[b][65], b < B (device arrays). */
fr3d_status fr3d_predictor_forward(fr3d_ctx* ctx, const float* X_dev, int32_t B, float* y_dev);
/* One training step on B rows (device arrays X_dev[B][65], t_dev[B] = log10
 * alpha targets): gradients of the mean squared error in standardised units,
 * then Adam (beta 0.9/0.999, eps 1e-8) with learning rate lr if lr > 0.
 * loss_dev (1 float) and grad_dev (25089 floats) receive the loss and the
 * gradients when not NULL. */
fr3d_status fr3d_predictor_train_step(fr3d_ctx* ctx, const float* X_dev, const float* t_dev, int32_t B, double lr,
                                      float* loss_dev, float* grad_dev);
/* Checkpoint: parameters, normalisation, Adam moments and step, with a
 * checksum; load rejects a corrupt or foreign file with FR3D_E_INVALID. */
fr3d_status fr3d_predictor_save(fr3d_ctx* ctx, const char* path);
fr3d_status fr3d_predictor_load(fr3d_ctx* ctx, const char* path);
/* Calibration of the network's seed for one geometry (callers that fit it on
 * instances of that geometry, e.g. by least squares): the seed becomes
 * clip(prediction + coef[0] + sum_k coef[1+k] x_k) with x the 65 raw
 * features.  coef: 66 host doubles, copied; NULL or n = 0 clears it.
 * Setting or loading a network clears it.  FR3D_E_INVALID for n != 66 or
 * non-finite values, FR3D_E_STATE without a network; synchronises. */
fr3d_status fr3d_predictor_set_calibration(fr3d_ctx* ctx, const double* coef, int64_t n);

/* Tile size and radix plan of a pass (ids as for timing): shift 0 = a 32 KiB
 * LDS tile of pencils, 1 = half, 2 = quarter (row passes 0, 1, 4); for the
 * inverse z pass (3) shift 2 is the half tile of ky columns with u^ and r^
 * transformed together as one 32 KiB tile.  Lengths below 64 always use
 * shift 0.  shift + 4 v selects radix plan variant v (0 default; 1, 2 other
 * orders of the stage radices) for the FP32 transforms of lengths 192
 * (16.4.3, 8.8.3, 4.16.3), 384 (16.8.3, 8.16.3, 3.16.8) and 512 (8.8.8,
 * 16.8.4, 16.16.2); other lengths and FP64 use plan 0.  Results do not depend
 * on either beyond rounding; the autotuner picks both. */
fr3d_status fr3d_set_tile(fr3d_ctx* ctx, int32_t pass, int32_t shift);

/* Regularising filter of every later evaluation (Sec. 5 names Tikhonov,
 * iterated Tikhonov and truncated SVD as the algorithms applied): kind 0 =
 * Tikhonov (default), 1 = iterated Tikhonov of the given order (1..64; the
 * minimiser of ||A u - F||^2 + alpha ||u - u_prev||^2 applied `order` times
 * from 0), 2 = truncated SVD of the embedded operator with cut alpha
 * (spectral modes with |k^|^2 >= alpha inverted, the others dropped).
 * alpha keeps the units of geom.alpha_relative; the discrepancy searches
 * apply unchanged (r grows with alpha for all three).  Waits for the
 * context's streams.  E_INVALID on a bad kind or order. */
fr3d_status fr3d_set_filter(fr3d_ctx* ctx, int32_t kind, int32_t order);

/* Diagnostics of the 3D form: with enable = 1 every single evaluation also
 * forms the full-box residual (one more read of the spectrum and the
 * octant, and a small reduction), reported as residual_full_box; it is the
 * residual on the whole padded box, a diagnostic beside the residual on Y
 * that the discrepancy rule uses.  Default 0 (the field is -1).
 * Synchronises the context's lanes. */
fr3d_status fr3d_set_diagnostics(fr3d_ctx* ctx, int32_t enable);

/* With enable = 1, each lane captures its evaluation's launch sequence (the
 * z, y and x passes and the norm kernel, for K-candidate searches both the
 * K-candidate step and the single evaluation) into a HIP graph once and
 * replays it for every later evaluation; the search state and the zeta
 * pointer live in the lane's control block, so one graph serves every item.
 * Results are identical either way.  Ignored while timing is on.  A graph
 * is re-captured after a change of geometry, tile sizes or K. */
fr3d_status fr3d_set_graphs(fr3d_ctx* ctx, int32_t enable);

/* Per-pass timing with HIP events on the context's stream (for measurement).
 * Pass ids: 0..2 forward x,y,z; 3..5 inverse z,y,x. */
fr3d_status fr3d_set_timing(fr3d_ctx* ctx, int32_t enable);
fr3d_status fr3d_get_timing(fr3d_ctx* ctx, int32_t pass, double* total_ms, int64_t* launches);

const char* fr3d_status_string(fr3d_status s);
const char* fr3d_last_error(const fr3d_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FR3D_H */

/*
 * stokesreg — extrapolated-regularization Stokes single- and double-layer sums on MI355X (gfx950).
 *
 * C ABI of libstokesreg.so.  The method is that of Siebor & Tlupova (arXiv 2507.00156), which
 * localizes and accelerates the extrapolated regularization of Beale & Tlupova:
 *
 *   single layer (Stokeslet), paper eqs. (Stokes_SL), (Stokeslet), (Stokes_SL1):
 *     u_i(y) = 1/(8 pi) sum_p S_ij(y, x_p) [f_j(x_p) - f_k(x0) n_k(x0) n_j(x_p)] w_p
 *   double layer (stresslet), eqs. (Stokes_DL), (Stresslet), (Stokes_DL1):
 *     v_i(y) = 1/(8 pi) sum_p T_ijk(y, x_p) [q_j(x_p) - q_j(x0)] n_k(x_p) w_p + chi(y) q_i(x0)
 *
 * evaluated with the regularized kernels of eqs. (Sreg), (Treg) and the split stresslet (Tsplit) at
 * three smoothing lengths delta_j = rho_j h (smoothing factors (s1)-(s3), set to 1 for r/delta > 6,
 * section 3.2), and combined by the 3x3 extrapolation of eq. (extrap_eqn) with I0, I2 of eqs. (I0),
 * (I2).  The sum over quadrature points is split as in eq. (near_far): pairs with r <= 6 max_j delta_j
 * ("near") are summed with the regularized kernels for each delta_j; all other pairs ("far") are
 * summed once with the original kernels and shared by the three deltas (section 3.3).  The far part
 * is a direct sum, or the barycentric-Lagrange treecode of section 3.4.
 *
 * Conventions common to every entry point
 *   - Every array argument is a DEVICE pointer (HBM of the context's GPU), double precision,
 *     row-major: a "(k,3)" array holds k consecutive xyz triples; a "(k)" array k scalars.  The
 *     evaluation calls sr_eval and sr_eval_far also accept HOST pointers when SR_HOST is or'ed into
 *     `layers`; they then copy through device buffers of the context and return after the results
 *     are back in host memory.
 *   - Arrays are borrowed for the duration of the call; the library copies what it keeps.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it and the call
 *     returns without waiting, except for the set-up calls noted below.  Calls on one context must
 *     not overlap (use one stream, or synchronize between streams): the context's work buffers are
 *     shared by its calls.
 *   - Every entry point returns an sr_status; none aborts.  On failure sr_last_error() gives a
 *     message (thread-local, valid until the next call from the same thread).
 *   - Output is in the paper's normalization (the 1/(8 pi) factor included).
 */
#ifndef STOKESREG_H
#define STOKESREG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sr_ctx sr_ctx;

typedef enum {
    SR_OK = 0,
    SR_EINVAL = -1,  /* invalid argument (null pointer, bad size, bad parameter value)      */
    SR_ENOMEM = -2,  /* device or host allocation failed                                    */
    SR_ENODEV = -3,  /* no GPU, or the requested device ordinal does not exist              */
    SR_ESTATE = -4,  /* call out of order (e.g. sr_eval before the surface/density is set)  */
    SR_EHIP = -5,    /* a HIP runtime call or kernel launch failed                          */
    SR_ENOCONV = -6, /* an iterative solve did not reach its tolerance                      */
    SR_ENEAR = -7    /* a target treated as far from the surface lies within the near radius
                        of a source (reported by sr_check)                                  */
} sr_status;

/* Layer selection bits for sr_set_density / sr_eval.  SR_HOST (sr_eval, sr_eval_far only): the
 * array arguments are host pointers. */
enum { SR_SL = 1, SR_DL = 2, SR_HOST = 16 };

/* Far-field precision.  SR_FP64: every sum in double.  SR_MIXED: far-field pair kernels in single
 * precision with double accumulation of 32-pair partial sums; the near regularized sums, the
 * far/near bookkeeping and the extrapolation stay in double. */
enum { SR_FP64 = 0, SR_MIXED = 1 };

/* Far-field method: direct O(MN) sum, or the barycentric Lagrange treecode (section 3.4). */
enum { SR_DIRECT = 0, SR_TREE = 1 };

typedef struct {
    double h;           /* quadrature grid spacing h (> 0)                                        */
    double rho[3];      /* smoothing ratios: delta_j = rho_j h (> 0, pairwise distinct); e.g. 2,3,4 */
    double cutoff;      /* smoothing cut-off in t = r/delta; the paper uses 6 (> 0)               */
    int precision;      /* SR_FP64 or SR_MIXED                                                    */
    int far_method;     /* SR_DIRECT or SR_TREE                                                   */
    int tree_degree;    /* treecode: Chebyshev interpolation degree p (1..16)                     */
    double tree_theta;  /* treecode: multipole acceptance parameter theta, MAC r_c / R <= theta,
                           and the cluster's box farther than the near radius R_n = cutoff
                           max(rho, sharp_rho if surface_sharp) h.  With SR_MIXED the box must lie
                           farther than R_n (1 + 1e-5) + 2^-22 (2 E + R_n), E = max_d (max_i x_id
                           - min_i x_id) / 2 (the reach of the single-precision near-pair test), so
                           that no source of an accepted cluster is also summed as a near pair     */
    int tree_leaf;      /* treecode: maximum number of points in a leaf N0 (>= 1)                 */
    int surface_sharp;  /* 1: targets ON the surface (b == 0) use the modified smoothing functions
                           s1#, s2#, s3# of paper section 2.1 at the single delta sharp_rho h, with no
                           extrapolation (single layer: eq. (Sreg) with s1#, s2#; double layer: the
                           stresslet with s3#(r/delta)/r^5 in place of 1/r^5); other targets are
                           extrapolated as usual.  0 (default): every target is extrapolated.      */
    double sharp_rho;   /* delta / h of the modified smoothing (> 0); default 3                     */
} sr_params;

/* Fill *p with defaults: h = 0 (must be set), rho = (2,3,4), cutoff = 6, SR_FP64, SR_DIRECT,
 * tree_degree = 8, tree_theta = 0.7, tree_leaf = 2000. */
void sr_default_params(sr_params *p);

/* Create a context on HIP device `device` (ordinal).  SR_ENODEV if it does not exist.  The context
 * owns one non-blocking, default-priority stream and two events on that device (the concurrent
 * near-field phase of sr_eval), released by sr_destroy; SR_EHIP if they cannot be created. */
sr_status sr_create(sr_ctx **out, int device);

/* Release the context and all device memory it owns.  NULL is accepted. */
sr_status sr_destroy(sr_ctx *c);

/* Set the method parameters (copied).  May be called again; a change of h, rho or cutoff rebuilds
 * the near-pair cell list at the next evaluation. */
sr_status sr_set_params(sr_ctx *c, const sr_params *p);

/* Set the surface quadrature (paper section 2.2, eq. (quadrature)): n points x (n,3), outward unit
 * normals nrm (n,3) and weights w (n).  1 <= n <= sr_max_targets().  The data are copied; this call synchronizes
 * `stream` (it reads the points back to build the spatial index on the host).  Invalidates any
 * densities set before. */
sr_status sr_set_surface(sr_ctx *c, int64_t n, const double *x, const double *nrm, const double *w,
                         void *stream);

/* Set the density of one layer at the quadrature points, (n,3) in the order of sr_set_surface:
 * layer = SR_SL: the force density f of eq. (Stokes_SL); layer = SR_DL: q of eq. (Stokes_DL).
 * Copied; asynchronous on `stream`. */
sr_status sr_set_density(sr_ctx *c, int layer, const double *dens, void *stream);

/* Evaluate the extrapolated layer potentials at m targets (paper section 2, eqs. (Stokes_SL1),
 * (Stokes_DL1), (extrap_eqn); y = x0 + b n0 as defined there).
 *   layers      SR_SL, SR_DL or SR_SL|SR_DL (both in one pass, sharing the pair geometry); | SR_HOST
 *               for host arrays (the call then synchronizes `stream`).
 *   m           0 <= m <= sr_max_targets() (2^28); SR_EINVAL otherwise.  Evaluated in chunks of at
 *               most 2^20 targets, one after the other, so that the context's work space (768 bytes per
 *               target of a chunk for the far-field partial sums) stays bounded.
 *   y (m,3)     target points.
 *   x0 (m,3)    closest point on the surface to each target;  n0 (m,3) the outward unit normal there;
 *   b (m)       signed distance, y = x0 + b n0 (b > 0 outside, b < 0 inside, b == 0 on the surface).
 *               A target with |b| >= cutoff max_j delta_j takes the far rule: one smoothing length, no
 *               extrapolation (every pair is beyond the cut-off there).  If such a target has a
 *               source closer than cutoff max_j delta_j, its b (or x0) is wrong; the evaluation still
 *               completes and the next sr_check returns SR_ENEAR.  Targets with no closest point
 *               belong to sr_eval_far.
 *   f0 (m,3)    f(x0), needed if SR_SL is requested (else may be NULL);
 *   q0 (m,3)    q(x0), needed if SR_DL is requested (else may be NULL).
 *   u (m,3)     output single layer (if SR_SL);  v (m,3) output double layer incl. chi q(x0) (if SR_DL).
 *   u_delta, v_delta  optional (may be NULL): (m,3,3) regularized values before extrapolation,
 *               [target][j][component] for delta_j, 1/(8 pi) included, chi q(x0) excluded.
 * m == 0 is a no-op.  SR_ESTATE if the surface, the parameters or a requested density is not set.
 * The work is asynchronous on `stream`.  When u_delta and v_delta are NULL and profiling is off,
 * the near-field kernel runs on a stream the context owns, concurrently with the far field on
 * `stream`: it starts after the work enqueued on `stream` before the call, and work enqueued on
 * `stream` after the call starts after it, so the call behaves as one operation on `stream`.  Two
 * calls on one context must not overlap in time from different host threads. */
sr_status sr_eval(sr_ctx *c, int layers, int64_t m, const double *y, const double *x0, const double *n0,
                  const double *b, const double *f0, const double *q0, double *u, double *v,
                  double *u_delta, double *v_delta, void *stream);

/* Evaluate the layer potentials at m targets that have no closest point (targets far from the
 * surface, e.g. a flow field): the plain sums of eqs. (Stokes_SL), (Stokes_DL) with the original
 * kernels (Stokeslet), (Stresslet), no subtraction and no regularization,
 *   u = 1/(8 pi) sum_p S(y, x_p) f_p w_p,   v = 1/(8 pi) sum_p T(y, x_p) q_p n_p w_p,
 * which is accurate only where no source lies within the near radius (paper section 3.3).  Pairs
 * inside the near radius are left out and the target is reported: the next sr_check returns
 * SR_ENEAR.  Direct far-field sum whatever far_method says.  layers as sr_eval (SR_HOST accepted);
 * y (m,3); u (m,3) if SR_SL, v (m,3) if SR_DL; 0 <= m <= sr_max_targets(). */
sr_status sr_eval_far(sr_ctx *c, int layers, int64_t m, const double *y, double *u, double *v, void *stream);

/* Wait for `stream` and the context's own stream, then report the targets of the evaluations since
 * the last sr_check that were treated as far from the surface while a source lay within the near
 * radius: SR_ENEAR (sr_last_error names the first such target and the call that met it), SR_OK if
 * none.  Clears the report. */
sr_status sr_check(sr_ctx *c, void *stream);

/* Largest number of targets (and of surface points) the evaluation calls accept: 2^28. */
int64_t sr_max_targets(void);

/* The smoothing table that sr_eval's near-field phase uses for targets on the surface (b = 0), built
 * on the host for inspection.  At b = 0 the extrapolation weights w_j of the three runs (eq.
 * (extrap_eqn) with I0(0) = 1/sqrt(pi), I2(0) = 1/(3 sqrt(pi))) are the same for every target, so the
 * combined smoothing factors S_k(x) = sum_j w_j s_k(x / rho_j) (eqs. (s1)-(s3); s_k = 1 beyond the
 * cut-off, section 3.2) are fixed functions of x = r/h.  The table holds
 *   g1 = S1 / x,  g2 = S2 / x^3,  g3 = S3 / x^5
 * on SR_NEAR_TABLE_INTERVALS equal intervals of [0, xmax], each as a polynomial of degree
 * SR_NEAR_TABLE_DEGREE in s in [-1/2, 1/2] (x = (i + 1/2 + s) xmax / SR_NEAR_TABLE_INTERVALS on
 * interval i).  Coefficient e of function f (0..2) on interval i is
 *   tab[((f * (D + 1) / 2 + e / 2) * NI + i) * 2 + e % 2]      (D the degree, NI the interval count).
 *   rho     the three delta/h ratios, positive and distinct (any order).
 *   cutoff  the cut-off of the smoothing functions (> 0).   xmax  > 0.
 *   tab     host array of n >= SR_NEAR_TABLE_DOUBLES doubles, written on success.
 *   maxerr  if not NULL, receives the largest error of the double-precision Horner evaluation of
 *           the table against long-double evaluations, at 17 points per interval, relative to the
 *           function's largest value.
 * sr_eval builds it with xmax = cutoff max(rho) (1 + 1e-5) (the near radius over h, widened for the
 * rounding of the pair test), once per parameter set and process, when neither per-delta outputs
 * nor the modified smoothing are asked for.
 * SR_EINVAL for NULL rho or tab, n too small, or a parameter out of range; SR_ENOCONV if the checked
 * error exceeds 5e-14 (tab is then left unchanged; sr_eval uses the closed forms for such
 * parameters).  Host only: needs no GPU. */
#define SR_NEAR_TABLE_INTERVALS 160
#define SR_NEAR_TABLE_DEGREE 7
#define SR_NEAR_TABLE_DOUBLES (SR_NEAR_TABLE_INTERVALS * 3 * (SR_NEAR_TABLE_DEGREE + 1))
sr_status sr_near_table(const double rho[3], double cutoff, double xmax, double *tab, int64_t n, double *maxerr);

/* sr_eval for callers that cannot allocate device memory: code under HIP graph capture, serving loops
 * that must not call hipMalloc, harnesses that forbid it.  The same evaluation as sr_eval (same
 * kernels, same results) on DEVICE arrays, with no per-delta outputs and no SR_HOST; the far-field
 * partial sums go to a static device array of SR_NOALLOC_SCRATCH_BYTES (48 MiB) that every GPU the
 * library runs on holds until the process ends, instead of a context buffer.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).
 *   m           0 <= m <= SR_NOALLOC_MAX_TARGETS (65536); SR_EINVAL beyond it.
 *   other arguments as sr_eval.
 * SR_ESTATE if the context's cell list and source records are not built for its current surface and
 * parameters (one sr_eval call on the context builds them; a new surface or new h, rho, cutoff or
 * precision needs another); SR_EINVAL if far_method is SR_TREE (the treecode is not supported).  A
 * new density is packed into the existing records without allocation.  Profiling is ignored: the near
 * field always runs concurrently on the context's stream, as in sr_eval.  The static array keeps the
 * last call's contents and needs no clearing (every partial sum read is written by the same call);
 * all calls on one GPU share it, so two calls that overlap in time on one GPU race, whatever their
 * contexts and streams. */
#define SR_NOALLOC_MAX_TARGETS 65536
#define SR_NOALLOC_SCRATCH_BYTES (16 * 6 * 8 * SR_NOALLOC_MAX_TARGETS)
sr_status sr_eval_noalloc(sr_ctx *c, int layers, int64_t m, const double *y, const double *x0, const double *n0,
                          const double *b, const double *f0, const double *q0, double *u, double *v, void *stream);

/* Per-phase timing.  While profiling is on, every sr_eval runs its phases one after the other on
 * its stream (not concurrently) and records HIP events around each: SR_PHASE_FAR (the far-field
 * sum) and SR_PHASE_NEAR (near regularized sums plus extrapolation).  sr_get_profile waits for the recorded events, writes the accumulated
 * milliseconds per phase to ms[0..SR_NPHASES-1] and the number of recorded evaluations to *evals
 * (an evaluation of more than 2^20 targets counts once per chunk), and clears the record. */
enum { SR_PHASE_FAR = 0, SR_PHASE_NEAR = 1, SR_NPHASES = 2 };
sr_status sr_set_profiling(sr_ctx *c, int on);
sr_status sr_get_profile(sr_ctx *c, double *ms, int64_t *evals);

/* Work of the treecode far field (section 3.4, eq. (MAC)) for m targets y (HOST pointer, (m,3)
 * FP64): *proxy_pairs receives the number of target-proxy interactions (every accepted cluster
 * contributes (p+1)^3 per target), *leaf_pairs the number of target-point pairs summed directly at
 * leaves (near pairs included: the kernel visits them and skips their contribution) and, if
 * cluster_points is not NULL, *cluster_points the number of points inside the accepted clusters
 * (so cluster_points + leaf_pairs = m N).  Computed on the host with the kernels' acceptance test,
 * for measurement.  SR_ESTATE unless far_method is SR_TREE and a previous sr_eval built the tree
 * for the current parameters; SR_EINVAL for NULL pointers or m < 0. */
sr_status sr_tree_work(sr_ctx *c, int64_t m, const double *y, int64_t *proxy_pairs, int64_t *leaf_pairs,
                       int64_t *cluster_points);

/* ---------------------------------------------------------------------------------------------
 * Rigid spheres in Stokes flow: the completed double-layer equation for the exterior flow past
 * rigid spheres (Power & Miranda, SIAM J. Appl. Math. 47 (1987)), with every layer integral
 * evaluated by sr_eval (double layer; paper eqs. (Stokes_DL2), (extrap_eqn)):
 *
 *   (A q)(x) = -1/2 q(x) + sum_m DL_m[q_m](x) + sum_m C_m(x),          x on sphere b,
 *   C_m(x)   = (1/8 pi) [ S(x - c_m) F_m + L_m x (x - c_m) / |x - c_m|^3 ],
 *   F_m = sum_p q_p w_p,  L_m = sum_p (x_p - c_m) x q_p w_p   (sums over sphere m),
 *
 * where DL_m of a sphere's own points is the on-surface value (chi = 1/2) and of other points the
 * nearly singular exterior value with q(x0) interpolated on the quadrature grid (tensor Lagrange
 * on one coordinate family, 6 x 6 points (O(h^6)), else 5, 4, 3, 2 per axis where the sheet has no
 * wider stencil).  A q = U_b + Omega_b x (x - c_b)
 * is the rigid-motion problem.  Unknowns and targets: the quadrature points of all spheres, sphere
 * by sphere, (ntot,3).  The quadrature must be the grid-line quadrature of paper section 2.2 with
 * the parameters' h, generated in each sphere's frame centred at its centre. */
typedef struct sr_rigid sr_rigid;

sr_status sr_rigid_create(sr_rigid **out, int device);
sr_status sr_rigid_destroy(sr_rigid *r);
/* Parameters of every sphere's evaluator (precision, far method, h, rho, cutoff, treecode). */
sr_status sr_rigid_set_params(sr_rigid *r, const sr_params *p);
/* nsph spheres (1..64): centres (nsph,3), radii (nsph) and point counts (nsph) on the HOST; points
 * x, normals nrm (ntot,3) and weights w (ntot) on the device, concatenated sphere by sphere.
 * Builds the evaluators, closest points and interpolation stencils; synchronizes `stream`. */
sr_status sr_rigid_set_spheres(sr_rigid *r, int nsph, const double *centers, const double *radii,
                               const int64_t *counts, const double *x, const double *nrm, const double *w,
                               void *stream);
/* rhs (ntot,3, device) = U_b + Omega_b x (x - c_b); motion (nsph,6) = (U, Omega) per sphere, HOST. */
sr_status sr_rigid_rhs(sr_rigid *r, const double *motion, double *rhs, void *stream);
/* out = A q (device arrays (ntot,3)). */
sr_status sr_rigid_matvec(sr_rigid *r, const double *q, double *out, void *stream);
/* Replace the operator by A q = a_id q + a_dl sum_m DL_m[q] (+ the completion terms if completion != 0).
 * Default: -1/2, 1, 1 (rigid spheres).  The drops of paper section 4.3 (eq. (IE-2Surf), viscosity
 * ratio lambda, 1/(4 pi) integrals = twice the layers here) use lambda + 1, -2 (lambda - 1), 0. */
sr_status sr_rigid_set_operator(sr_rigid *r, double a_id, double a_dl, int completion);
/* out (ntot,3) = sum_m SL_m[f_m] at every point (f (ntot,3), device): own points on the surface, other
 * points nearly singular with f(x0) interpolated by the same stencils as q(x0). */
sr_status sr_rigid_single_layer(sr_rigid *r, const double *f, double *out, void *stream);
/* Solve A x = rhs by restarted GMRES (device arrays).  x_is_guess != 0: x holds the initial guess,
 * else the iteration starts from 0.  Stops when the relative residual estimate |rhs - A x| / |rhs|
 * <= tol or after maxit matrix-vector products.  *iters = Arnoldi matrix-vector products;
 * *relres = the recomputed true relative residual.  SR_ENOCONV if not converged (x holds the last
 * iterate).  Synchronizes `stream`. */
sr_status sr_rigid_solve(sr_rigid *r, const double *rhs, double *x, int x_is_guess, double tol, int maxit,
                         int restart, int *iters, double *relres, void *stream);
/* Solve A x = rhs by iterative refinement: outer residuals rhs - A x with the operator evaluated in
 * FP64 with the direct far field (SR_FP64, SR_DIRECT evaluators, built on the first call), corrections
 * from restarted GMRES with the parameters' precision and far-field method, each reducing the residual by the factor max(inner_tol, tol |rhs| / (2 |r|))
 * (at most 0.5; 0 < inner_tol < 1, about 1e-6 suits SR_MIXED), so a pass stops once the outer
 * tolerance is within reach.  Use it
 * with SR_MIXED parameters when tol lies below the mixed operator's own error (about 1e-7 relative).
 * x_is_guess != 0: x holds the initial guess; a guess whose FP64 residual is not below |rhs| (or
 * is not finite) is replaced by zero.
 * Stops when the FP64 relative residual <= tol or after maxit inner matrix-vector products.
 * *iters = inner Arnoldi products, *outer = corrections applied, *relres = the final FP64 relative
 * residual.  SR_ENOCONV if not converged (x holds the last iterate).  Synchronizes `stream`. */
sr_status sr_rigid_solve_refined(sr_rigid *r, const double *rhs, double *x, int x_is_guess, double tol,
                                 double inner_tol, int maxit, int restart, int *iters, int *outer, double *relres,
                                 void *stream);
/* Exterior flow u (m,3) at points y (m,3) outside every sphere: sum_m DL_m[q_m] (chi = 0) + C_m.
 * Synchronizes `stream`. */
sr_status sr_rigid_velocity(sr_rigid *r, const double *q, int64_t m, const double *y, double *u, void *stream);
/* Message describing the last sr_rigid_* or sr_prolong_* failure on this thread. */
const char *sr_rigid_last_error(void);

/* Coarse-to-fine interpolation of densities on spheres (the warm start computes the density on a
 * coarse quadrature and the solve needs it on a fine one).  Each fine point's value is the tensor
 * Lagrange interpolant on the coarse grid of one coordinate family (6 x 6 points, else narrower;
 * the family with the largest |n_i| whose stencil exists), as for q(x0) above.
 * centers (nsph,3), radii, counts_c, counts_f on the HOST; xc, nc (coarse points and normals,
 * NC = sum counts_c) and xf (fine points, NF = sum counts_f) on the device, sphere by sphere, each
 * sphere's coarse set being the grid-line quadrature with spacing hc in its own frame.  Synchronizes
 * `stream`.  sr_prolong_apply: qf (NF,3) = interpolation of qc (NC,3), device arrays. */
typedef struct sr_prolong sr_prolong;
sr_status sr_prolong_create(sr_prolong **out, int device, int nsph, const double *centers, const double *radii,
                            double hc, const int64_t *counts_c, const double *xc, const double *nc,
                            const int64_t *counts_f, const double *xf, void *stream);
sr_status sr_prolong_apply(sr_prolong *p, const double *qc, double *qf, void *stream);
sr_status sr_prolong_destroy(sr_prolong *p);

/* ---------------------------------------------------------------------------------------------
 * Warm-start network for the rigid-sphere solve: gap g and the 12 motion parameters m (U, Omega of
 * sphere 1, then of sphere 2) -> the density at nout coarse unknowns (3 per coarse point).  The
 * density is linear in m, so the network is too:
 *   gt = (ln g - g_mid) / g_half;  h1 = tanh(W1 gt + b1);  h2 = tanh(W2 h1 + b2);  h3 = tanh(W3 h2 + b3)
 *   a4 = W4 h3 + b4 (12 width);  z_w = sum_k a4[12 w + k] m_k;  o = Wh z;  q = s o (s per output)
 * Matrix products run on BF16 matrix cores with FP32 accumulation; each FP32 operand is split into
 * BF16 hi + lo + lo2 (the whole FP32 significand); `passes` = 3 (default) sums hi*hi + hi*lo + lo*hi
 * (about 16 significant bits), passes = 6 adds lo*lo + hi*lo2 + lo2*hi (about 24 bits, twice the
 * matrix-core work), passes = 1 uses hi*hi only.
 * Training: loss = mean over batch and outputs of (o - y/s)^2; Adam (beta 0.9, 0.999, eps 1e-8)
 * on FP32 master weights.
 * Parameters: one FP32 vector, blocks in the order W1 (width,1), b1, W2 (width,width), b2, W3, b3,
 * W4 (12 width, width), b4 (12 width), Wh (nout, width), matrices row-major (row = output unit);
 * sr_mlp_num_params gives its length.  Arrays are device pointers unless noted; gap (batch),
 * motion (batch,12) and y (batch,nout) are FP64.  In the training calls gap, motion and y hold nrows
 * rows and idx (batch, int64, device) selects the batch's rows (NULL: rows 0..batch-1), so a data
 * set can stay resident; indices outside [0, nrows) are rejected (SR_EINVAL).  Calls on one network
 * must not overlap. */
typedef struct sr_mlp sr_mlp;
int64_t sr_mlp_num_params(int width, int64_t nout);
/* width: multiple of 32 in 32..4096; max_batch 1..4096. */
sr_status sr_mlp_create(sr_mlp **out, int device, int width, int64_t nout, int max_batch);
sr_status sr_mlp_destroy(sr_mlp *net);
/* passes 1, 3 or 6; input normalization g_mid, g_half > 0 of ln g (defaults: ln 0.02 .. ln 0.2 -> -1 .. 1,
 * g_mid = -2.7607, g_half = 1.1513).  The gap must be > 0. */
sr_status sr_mlp_set_options(sr_mlp *net, int passes, double g_mid, double g_half);
/* HOST parameter vector in, out.  Setting resets the Adam moments and step count, and the output
 * scale to 1 if none was set.  Synchronous. */
sr_status sr_mlp_set_params(sr_mlp *net, const float *params);
sr_status sr_mlp_get_params(sr_mlp *net, float *params);
/* Output scale s (nout, FP64 device): set it, fit it as the root mean square of each output over n
 * samples y (n,nout), or read it. */
sr_status sr_mlp_set_output_scale(sr_mlp *net, const double *s, void *stream);
sr_status sr_mlp_fit_output_scale(sr_mlp *net, int64_t n, const double *y, void *stream);
sr_status sr_mlp_get_output_scale(sr_mlp *net, double *s, void *stream);
/* o (batch,nout) FP32, standardized outputs. */
sr_status sr_mlp_forward(sr_mlp *net, int batch, const double *gap, const double *motion, float *out, void *stream);
/* q (batch,nout) FP64 = s o: the predicted density. */
sr_status sr_mlp_predict(sr_mlp *net, int batch, const double *gap, const double *motion, double *q, void *stream);
/* Gradient of the loss (FP32 device vector of sr_mlp_num_params) without an update; *loss (HOST,
 * may be NULL; if given the call synchronizes `stream`). */
sr_status sr_mlp_gradients(sr_mlp *net, int batch, const int64_t *idx, int64_t nrows, const double *gap,
                           const double *motion, const double *y, float *grad, double *loss, void *stream);
/* One Adam step with learning rate lr on the batch; *loss as above (the loss before the step). */
sr_status sr_mlp_train_step(sr_mlp *net, int batch, const int64_t *idx, int64_t nrows, const double *gap,
                            const double *motion, const double *y, float lr, double *loss, void *stream);
/* Profiling of training steps with HIP events on the step's stream: per step the phases
 * SR_MLP_PHASE_FORWARD, _BACKWARD (loss and gradients), _ADAM (the parameter update, one kernel)
 * and _COPIES (BF16 copies of the updated weights).  sr_mlp_get_profile waits for the recorded
 * events, writes the accumulated milliseconds per phase and the number of profiled steps, and
 * clears the record. */
enum { SR_MLP_PHASE_FORWARD = 0, SR_MLP_PHASE_BACKWARD = 1, SR_MLP_PHASE_ADAM = 2, SR_MLP_PHASE_COPIES = 3,
       SR_MLP_NPHASES = 4 };
sr_status sr_mlp_set_profiling(sr_mlp *net, int on);
sr_status sr_mlp_get_profile(sr_mlp *net, double *ms, int64_t *steps);
/* The matrix-product kernel alone, for testing: C (m,n) = A (m,k) B^T with B (n,k), FP32 row-major
 * device arrays, through the BF16 pieces of the operands and `passes` products.  Synchronizes `stream`. */
sr_status sr_mlp_gemm_test(int device, int passes, int m, int n, int k, const float *a, const float *b, float *c,
                           void *stream);
/* Message describing the last sr_mlp_* failure on this thread. */
const char *sr_mlp_last_error(void);

/* Message describing the last failure on this thread ("" if none). */
const char *sr_last_error(void);

/* Library build identification (static string). */
const char *sr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STOKESREG_H */

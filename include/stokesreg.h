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
 *     row-major: a "(k,3)" array holds k consecutive xyz triples; a "(k)" array k scalars.
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
    SR_ENOCONV = -6  /* an iterative solve did not reach its tolerance                      */
} sr_status;

/* Layer selection bits for sr_set_density / sr_eval. */
enum { SR_SL = 1, SR_DL = 2 };

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
    double tree_theta;  /* treecode: multipole acceptance parameter theta, MAC r_c / R <= theta   */
    int tree_leaf;      /* treecode: maximum number of points in a leaf N0 (>= 1)                 */
} sr_params;

/* Fill *p with defaults: h = 0 (must be set), rho = (2,3,4), cutoff = 6, SR_FP64, SR_DIRECT,
 * tree_degree = 8, tree_theta = 0.7, tree_leaf = 2000. */
void sr_default_params(sr_params *p);

/* Create a context on HIP device `device` (ordinal).  SR_ENODEV if it does not exist. */
sr_status sr_create(sr_ctx **out, int device);

/* Release the context and all device memory it owns.  NULL is accepted. */
sr_status sr_destroy(sr_ctx *c);

/* Set the method parameters (copied).  May be called again; a change of h, rho or cutoff rebuilds
 * the near-pair cell list at the next evaluation. */
sr_status sr_set_params(sr_ctx *c, const sr_params *p);

/* Set the surface quadrature (paper section 2.2, eq. (quadrature)): n points x (n,3), outward unit
 * normals nrm (n,3) and weights w (n).  n >= 1.  The data are copied; this call synchronizes
 * `stream` (it reads the points back to build the spatial index on the host).  Invalidates any
 * densities set before. */
sr_status sr_set_surface(sr_ctx *c, int64_t n, const double *x, const double *nrm, const double *w,
                         void *stream);

/* Set the density of one layer at the quadrature points, (n,3) in the order of sr_set_surface:
 * layer = SR_SL: the force density f of eq. (Stokes_SL); layer = SR_DL: q of eq. (Stokes_DL).
 * Copied; asynchronous on `stream`. */
sr_status sr_set_density(sr_ctx *c, int layer, const double *dens, void *stream);

/* Evaluate the extrapolated layer potentials at m targets.
 *   layers      SR_SL, SR_DL or SR_SL|SR_DL (both in one pass, sharing the pair geometry).
 *   y (m,3)     target points.
 *   x0 (m,3)    closest point on the surface to each target;  n0 (m,3) the outward unit normal there;
 *   b (m)       signed distance, y = x0 + b n0 (b > 0 outside, b < 0 inside, b == 0 on the surface).
 *               For a target farther than 6 max_j delta_j from the surface, x0 and n0 may be any
 *               point and unit vector and b any number of magnitude >= 6 max_j delta_j with the
 *               right sign: no smoothing acts there and the subtraction terms integrate to zero.
 *   f0 (m,3)    f(x0), needed if SR_SL is requested (else may be NULL);
 *   q0 (m,3)    q(x0), needed if SR_DL is requested (else may be NULL).
 *   u (m,3)     output single layer (if SR_SL);  v (m,3) output double layer incl. chi q(x0) (if SR_DL).
 *   u_delta, v_delta  optional (may be NULL): (m,3,3) regularized values before extrapolation,
 *               [target][j][component] for delta_j, 1/(8 pi) included, chi q(x0) excluded.
 * m == 0 is a no-op.  SR_ESTATE if the surface, the parameters or a requested density is not set. */
sr_status sr_eval(sr_ctx *c, int layers, int64_t m, const double *y, const double *x0, const double *n0,
                  const double *b, const double *f0, const double *q0, double *u, double *v,
                  double *u_delta, double *v_delta, void *stream);

/* Per-phase timing.  While profiling is on, every sr_eval records HIP events on its stream around
 * each phase: SR_PHASE_FAR (the far-field sum) and SR_PHASE_NEAR (near regularized sums plus
 * extrapolation).  sr_get_profile waits for the recorded events, writes the accumulated
 * milliseconds per phase to ms[0..SR_NPHASES-1] and the number of recorded evaluations to *evals,
 * and clears the record. */
enum { SR_PHASE_FAR = 0, SR_PHASE_NEAR = 1, SR_NPHASES = 2 };
sr_status sr_set_profiling(sr_ctx *c, int on);
sr_status sr_get_profile(sr_ctx *c, double *ms, int64_t *evals);

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
 * nearly singular exterior value with q(x0) interpolated on the quadrature grid (cubic, else
 * quadratic, else linear tensor Lagrange on one coordinate family).  A q = U_b + Omega_b x (x - c_b)
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
/* Solve A x = rhs by restarted GMRES (device arrays).  x_is_guess != 0: x holds the initial guess,
 * else the iteration starts from 0.  Stops when the relative residual estimate |rhs - A x| / |rhs|
 * <= tol or after maxit matrix-vector products.  *iters = Arnoldi matrix-vector products;
 * *relres = the recomputed true relative residual.  SR_ENOCONV if not converged (x holds the last
 * iterate).  Synchronizes `stream`. */
sr_status sr_rigid_solve(sr_rigid *r, const double *rhs, double *x, int x_is_guess, double tol, int maxit,
                         int restart, int *iters, double *relres, void *stream);
/* Solve A x = rhs by iterative refinement: outer residuals rhs - A x with the operator evaluated in
 * FP64 (SR_FP64 evaluators, built on the first call), corrections from restarted GMRES with the
 * parameters' precision, each solved to the relative residual inner_tol (0 < inner_tol < 1).  Use it
 * with SR_MIXED parameters when tol lies below the mixed operator's own error (about 1e-7 relative).
 * Stops when the FP64 relative residual <= tol or after maxit inner matrix-vector products.
 * *iters = inner Arnoldi products, *outer = corrections applied, *relres = the final FP64 relative
 * residual.  SR_ENOCONV if not converged (x holds the last iterate).  Synchronizes `stream`. */
sr_status sr_rigid_solve_refined(sr_rigid *r, const double *rhs, double *x, int x_is_guess, double tol,
                                 double inner_tol, int maxit, int restart, int *iters, int *outer, double *relres,
                                 void *stream);
/* Exterior flow u (m,3) at points y (m,3) outside every sphere: sum_m DL_m[q_m] (chi = 0) + C_m.
 * Synchronizes `stream`. */
sr_status sr_rigid_velocity(sr_rigid *r, const double *q, int64_t m, const double *y, double *u, void *stream);
/* Message describing the last sr_rigid_* failure on this thread. */
const char *sr_rigid_last_error(void);

/* Message describing the last failure on this thread ("" if none). */
const char *sr_last_error(void);

/* Library build identification (static string). */
const char *sr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STOKESREG_H */

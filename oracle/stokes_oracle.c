/*
 * Plain FP64 CPU oracle for the extrapolated-regularization Stokes single- and double-layer sums
 * (Siebor & Tlupova, "Localized evaluation and fast summation in the extrapolated regularization
 * method for integrals in Stokes flow", arXiv 2507.00156).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg load this library.  It shares no code, header or table with the GPU library, and the GPU
 * library never links or calls it.
 *
 * It is deliberately slow and literal: for every target and every smoothing parameter delta_j it
 * sums over ALL quadrature points with the regularized kernels written out index by index exactly as
 * printed, cuts the smoothing off for r/delta > 6, then solves the 3x3 extrapolation system by
 * Gaussian elimination.  No near/far split, no blocking, no reordering.
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *   - cut-off: the smoothing factors are set to 1 only for t = r/delta > 6 (t == 6 is regularized);
 *   - r == 0 (a target that coincides with a quadrature point): the single-layer kernel takes its
 *     limit delta_ij * 2/(sqrt(pi) delta); the double-layer term is 0 (x_hat = 0, b = 0, q - q0 = 0);
 *   - |b| >= 6 * max_j delta_j: every quadrature point is beyond the cut-off for every delta_j, so the
 *     three regularized values coincide and the extrapolated value is taken as that common value
 *     (the 3x3 matrix is then numerically singular because I0, I2 underflow);
 *   - chi = 1 for b < 0 (inside), 0 for b > 0 (outside), 1/2 for b == 0 (on the surface).
 *
 * Array layout: row-major (K,3) for vectors, (K,) for scalars, all double, caller-owned.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;

/* Smoothing factors, paper section 2, eqs. (s1)-(s3):
 *   s1(t) = erf t
 *   s2(t) = erf t - (2/sqrt(pi)) t e^{-t^2}
 *   s3(t) = erf t - (2/sqrt(pi)) (t + (2/3) t^3) e^{-t^2}
 * and section 3.2: s1 = s2 = s3 = 1 for t > 6. */
void orc_smoothing(double t, double s[3])
{
    if (t > 6.0) {
        s[0] = s[1] = s[2] = 1.0;
        return;
    }
    double e = exp(-t * t);
    double c = 2.0 / sqrt(PI);
    s[0] = erf(t);
    s[1] = erf(t) - c * t * e;
    s[2] = erf(t) - c * (t + (2.0 / 3.0) * t * t * t) * e;
}

/* Paper section 2, eq. (I0): I0(lambda) = e^{-lambda^2}/sqrt(pi) - |lambda| erfc|lambda|. */
double orc_I0(double lam)
{
    double a = fabs(lam);
    return exp(-lam * lam) / sqrt(PI) - a * erfc(a);
}

/* Paper section 2, eq. (I2): I2(lambda) = (2/3) ((1/2 - lambda^2) e^{-lambda^2}/sqrt(pi) + |lambda|^3 erfc|lambda|). */
double orc_I2(double lam)
{
    double a = fabs(lam);
    return (2.0 / 3.0) * ((0.5 - lam * lam) * exp(-lam * lam) / sqrt(PI) + a * a * a * erfc(a));
}

/* Paper section 2, eq. (extrap_eqn): for the three smoothing parameters delta_j = rho_j h,
 *     u + c1 rho_j I0(lambda_j) + c2 rho_j^3 I2(lambda_j) = u^{delta_j},   lambda_j = b / delta_j,
 * solved for (u, c1, c2) separately for each of the three velocity components.
 * ud[j*3 + i] = component i at delta_j;  u[i] = extrapolated component i.
 * Gaussian elimination with partial pivoting on the 3x3 system.  Returns 0, or -1 if singular. */
int orc_extrapolate(double b, double h, const double rho[3], const double ud[9], double u[3])
{
    double rmax = rho[0];
    for (int j = 1; j < 3; ++j)
        if (rho[j] > rmax) rmax = rho[j];
    if (fabs(b) >= 6.0 * rmax * h) { /* all three regularized sums coincide (see header) */
        for (int i = 0; i < 3; ++i) u[i] = ud[i];
        return 0;
    }
    double A[3][3], B[3][3];
    for (int j = 0; j < 3; ++j) {
        double lam = b / (rho[j] * h);
        A[j][0] = 1.0;
        A[j][1] = rho[j] * orc_I0(lam);
        A[j][2] = rho[j] * rho[j] * rho[j] * orc_I2(lam);
        for (int i = 0; i < 3; ++i) B[j][i] = ud[j * 3 + i];
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col) {
            for (int k = 0; k < 3; ++k) {
                double t = A[col][k]; A[col][k] = A[piv][k]; A[piv][k] = t;
                t = B[col][k]; B[col][k] = B[piv][k]; B[piv][k] = t;
            }
        }
        for (int r = col + 1; r < 3; ++r) {
            double f = A[r][col] / A[col][col];
            for (int k = col; k < 3; ++k) A[r][k] -= f * A[col][k];
            for (int k = 0; k < 3; ++k) B[r][k] -= f * B[col][k];
        }
    }
    /* back substitution; only the first unknown (u) is needed, but solve fully for clarity */
    for (int i = 0; i < 3; ++i) {
        double X[3];
        for (int r = 2; r >= 0; --r) {
            double s = B[r][i];
            for (int k = r + 1; k < 3; ++k) s -= A[r][k] * X[k];
            X[r] = s / A[r][r];
        }
        u[i] = X[0];
    }
    return 0;
}

/* Regularized single layer at one delta, paper eqs. (Stokes_SL2) and (Sreg):
 *   u_i^delta(y) = (1/8pi) sum_p S^delta_ij(y, x_p) [f_j(x_p) - f_k(x0) n_k(x0) n_j(x_p)] w_p,
 *   S^delta_ij = delta_ij s1(r/delta)/r + (y_i - x_i)(y_j - x_j) s2(r/delta)/r^3.
 * out: (m,3). */
void orc_sl_delta(int64_t n, const double *x, const double *nrm, const double *w, const double *f,
                  int64_t m, const double *y, const double *n0, const double *f0, double delta,
                  double *out)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t it = 0; it < m; ++it) {
        const double *yt = y + 3 * it;
        double c = 0.0; /* f_k(x0) n_k(x0) */
        for (int k = 0; k < 3; ++k) c += f0[3 * it + k] * n0[3 * it + k];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < n; ++p) {
            double d[3], g[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = yt[k] - x[3 * p + k];
                g[k] = (f[3 * p + k] - c * nrm[3 * p + k]) * w[p];
            }
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r == 0.0) { /* limit of s1(r/delta)/r; the d d s2/r^3 term vanishes */
                for (int i = 0; i < 3; ++i) acc[i] += 2.0 / (sqrt(PI) * delta) * g[i];
                continue;
            }
            double s[3];
            orc_smoothing(r / delta, s);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double S = (i == j ? 1.0 : 0.0) * s[0] / r + d[i] * d[j] * s[1] / (r * r * r);
                    acc[i] += S * g[j];
                }
        }
        for (int i = 0; i < 3; ++i) out[3 * it + i] = acc[i] / (8.0 * PI);
    }
}

/* Regularized double layer at one delta, WITHOUT the chi q(x0) term, paper eqs. (Stokes_DL2),
 * (Treg) and (Tsplit):
 *   v_i^delta(y) = (1/8pi) sum_p T^delta_ijk [q_j(x_p) - q_j(x0)] n_k(x_p) w_p,
 *   T^delta_ijk = -6 ( t1_ijk s2(t)/r^3 + (t2_ijk - (r^2 - b^2) t1_ijk) s3(t)/r^5 ),
 *   t1_ijk = b n_i n_j n_k - (xh_i n_j n_k + n_i xh_j n_k + n_i n_j xh_k),
 *   t2_ijk = b (xh_i xh_j n_k + xh_i n_j xh_k + n_i xh_j xh_k) - xh_i xh_j xh_k,
 * with n = n0 (normal at the closest point x0) and xh = x_p - x0.  out: (m,3). */
void orc_dl_delta(int64_t n, const double *x, const double *nrm, const double *w, const double *q,
                  int64_t m, const double *y, const double *x0, const double *n0, const double *b,
                  const double *q0, double delta, double *out)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t it = 0; it < m; ++it) {
        const double *yt = y + 3 * it;
        const double *nn = n0 + 3 * it;
        double bb = b[it];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < n; ++p) {
            double d[3], xh[3], a[3], mw[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = yt[k] - x[3 * p + k];
                xh[k] = x[3 * p + k] - x0[3 * it + k];
                a[k] = q[3 * p + k] - q0[3 * it + k];
                mw[k] = nrm[3 * p + k] * w[p];
            }
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r == 0.0) continue; /* xh = 0, b = 0 and q - q0 = 0: the term vanishes */
            double s[3];
            orc_smoothing(r / delta, s);
            double r3 = r * r * r, r5 = r3 * r * r;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    for (int k = 0; k < 3; ++k) {
                        double t1 = bb * nn[i] * nn[j] * nn[k]
                                  - (xh[i] * nn[j] * nn[k] + nn[i] * xh[j] * nn[k] + nn[i] * nn[j] * xh[k]);
                        double t2 = bb * (xh[i] * xh[j] * nn[k] + xh[i] * nn[j] * xh[k] + nn[i] * xh[j] * xh[k])
                                  - xh[i] * xh[j] * xh[k];
                        double T = -6.0 * (t1 * s[1] / r3 + (t2 - (r * r - bb * bb) * t1) * s[2] / r5);
                        acc[i] += T * a[j] * mw[k];
                    }
        }
        for (int i = 0; i < 3; ++i) out[3 * it + i] = acc[i] / (8.0 * PI);
    }
}

/* Extrapolated single layer at targets: the three regularized sums, then eq. (extrap_eqn).
 * out: (m,3) extrapolated u; out_delta (optional, may be NULL): (m,3,3) as [target][j][i]. */
int orc_sl(int64_t n, const double *x, const double *nrm, const double *w, const double *f,
           int64_t m, const double *y, const double *x0, const double *n0, const double *b,
           const double *f0, double h, const double rho[3], double *out, double *out_delta,
           double *scratch /* 9*m */)
{
    (void)x0;
    for (int j = 0; j < 3; ++j) {
        orc_sl_delta(n, x, nrm, w, f, m, y, n0, f0, rho[j] * h, scratch + 3 * m * j);
    }
    int bad = 0;
    for (int64_t it = 0; it < m; ++it) {
        double ud[9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) ud[3 * j + i] = scratch[3 * m * j + 3 * it + i];
        if (out_delta) memcpy(out_delta + 9 * it, ud, sizeof ud);
        if (orc_extrapolate(b[it], h, rho, ud, out + 3 * it)) bad = 1;
    }
    return bad ? -1 : 0;
}

/* Extrapolated double layer at targets, eqs. (Stokes_DL2), (extrap_eqn), plus chi(y) q(x0). */
int orc_dl(int64_t n, const double *x, const double *nrm, const double *w, const double *q,
           int64_t m, const double *y, const double *x0, const double *n0, const double *b,
           const double *q0, double h, const double rho[3], double *out, double *out_delta,
           double *scratch /* 9*m */)
{
    for (int j = 0; j < 3; ++j) {
        orc_dl_delta(n, x, nrm, w, q, m, y, x0, n0, b, q0, rho[j] * h, scratch + 3 * m * j);
    }
    int bad = 0;
    for (int64_t it = 0; it < m; ++it) {
        double ud[9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) ud[3 * j + i] = scratch[3 * m * j + 3 * it + i];
        if (out_delta) memcpy(out_delta + 9 * it, ud, sizeof ud);
        if (orc_extrapolate(b[it], h, rho, ud, out + 3 * it)) bad = 1;
        double chi = b[it] < 0.0 ? 1.0 : (b[it] > 0.0 ? 0.0 : 0.5);
        for (int i = 0; i < 3; ++i) out[3 * it + i] += chi * q0[3 * it + i];
    }
    return bad ? -1 : 0;
}

/* Plain (unregularized, unsubtracted) layer sums, paper eqs. (Stokes_SL), (Stokes_DL) with the
 * quadrature of eq. (quadrature).  Used only for targets far from the surface, where the kernels
 * are smooth and the quadrature alone is accurate (brute force at a finer h checks the oracle). */
void orc_plain(int64_t n, const double *x, const double *nrm, const double *w, const double *f,
               const double *q, int64_t m, const double *y, double *out_sl, double *out_dl)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t it = 0; it < m; ++it) {
        double us[3] = {0, 0, 0}, ud[3] = {0, 0, 0};
        for (int64_t p = 0; p < n; ++p) {
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = y[3 * it + k] - x[3 * p + k];
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double S = (i == j ? 1.0 : 0.0) / r + d[i] * d[j] / (r * r * r);
                    us[i] += S * f[3 * p + j] * w[p];
                    for (int k = 0; k < 3; ++k) {
                        double T = -6.0 * d[i] * d[j] * d[k] / (r * r * r * r * r);
                        ud[i] += T * q[3 * p + j] * nrm[3 * p + k] * w[p];
                    }
                }
        }
        for (int i = 0; i < 3; ++i) {
            out_sl[3 * it + i] = us[i] / (8.0 * PI);
            out_dl[3 * it + i] = ud[i] / (8.0 * PI);
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

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
 *   - small t (< 0.2): s1, s2, s3 from their Maclaurin series (the printed differences cancel: s2 ~ t^3,
 *     s3 ~ t^5); needed where two quadrature points of different families coincide up to rounding;
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
#include <stdlib.h>
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
    double c = 2.0 / sqrt(PI);
    if (t < 0.2) {
        /* The same functions from the Maclaurin series of erf and exp, free of the cancellation of
         * the differences above (s2 ~ t^3, s3 ~ t^5):
         *   s1 = c sum_n (-1)^n t^(2n+1) / (n! (2n+1))
         *   s2 = c t^3 sum_n (-1)^n 2 t^(2n) / (n! (2n+3))
         *   s3 = c t^5 sum_n (-1)^n 4 t^(2n) / (3 n! (2n+5))
         * 12 terms: the next term is below 1e-20 relative for t < 0.2. */
        double a1 = 0.0, a2 = 0.0, a3 = 0.0, p = 1.0; /* p = (-1)^n t^(2n) / n! */
        for (int n = 0; n < 12; ++n) {
            a1 += p / (2 * n + 1);
            a2 += 2.0 * p / (2 * n + 3);
            a3 += 4.0 * p / (3.0 * (2 * n + 5));
            p *= -t * t / (n + 1);
        }
        s[0] = c * t * a1;
        s[1] = c * t * t * t * a2;
        s[2] = c * t * t * t * t * t * a3;
        return;
    }
    double e = exp(-t * t);
    s[0] = erf(t);
    s[1] = erf(t) - c * t * e;
    s[2] = erf(t) - c * (t + (2.0 / 3.0) * t * t * t) * e;
}

/* Paper section 2.1 (evaluation on the surface): the modified smoothing functions
 *   s1#(t) = erf t + (2/(3 sqrt(pi))) (5t - 2t^3) e^{-t^2}
 *   s2#(t) = erf t - (2/(3 sqrt(pi))) (3t - 14t^3 + 4t^5) e^{-t^2}
 *   s3#(t) = erf t - (2/(9 sqrt(pi))) (9t + 6t^3 - 4t^5) e^{-t^2}
 * that give O(delta^5) on the surface with one delta; 1 for t > 6 as in section 3.2. */
void orc_smoothing_sharp(double t, double s[3])
{
    if (t > 6.0) {
        s[0] = s[1] = s[2] = 1.0;
        return;
    }
    double c = 2.0 / sqrt(PI);
    if (t < 0.2) {
        /* Maclaurin series: with e^{-t^2} = sum_m (-1)^m t^(2m) / m! and
         * erf t = c sum_n (-1)^n t^(2n+1) / (n! (2n+1)), the coefficient of c t^(2n+1) is
         *   s1#: E_n + (5 X_n - 2 X_{n-1}) / 3,
         *   s2#: E_n - (3 X_n - 14 X_{n-1} + 4 X_{n-2}) / 3,
         *   s3#: E_n - (9 X_n + 6 X_{n-1} - 4 X_{n-2}) / 9,
         * E_n = (-1)^n / (n! (2n+1)), X_j = (-1)^j / j! (0 for j < 0).  The first term of s2# and the
         * first two of s3# vanish exactly (s2# ~ t^3, s3# ~ t^5) and are left out. */
        double X[16], a1 = 0.0, a2 = 0.0, a3 = 0.0, tp = t; /* tp = t^(2n+1) */
        X[0] = 1.0;
        for (int j = 1; j < 16; ++j) X[j] = -X[j - 1] / j;
        for (int n = 0; n < 14; ++n) {
            const double E = X[n] / (2 * n + 1);
            const double x1 = n >= 1 ? X[n - 1] : 0.0, x2 = n >= 2 ? X[n - 2] : 0.0;
            a1 += (E + (5.0 * X[n] - 2.0 * x1) / 3.0) * tp;
            if (n >= 1) a2 += (E - (3.0 * X[n] - 14.0 * x1 + 4.0 * x2) / 3.0) * tp;
            if (n >= 2) a3 += (E - (9.0 * X[n] + 6.0 * x1 - 4.0 * x2) / 9.0) * tp;
            tp *= t * t;
        }
        s[0] = c * a1;
        s[1] = c * a2;
        s[2] = c * a3;
        return;
    }
    double e = exp(-t * t), t3 = t * t * t, t5 = t3 * t * t;
    s[0] = erf(t) + (c / 3.0) * (5.0 * t - 2.0 * t3) * e;
    s[1] = erf(t) - (c / 3.0) * (3.0 * t - 14.0 * t3 + 4.0 * t5) * e;
    s[2] = erf(t) - (c / 9.0) * (9.0 * t + 6.0 * t3 - 4.0 * t5) * e;
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
static void sl_delta_kind(int64_t n, const double *x, const double *nrm, const double *w, const double *f,
                          int64_t m, const double *y, const double *n0, const double *f0, double delta,
                          int sharp, double *out)
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
            if (r == 0.0) { /* limit of s1(r/delta)/r (2/sqrt(pi), or 16/(3 sqrt(pi)) for s1#) / delta;
                               the d d s2/r^3 term vanishes */
                const double lim = (sharp ? 16.0 / 3.0 : 2.0) / (sqrt(PI) * delta);
                for (int i = 0; i < 3; ++i) acc[i] += lim * g[i];
                continue;
            }
            double s[3];
            if (sharp)
                orc_smoothing_sharp(r / delta, s);
            else
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

void orc_sl_delta(int64_t n, const double *x, const double *nrm, const double *w, const double *f,
                  int64_t m, const double *y, const double *n0, const double *f0, double delta,
                  double *out)
{
    sl_delta_kind(n, x, nrm, w, f, m, y, n0, f0, delta, 0, out);
}

/* On-surface single layer with the modified smoothing (section 2.1): the regularized sum of eqs.
 * (Stokes_SL2), (Sreg) with s1#, s2# at one delta, no extrapolation.  Targets y on the surface
 * (y = x0), n0 their normals, f0 = f(y).  out: (m,3). */
void orc_sl_sharp(int64_t n, const double *x, const double *nrm, const double *w, const double *f,
                  int64_t m, const double *y, const double *n0, const double *f0, double delta,
                  double *out)
{
    sl_delta_kind(n, x, nrm, w, f, m, y, n0, f0, delta, 1, out);
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

/* On-surface double layer with the modified smoothing (section 2.1): the stresslet of eq. (Stresslet)
 * with its factor 1/r^5 replaced by s3#(r/delta)/r^5 (eq. (Treg) with s3 -> s3#), at one delta,
 * applied to the subtracted density of eq. (Stokes_DL1), plus q(y)/2 (chi = 1/2 on the surface):
 *   v_i(y) = (1/8pi) sum_p -6 d_i d_j d_k s3#(r/delta)/r^5 [q_j(x_p) - q_j(y)] n_k(x_p) w_p + q_i(y)/2,
 * d = y - x_p.  (The split of eq. (Tsplit) serves the extrapolated off-surface values: on the surface
 * its t1 part is multiplied by s2 - s3, which vanishes for the original factors only.)  out: (m,3). */
void orc_dl_sharp(int64_t n, const double *x, const double *nrm, const double *w, const double *q,
                  int64_t m, const double *y, const double *n0, const double *q0, double delta, double *out)
{
    (void)n0;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t it = 0; it < m; ++it) {
        const double *yt = y + 3 * it;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < n; ++p) {
            double d[3], a[3], mw[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = yt[k] - x[3 * p + k];
                a[k] = q[3 * p + k] - q0[3 * it + k];
                mw[k] = nrm[3 * p + k] * w[p];
            }
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r == 0.0) continue; /* d = 0 and q - q0 = 0: the term vanishes */
            double s[3];
            orc_smoothing_sharp(r / delta, s);
            double r5 = r * r * r * r * r;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    for (int k = 0; k < 3; ++k) acc[i] += -6.0 * d[i] * d[j] * d[k] * s[2] / r5 * a[j] * mw[k];
        }
        for (int i = 0; i < 3; ++i) out[3 * it + i] = acc[i] / (8.0 * PI) + 0.5 * q0[3 * it + i];
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

/* ------------------------------------------------------------------------------------------------
 * Treecode far field, paper section 3.4 (kernel-independent treecode with barycentric Lagrange
 * interpolation at Chebyshev points), evaluated literally per target as the paper describes: start
 * at the root; if the MAC r_c / R <= theta holds the cluster interacts through its Chebyshev proxy
 * points (eq. (particle-cluster-KITC)) with the ORIGINAL kernels; otherwise a leaf is summed
 * directly with the regularized kernels for the three deltas (t > 6 -> s = 1), and a non-leaf is
 * replaced by its children.  Then the 3x3 extrapolation as in orc_sl / orc_dl.
 *
 * Readings of points the paper leaves open (also in the design notes):
 *   - octree: a cluster with more than N0 points is split at the midpoint of its box into 8
 *     octants (a point goes to the upper half of an axis when x >= mid); empty octants are dropped;
 *     a cluster whose points all coincide (one octant only) is not split;
 *     every cluster's box is the bounding box of its points; children are visited in octant order
 *     (bit 0: x upper, bit 1: y upper, bit 2: z upper);
 *   - cluster radius r_c = half the box diagonal, R = distance from the target to the box centre;
 *   - the MAC additionally requires the box to lie farther than the near radius 6 max_j delta_j
 *     from the target (squared distance to the box > (6 max delta)^2); otherwise pairs that need
 *     regularization would be approximated with the singular kernels.  The MAC is evaluated on
 *     squared quantities: r_c^2 <= theta^2 R^2;
 *   - Chebyshev points of the second kind s_k = c + (h/2) cos(k pi / p), k = 0..p per axis, with the
 *     barycentric weights (-1)^k, halved at k = 0 and k = p; a coordinate equal to a node gets
 *     L = 1 there and 0 elsewhere; an axis of zero extent puts all weight on k = 0;
 *   - modified weights for the 15 channels f w (3), n w (3), q_j n_k w (9); the single layer uses
 *     F - (f(x0).n0) N, the double layer Q - q(x0) (x) N (eq. (mod_weights) and the text after it).
 * ------------------------------------------------------------------------------------------------ */
#include <stdlib.h>

typedef struct {
    int64_t begin, end;    /* range in the tree-ordered point array */
    double lo[3], hi[3];   /* bounding box of the cluster's points */
    int child[8], nchild;
} orc_node;

typedef struct {
    orc_node *nodes;
    int nnodes, cap;
    int64_t *order;        /* tree order -> caller index */
} orc_tree_t;

static int tree_push(orc_tree_t *T)
{
    if (T->nnodes == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 64;
        T->nodes = (orc_node *)realloc(T->nodes, sizeof(orc_node) * (size_t)T->cap);
    }
    memset(&T->nodes[T->nnodes], 0, sizeof(orc_node));
    return T->nnodes++;
}

static void tree_bbox(orc_tree_t *T, const double *x, int id)
{
    orc_node *nd = &T->nodes[id];
    for (int d = 0; d < 3; ++d) {
        nd->lo[d] = INFINITY;
        nd->hi[d] = -INFINITY;
    }
    for (int64_t i = nd->begin; i < nd->end; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * T->order[i] + d];
            if (v < nd->lo[d]) nd->lo[d] = v;
            if (v > nd->hi[d]) nd->hi[d] = v;
        }
}

static void tree_split(orc_tree_t *T, const double *x, int id, int64_t leaf)
{
    if (T->nodes[id].end - T->nodes[id].begin <= leaf) return;
    double mid[3];
    for (int d = 0; d < 3; ++d) mid[d] = (T->nodes[id].lo[d] + T->nodes[id].hi[d]) * 0.5;
    int64_t b = T->nodes[id].begin, e = T->nodes[id].end;
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(e - b));
    int64_t cnt[8] = {0};
    for (int64_t i = b; i < e; ++i) {
        const double *p = x + 3 * T->order[i];
        int oct = (p[0] >= mid[0]) | ((p[1] >= mid[1]) << 1) | ((p[2] >= mid[2]) << 2);
        cnt[oct]++;
    }
    int nonempty = 0;
    for (int o = 0; o < 8; ++o) nonempty += cnt[o] > 0;
    if (nonempty < 2) { /* all points coincide: the cluster cannot be split and stays a leaf */
        free(tmp);
        return;
    }
    int64_t start[8], fill[8];
    start[0] = 0;
    for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
    for (int o = 0; o < 8; ++o) fill[o] = start[o];
    for (int64_t i = b; i < e; ++i) {
        const double *p = x + 3 * T->order[i];
        int oct = (p[0] >= mid[0]) | ((p[1] >= mid[1]) << 1) | ((p[2] >= mid[2]) << 2);
        tmp[fill[oct]++] = T->order[i];
    }
    memcpy(T->order + b, tmp, sizeof(int64_t) * (size_t)(e - b));
    free(tmp);
    for (int o = 0; o < 8; ++o) {
        if (cnt[o] == 0) continue;
        int c = tree_push(T);
        T->nodes[c].begin = b + start[o];
        T->nodes[c].end = b + start[o] + cnt[o];
        tree_bbox(T, x, c);
        T->nodes[id].child[T->nodes[id].nchild++] = c;
    }
    for (int k = 0; k < T->nodes[id].nchild; ++k) tree_split(T, x, T->nodes[id].child[k], leaf);
}

/* barycentric Lagrange basis L_0..L_p at coordinate v for the Chebyshev points of [lo, hi] */
static void lagrange_1d(double v, double lo, double hi, int p, double *L)
{
    if (hi == lo) {
        for (int k = 0; k <= p; ++k) L[k] = k == 0 ? 1.0 : 0.0;
        return;
    }
    double c = 0.5 * (lo + hi), hw = 0.5 * (hi - lo), den = 0.0;
    for (int k = 0; k <= p; ++k) {
        double s = c + hw * cos(k * PI / p);
        if (v == s) {
            for (int j = 0; j <= p; ++j) L[j] = j == k ? 1.0 : 0.0;
            return;
        }
        double wk = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == p) ? 0.5 : 1.0);
        L[k] = wk / (v - s);
        den += L[k];
    }
    for (int k = 0; k <= p; ++k) L[k] /= den;
}

/* regularized single and double layer of one source at the three deltas (the sums of orc_sl_delta
 * and orc_dl_delta for one pair), added to us[j][i], vs[j][i] before the 1/(8 pi) factor */
static void pair_regularized(const double *yt, const double *x0t, const double *nn, double bb, double c,
                             const double *q0t, const double *xp, const double *np_, double wp, const double *fp,
                             const double *qp, double h, const double rho[3], double us[3][3], double vs[3][3])
{
    double d[3], g[3], xh[3], a[3], mw[3];
    for (int k = 0; k < 3; ++k) {
        d[k] = yt[k] - xp[k];
        g[k] = (fp[k] - c * np_[k]) * wp;
        xh[k] = xp[k] - x0t[k];
        a[k] = qp[k] - q0t[k];
        mw[k] = np_[k] * wp;
    }
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int jd = 0; jd < 3; ++jd) {
        double delta = rho[jd] * h;
        if (r == 0.0) {
            for (int i = 0; i < 3; ++i) us[jd][i] += 2.0 / (sqrt(PI) * delta) * g[i];
            continue;
        }
        double s[3];
        orc_smoothing(r / delta, s);
        double r3 = r * r * r, r5 = r3 * r * r;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                us[jd][i] += ((i == j ? 1.0 : 0.0) * s[0] / r + d[i] * d[j] * s[1] / r3) * g[j];
                for (int k = 0; k < 3; ++k) {
                    double t1 = bb * nn[i] * nn[j] * nn[k]
                              - (xh[i] * nn[j] * nn[k] + nn[i] * xh[j] * nn[k] + nn[i] * nn[j] * xh[k]);
                    double t2 = bb * (xh[i] * xh[j] * nn[k] + xh[i] * nn[j] * xh[k] + nn[i] * xh[j] * xh[k])
                              - xh[i] * xh[j] * xh[k];
                    vs[jd][i] += -6.0 * (t1 * s[1] / r3 + (t2 - (r * r - bb * bb) * t1) * s[2] / r5) * a[j] * mw[k];
                }
            }
    }
}

typedef struct {
    const double *x, *nrm, *w, *f, *q;
    const orc_tree_t *T;
    const double *mw;  /* modified weights: [node][proxy][15] */
    int p;
    double theta, rnear, h, rho[3];
    double mac_rnear; /* the MAC's near radius (>= rnear) */
} tree_ctx;

static void tree_visit(const tree_ctx *C, int id, const double *yt, const double *x0t, const double *nn, double bb,
                       double c, const double *q0t, double us[3][3], double vs[3][3])
{
    const orc_node *nd = &C->T->nodes[id];
    /* MAC: r_c <= theta R, and the whole box farther than the near radius (mac_rnear: a caller whose
     * near-pair test rounds may widen it, so that no source of an accepted cluster is a near pair) */
    double rc2 = 0.0, R2 = 0.0, g2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = nd->hi[d] - nd->lo[d];
        rc2 += 0.25 * e * e;
        double dc = yt[d] - 0.5 * (nd->lo[d] + nd->hi[d]);
        R2 += dc * dc;
        double gap = nd->lo[d] - yt[d] > 0.0 ? nd->lo[d] - yt[d] : (yt[d] - nd->hi[d] > 0.0 ? yt[d] - nd->hi[d] : 0.0);
        g2 += gap * gap;
    }
    if (rc2 <= C->theta * C->theta * R2 && g2 > C->mac_rnear * C->mac_rnear) {
        int np1 = C->p + 1;
        const double *W = C->mw + (size_t)id * np1 * np1 * np1 * 15;
        double su[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
        for (int k1 = 0; k1 <= C->p; ++k1)
            for (int k2 = 0; k2 <= C->p; ++k2)
                for (int k3 = 0; k3 <= C->p; ++k3) {
                    int kk[3] = {k1, k2, k3};
                    double s[3], d[3];
                    for (int dd = 0; dd < 3; ++dd) {
                        double cc = 0.5 * (nd->lo[dd] + nd->hi[dd]), hw = 0.5 * (nd->hi[dd] - nd->lo[dd]);
                        s[dd] = nd->hi[dd] == nd->lo[dd] ? nd->lo[dd] : cc + hw * cos(kk[dd] * PI / C->p);
                        d[dd] = yt[dd] - s[dd];
                    }
                    const double *g = W + ((size_t)(k1 * np1 + k2) * np1 + k3) * 15;
                    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    double r3 = r * r * r, r5 = r3 * r * r;
                    /* single layer: S_ij (F_j - c N_j) */
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            su[i] += ((i == j ? 1.0 : 0.0) / r + d[i] * d[j] / r3) * (g[j] - c * g[3 + j]);
                    /* double layer: T_ijk (Q_jk - q0_j N_k) */
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            for (int k = 0; k < 3; ++k)
                                sv[i] += -6.0 * d[i] * d[j] * d[k] / r5 * (g[6 + 3 * j + k] - q0t[j] * g[3 + k]);
                }
        for (int jd = 0; jd < 3; ++jd)
            for (int i = 0; i < 3; ++i) {
                us[jd][i] += su[i];
                vs[jd][i] += sv[i];
            }
        return;
    }
    if (nd->nchild == 0) {
        for (int64_t i = nd->begin; i < nd->end; ++i) {
            int64_t o = C->T->order[i];
            pair_regularized(yt, x0t, nn, bb, c, q0t, C->x + 3 * o, C->nrm + 3 * o, C->w[o], C->f + 3 * o,
                             C->q + 3 * o, C->h, C->rho, us, vs);
        }
        return;
    }
    for (int k = 0; k < nd->nchild; ++k) tree_visit(C, nd->child[k], yt, x0t, nn, bb, c, q0t, us, vs);
}

/* Treecode evaluation of both layers.  out_sl, out_dl: (m,3); optional out_*_delta (m,3,3).
 * mac_rnear: the radius the MAC requires a cluster's box to lie beyond; <= 0 for the near radius.
 * Returns the number of tree nodes, or -1 if an extrapolation system is singular. */
int orc_tree(int64_t n, const double *x, const double *nrm, const double *w, const double *f, const double *q,
             int64_t m, const double *y, const double *x0, const double *n0, const double *b, const double *f0,
             const double *q0, double h, const double rho[3], int p, double theta, int64_t leaf, double mac_rnear,
             double *out_sl, double *out_dl, double *out_sl_delta, double *out_dl_delta)
{
    orc_tree_t T = {0};
    T.order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) T.order[i] = i;
    int root = tree_push(&T);
    T.nodes[root].begin = 0;
    T.nodes[root].end = n;
    tree_bbox(&T, x, root);
    tree_split(&T, x, root, leaf);

    /* modified weights, eq. (mod_weights), for every cluster */
    int np1 = p + 1, nprox = np1 * np1 * np1;
    double *mw = (double *)calloc((size_t)T.nnodes * nprox * 15, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int id = 0; id < T.nnodes; ++id) {
        const orc_node *nd = &T.nodes[id];
        double L[3][17];
        for (int64_t i = nd->begin; i < nd->end; ++i) {
            int64_t o = T.order[i];
            for (int d = 0; d < 3; ++d) lagrange_1d(x[3 * o + d], nd->lo[d], nd->hi[d], p, L[d]);
            double ch[15];
            for (int j = 0; j < 3; ++j) {
                ch[j] = f[3 * o + j] * w[o];
                ch[3 + j] = nrm[3 * o + j] * w[o];
            }
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) ch[6 + 3 * j + k] = q[3 * o + j] * nrm[3 * o + k] * w[o];
            for (int k1 = 0; k1 <= p; ++k1)
                for (int k2 = 0; k2 <= p; ++k2)
                    for (int k3 = 0; k3 <= p; ++k3) {
                        double lk = L[0][k1] * L[1][k2] * L[2][k3];
                        double *g = mw + ((size_t)id * nprox + (k1 * np1 + k2) * np1 + k3) * 15;
                        for (int c = 0; c < 15; ++c) g[c] += lk * ch[c];
                    }
        }
    }
    double rmax = rho[0];
    for (int j = 1; j < 3; ++j)
        if (rho[j] > rmax) rmax = rho[j];
    tree_ctx C = {x, nrm, w, f, q, &T, mw, p, theta, 6.0 * rmax * h, h, {rho[0], rho[1], rho[2]}, 0.0};
    C.mac_rnear = mac_rnear > 0.0 ? mac_rnear : C.rnear;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t it = 0; it < m; ++it) {
        double us[3][3] = {{0}}, vs[3][3] = {{0}};
        const double *nn = n0 + 3 * it;
        double c = f0[3 * it] * nn[0] + f0[3 * it + 1] * nn[1] + f0[3 * it + 2] * nn[2];
        tree_visit(&C, root, y + 3 * it, x0 + 3 * it, nn, b[it], c, q0 + 3 * it, us, vs);
        double ud[9], vd[9];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                ud[3 * j + i] = us[j][i] / (8.0 * PI);
                vd[3 * j + i] = vs[j][i] / (8.0 * PI);
            }
        if (out_sl_delta) memcpy(out_sl_delta + 9 * it, ud, sizeof ud);
        if (out_dl_delta) memcpy(out_dl_delta + 9 * it, vd, sizeof vd);
        if (orc_extrapolate(b[it], h, rho, ud, out_sl + 3 * it)) bad |= 1;
        if (orc_extrapolate(b[it], h, rho, vd, out_dl + 3 * it)) bad |= 1;
        double chi = b[it] < 0.0 ? 1.0 : (b[it] > 0.0 ? 0.0 : 0.5);
        for (int i = 0; i < 3; ++i) out_dl[3 * it + i] += chi * q0[3 * it + i];
    }
    int nn_ = T.nnodes;
    free(mw);
    free(T.nodes);
    free(T.order);
    return bad ? -1 : nn_;
}

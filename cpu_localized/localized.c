/*
 * Paper-style localized CPU evaluation of the extrapolated single and double layers: a timing
 * baseline for the GPU path, not a checker (the tests compare the GPU with the oracle only).
 *
 * Per target (OpenMP over targets, as in the paper's section 4 runs), each source pair is classified
 * once by r <= R = cutoff * max_j delta_j (eq. (near_far), section 3.3):
 *   - far pairs: the original Stokeslet / stresslet (eqs. (Stokeslet), (Stresslet)) applied to the
 *     subtracted densities of eqs. (Stokes_SL1), (Stokes_DL1), summed once for all three deltas;
 *   - near pairs: the regularized kernels of eqs. (Sreg), (Treg), (Tsplit) at the three delta_j, with
 *     the smoothing factors (s1)-(s3) taken as 1 for r / delta > cutoff (section 3.2);
 * then u = sum_j w_j u_j with the weights of the 3 x 3 extrapolation (eqs. (extrap_eqn), (I0), (I2)),
 * w = (1, 0, 0) when |b| >= cutoff * max delta, and + chi q(x0) for the double layer.
 * Small t (< 0.2) use the Maclaurin series of s1, s2, s3; r = 0 takes the single layer's limit.
 * Built with -O2 -fopenmp, the paper's optimization level.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846;

/* s1, s2, s3 at t (eqs. (s1)-(s3)): s1 = erf t, s2 = erf t - (2/sqrt(pi)) t e^{-t^2},
 * s3 = s2 - (4/(3 sqrt(pi))) t^3 e^{-t^2}; small t from the series of erf and exp. */
static void smooth(double t, double cutoff, double *s1, double *s2, double *s3)
{
    const double c = 2.0 / sqrt(PI);
    if (t > cutoff) {
        *s1 = *s2 = *s3 = 1.0;
        return;
    }
    if (t < 0.2) {
        double a1 = 0, a2 = 0, a3 = 0, f = 1.0, t2 = t * t, p = 1.0;
        for (int k = 0; k < 14; ++k) {
            a1 += f * p / (2 * k + 1);
            a2 += 2.0 * f * p / (2 * k + 3);
            a3 += 4.0 * f * p / (3.0 * (2 * k + 5));
            f = -f / (k + 1);
            p *= t2;
        }
        *s1 = c * t * a1;
        *s2 = c * t * t2 * a2;
        *s3 = c * t * t2 * t2 * a3;
        return;
    }
    const double e = exp(-t * t), er = erf(t);
    *s1 = er;
    *s2 = er - c * t * e;
    *s3 = *s2 - (2.0 / 3.0) * c * t * t * t * e;
}

static double I0f(double l)
{
    const double a = fabs(l);
    return exp(-l * l) / sqrt(PI) - a * erfc(a);
}

static double I2f(double l)
{
    const double a = fabs(l);
    return (2.0 / 3.0) * ((0.5 - l * l) * exp(-l * l) / sqrt(PI) + a * a * a * erfc(a));
}

int loc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void loc_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Both layers at m targets: x, nrm (n,3), w (n), f, q (n,3); y, x0, n0 (m,3), b (m), f0, q0 (m,3);
 * rho[3]; outputs u, v (m,3) in the paper's normalization (1/(8 pi) included). */
void loc_eval(int64_t n, const double *x, const double *nrm, const double *w, const double *f, const double *q,
              int64_t m, const double *y, const double *x0, const double *n0, const double *b, const double *f0,
              const double *q0, double h, const double *rho, double cutoff, double *u, double *v)
{
    double dmax = 0.0;
    for (int j = 0; j < 3; ++j) dmax = fmax(dmax, rho[j] * h);
    const double R = cutoff * dmax, R2 = R * R;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t it = 0; it < m; ++it) {
        const double *yt = y + 3 * it, *xo = x0 + 3 * it, *no = n0 + 3 * it, *qo = q0 + 3 * it;
        const double bt = b[it];
        const double cf = f0[3 * it] * no[0] + f0[3 * it + 1] * no[1] + f0[3 * it + 2] * no[2];
        double fs[3] = {0, 0, 0}, fd[3] = {0, 0, 0};          /* far sums (shared by the deltas) */
        double ns[3][3] = {{0}}, nd[3][3] = {{0}};            /* near sums per delta */
        for (int64_t p = 0; p < n; ++p) {
            const double *xp = x + 3 * p, *np_ = nrm + 3 * p;
            const double wp = w[p];
            const double d[3] = {yt[0] - xp[0], yt[1] - xp[1], yt[2] - xp[2]};
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double g[3], a[3], mm[3];
            for (int k = 0; k < 3; ++k) {
                g[k] = (f[3 * p + k] - cf * np_[k]) * wp;
                a[k] = q[3 * p + k] - qo[k];
                mm[k] = np_[k] * wp;
            }
            if (r2 > R2) {
                const double r = sqrt(r2), i1 = 1.0 / r, i3 = i1 * i1 * i1, i5 = i3 * i1 * i1;
                const double dg = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
                const double da = d[0] * a[0] + d[1] * a[1] + d[2] * a[2];
                const double dm = d[0] * mm[0] + d[1] * mm[1] + d[2] * mm[2];
                for (int k = 0; k < 3; ++k) {
                    fs[k] += g[k] * i1 + d[k] * dg * i3;
                    fd[k] += d[k] * da * dm * i5;
                }
                continue;
            }
            if (r2 == 0.0) {
                for (int j = 0; j < 3; ++j)
                    for (int k = 0; k < 3; ++k) ns[j][k] += 2.0 / (sqrt(PI) * rho[j] * h) * g[k];
                continue;
            }
            const double r = sqrt(r2), i1 = 1.0 / r, i3 = i1 * i1 * i1, i5 = i3 * i1 * i1;
            const double dg = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
            /* double layer split form about x0: xh = x - x0 */
            const double xh[3] = {xp[0] - xo[0], xp[1] - xo[1], xp[2] - xo[2]};
            const double na = no[0] * a[0] + no[1] * a[1] + no[2] * a[2];
            const double nm = no[0] * mm[0] + no[1] * mm[1] + no[2] * mm[2];
            const double xa = xh[0] * a[0] + xh[1] * a[1] + xh[2] * a[2];
            const double xm = xh[0] * mm[0] + xh[1] * mm[1] + xh[2] * mm[2];
            const double xn = xh[0] * no[0] + xh[1] * no[1] + xh[2] * no[2];
            const double xx = xh[0] * xh[0] + xh[1] * xh[1] + xh[2] * xh[2];
            double t1[3], t2[3];
            for (int k = 0; k < 3; ++k) {
                t1[k] = no[k] * (bt * na * nm - xa * nm - na * xm) - xh[k] * na * nm;
                t2[k] = xh[k] * (bt * (xa * nm + na * xm) - xa * xm) + no[k] * bt * xa * xm;
            }
            const double rmb = xx - 2.0 * bt * xn;
            for (int j = 0; j < 3; ++j) {
                double s1, s2, s3;
                smooth(r / (rho[j] * h), cutoff, &s1, &s2, &s3);
                for (int k = 0; k < 3; ++k) {
                    ns[j][k] += g[k] * s1 * i1 + d[k] * dg * s2 * i3;
                    nd[j][k] += t1[k] * s2 * i3 + (t2[k] - rmb * t1[k]) * s3 * i5;
                }
            }
        }
        double wt[3] = {1.0, 0.0, 0.0};
        if (fabs(bt) < cutoff * dmax) {
            double al[3], be[3];
            for (int j = 0; j < 3; ++j) {
                const double l = bt / (rho[j] * h);
                al[j] = rho[j] * I0f(l);
                be[j] = rho[j] * rho[j] * rho[j] * I2f(l);
            }
            const double C0 = al[1] * be[2] - al[2] * be[1];
            const double C1 = al[2] * be[0] - al[0] * be[2];
            const double C2 = al[0] * be[1] - al[1] * be[0];
            const double D = C0 + C1 + C2;
            wt[0] = C0 / D;
            wt[1] = C1 / D;
            wt[2] = C2 / D;
        }
        const double chi = bt < 0.0 ? 1.0 : (bt > 0.0 ? 0.0 : 0.5);
        for (int k = 0; k < 3; ++k) {
            double us = 0.0, vd = 0.0;
            for (int j = 0; j < 3; ++j) {
                us += wt[j] * (fs[k] + ns[j][k]);
                vd += wt[j] * (-6.0 * fd[k] + nd[j][k] * -6.0);
            }
            u[3 * it + k] = us / (8.0 * PI);
            v[3 * it + k] = vd / (8.0 * PI) + chi * qo[k];
        }
    }
}

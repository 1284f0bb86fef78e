// Near-field regularized sums and extrapolation (paper sections 2 and 3.2-3.3).
//
// For each target, the pairs with r^2 <= rc2 (the same pair_r2 test as the far-field kernel, on the
// same rounded operands) are summed with the regularized kernels at the three smoothing lengths:
//   single layer, eq. (Sreg):  S^d g = g s1(t)/r + d (d.g) s2(t)/r^3,   g = (f - (f0.n0) n) w
//   double layer, eqs. (Treg), (Tsplit):
//        T^d a m = -6 [ t1 s2(t)/r^3 + (t2 - (r^2 - b^2) t1) s3(t)/r^5 ],   a = q - q0, m = n w
//        t1 = n0 (b (n0.a)(n0.m) - (xh.a)(n0.m) - (n0.a)(xh.m)) - xh (n0.a)(n0.m)
//        t2 = xh (b ((xh.a)(n0.m) + (n0.a)(xh.m)) - (xh.a)(xh.m)) + n0 b (xh.a)(xh.m),  xh = x - x0
//   (t1, t2 are the contractions of t^(1)_ijk, t^(2)_ijk with a_j m_k; r^2 - b^2 = |xh|^2 - 2 b xh.n0)
// with the smoothing factors of eqs. (s1)-(s3) set to 1 for t = r/delta > cutoff (section 3.2).
// The far-field partial sums are then added (eq. (near_far)): by this kernel, or, when it runs
// concurrently with the far-field kernel (nparts = 0), afterwards by far_add_kernel.  The three values
// are combined by the 3x3 extrapolation of eq. (extrap_eqn): u = sum_j w_j u^{delta_j}, w = e_1^T A^{-1} with rows
// A_j = [1, rho_j I0(lambda_j), rho_j^3 I2(lambda_j)], lambda_j = b/delta_j, by Cramer's rule.
// If |b| >= cutoff * max delta every pair is beyond the cut-off for every delta, the three values
// coincide and w = (1, 0, 0) (the matrix is numerically singular there).
// Double layer: + chi q0 with chi = 1, 0, 1/2 for b < 0, b > 0, b == 0 (eq. (Stokes_DL1)).
//
// Work decomposition: one wavefront per target (4 per workgroup).  The target's cell and its
// neighbours in the uniform cell grid (side >= near radius) hold every near pair; with cells in
// z-fastest order, the 27 neighbour cells are 9 contiguous ranges.  The 64 lanes test candidates 64 at
// a time (compact single- or double-precision positions; several such loads in flight per wavefront)
// and append the near ones to a per-wave ring buffer in LDS; each time it holds 64 pairs, all 64 lanes
// evaluate one pair each, so the FP64 regularized kernels run without idle lanes.  The three smoothing
// factors of a pair share one exp(-t^2) and one polynomial (no branches): s_k = 1 - exp(-t^2) P_k(t)
// with P_1 = erfcx(t), P_2 = P_1 + (2/sqrt(pi)) t, P_3 = P_2 + (4/(3 sqrt(pi))) t^3.
// When only the extrapolated values are asked for, the weights w_j are computed first and a pair
// adds K(S), S_k = sum_j w_j s_k(t_j), to one set of accumulators (the kernels are linear in s_k).
// A batch of 64 pairs skips a smoothing length when none of its pairs lies within that length's
// cut-off ball (a wavefront-uniform test).  Skipping per pair would save about 40% of the smoothing
// work, but it needs pairs sorted into per-class queues so that a batch of 64 shares its class;
// measured on MI355X, the queue bookkeeping cost more than the smoothing it saved (per-class queues:
// 27% fewer FP64 FMAs, 19% more VALU instructions in all).
// Per-lane FP64 partial sums are combined by a butterfly wavefront reduction.
// A target whose |b| selects w = (1, 0, 0) lies, by its own b, at least cutoff * max delta from the
// surface; if a source is closer than that (less a rounding margin) the caller's b is wrong and the
// near regularization it skipped was needed: the scan reports it in the context's NearFlag.
#include <math.h>

#include <type_traits>

#include "sr_erfcx_table.h"
#include "sr_internal.h"

namespace sr {

// The erfcx coefficients as device variables with external linkage: the compiler cannot fold them
// into immediates, so the polynomial reads them with scalar loads into SGPRs instead of keeping 17
// FP64 constants (34 VGPRs) live across the pair loop.  Two tables: degree 16 (|erfc error| ~6e-16)
// for the double-precision path, degree 11 (~2e-11) for the mixed-precision path, whose
// single-precision far field (relative error ~1e-7) dominates its error; 5 fewer FMAs per
// smoothing evaluation and 10 fewer scalar registers.
template <class EP>
struct ErfcxCoef {
    double c[EP::kDegree + 1];
};
template <class EP>
constexpr ErfcxCoef<EP> make_erfcx_coef()
{
    ErfcxCoef<EP> r{};
    for (int k = 0; k <= EP::kDegree; ++k) r.c[k] = EP::kC[k];
    return r;
}
__constant__ ErfcxCoef<erfcx_poly::Fp64> g_erfcx_coef = make_erfcx_coef<erfcx_poly::Fp64>();
__constant__ ErfcxCoef<erfcx_poly::Mixed> g_erfcx_coef_mixed = make_erfcx_coef<erfcx_poly::Mixed>();

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoOverSqrtPi = 1.12837916709551257389615890312154517;
constexpr double kInvSqrtPi = 0.564189583547756286948079451560772586;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// orders this wavefront's LDS accesses across lanes (no workgroup barrier needed: one wave owns the queue)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double I0f(double lam)
{
    const double a = fabs(lam);
    return exp(-lam * lam) * kInvSqrtPi - a * erfc(a);
}

__device__ __forceinline__ double I2f(double lam)
{
    const double a = fabs(lam);
    return (2.0 / 3.0) * ((0.5 - lam * lam) * exp(-lam * lam) * kInvSqrtPi + a * a * a * erfc(a));
}

// Maclaurin coefficients for t < kSeriesT: s1 = c t sum A1_n t^2n, s2 = c t^3 sum A2_n t^2n,
// s3 = c t^5 sum A3_n t^2n (c = 2/sqrt(pi)), with A1_n = (-1)^n / (n! (2n+1)),
// A2_n = (-1)^n 2 / (n! (2n+3)), A3_n = (-1)^n 4 / (3 n! (2n+5)) (series of erf and exp).
constexpr double kSeriesT = 0.2;
constexpr int kSeriesN = 12;
struct SeriesCoef {
    double a1[kSeriesN], a2[kSeriesN], a3[kSeriesN];
};
constexpr SeriesCoef make_series()
{
    SeriesCoef c{};
    double f = 1.0;  // (-1)^n / n!
    for (int n = 0; n < kSeriesN; ++n) {
        c.a1[n] = f / (2 * n + 1);
        c.a2[n] = 2.0 * f / (2 * n + 3);
        c.a3[n] = 4.0 * f / (3.0 * (2 * n + 5));
        f = -f / (n + 1);
    }
    return c;
}
__constant__ constexpr SeriesCoef kSeries = make_series();

// s1, s2, s3 at t >= 0 (eqs. (s1)-(s3)) given E = exp(-t^2), replaced by 1 for t > cutoff and by 0 for
// t < kSeriesT (the
// pairs closer than kSeriesT delta are added separately by near_pair_series, whose Maclaurin series
// keep the relative accuracy of s2 ~ t^3 and s3 ~ t^5 that the differences below would lose).
// erfcx(t) for 0 <= t <= 6.25 from the interpolating polynomial of sr_erfcx_table.h: the degree-16
// table, or with LO the mixed-precision path's degree-11 table.
template <bool LO>
__device__ __forceinline__ double erfcx_eval(double tc)
{
    using EP = std::conditional_t<LO, erfcx_poly::Mixed, erfcx_poly::Fp64>;
    const double den = tc + EP::kL;
    double inv = __builtin_amdgcn_rcp(den);
    double e = __builtin_fma(-den, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    e = __builtin_fma(-den, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    const double x = __builtin_fma(EP::kA, (tc - EP::kL) * inv, EP::kB);
    double pz;
    if constexpr (LO) {
        pz = g_erfcx_coef_mixed.c[EP::kDegree];
#pragma unroll
        for (int k = EP::kDegree - 1; k >= 0; --k) pz = __builtin_fma(pz, x, g_erfcx_coef_mixed.c[k]);
    } else {
        pz = g_erfcx_coef.c[EP::kDegree];
#pragma unroll
        for (int k = EP::kDegree - 1; k >= 0; --k) pz = __builtin_fma(pz, x, g_erfcx_coef.c[k]);
    }
    return EP::kL * inv * pz;
}

// erfc(t) = exp(-t^2) erfcx(t) (|erfc error| < 1e-15 on [0, 6.25] with the degree-16 table, 2e-11 with
// LO); beyond 6.25 exp(-t^2) < 1e-16 makes the clamped erfcx value irrelevant.
template <bool LO>
__device__ __forceinline__ void smoothing3(double t, double E, double cutoff, double &s1, double &s2, double &s3)
{
    const double R = erfcx_eval<LO>(fmin(t, 6.25));
    const double P2 = __builtin_fma(kTwoOverSqrtPi, t, R);
    const double P3 = __builtin_fma((2.0 / 3.0) * kTwoOverSqrtPi * t * t, t, P2);
    const double Ec = t > cutoff ? 0.0 : E;  // beyond the cut-off s1 = s2 = s3 = 1 exactly
    const bool ser = t < kSeriesT;
    s1 = ser ? 0.0 : __builtin_fma(-Ec, R, 1.0);
    s2 = ser ? 0.0 : __builtin_fma(-Ec, P2, 1.0);
    s3 = ser ? 0.0 : __builtin_fma(-Ec, P3, 1.0);
}

// s1, s2, s3 for t < kSeriesT from their Maclaurin series.
__device__ __forceinline__ void series3(double t, double &s1, double &s2, double &s3)
{
    const double t2 = t * t;
    double b1 = kSeries.a1[kSeriesN - 1], b2 = kSeries.a2[kSeriesN - 1], b3 = kSeries.a3[kSeriesN - 1];
#pragma unroll 1
    for (int n = kSeriesN - 2; n >= 0; --n) {
        b1 = __builtin_fma(b1, t2, kSeries.a1[n]);
        b2 = __builtin_fma(b2, t2, kSeries.a2[n]);
        b3 = __builtin_fma(b3, t2, kSeries.a3[n]);
    }
    const double ct = kTwoOverSqrtPi * t;
    s1 = ct * b1;
    s2 = ct * t2 * b2;
    s3 = ct * t2 * t2 * b3;
}

// Modified smoothing for targets on the surface (section 2.1), with erf t = 1 - e^{-t^2} erfcx(t):
//   s1# = 1 - E (R - (c/3)(5t - 2t^3)),  s2# = 1 - E (R + (c/3)(3t - 14t^3 + 4t^5)),
//   s3# = 1 - E (R + (c/9)(9t + 6t^3 - 4t^5)),  c = 2/sqrt(pi), R = erfcx(t);
// 1 beyond the cut-off, 0 below kSeriesT (added by the series pass).
template <bool LO>
__device__ __forceinline__ void smoothing3_sharp(double t, double cutoff, double &s1, double &s2, double &s3)
{
    const double E = exp(-t * t);
    const double R = erfcx_eval<LO>(fmin(t, 6.25));
    const double t2 = t * t, c3 = kTwoOverSqrtPi / 3.0, c9 = kTwoOverSqrtPi / 9.0;
    const double P1 = R - c3 * t * __builtin_fma(-2.0, t2, 5.0);
    const double P2 = __builtin_fma(c3 * t, __builtin_fma(t2, __builtin_fma(4.0, t2, -14.0), 3.0), R);
    const double P3 = __builtin_fma(c9 * t, __builtin_fma(t2, __builtin_fma(-4.0, t2, 6.0), 9.0), R);
    const double Ec = t > cutoff ? 0.0 : E;
    const bool ser = t < kSeriesT;
    s1 = ser ? 0.0 : __builtin_fma(-Ec, P1, 1.0);
    s2 = ser ? 0.0 : __builtin_fma(-Ec, P2, 1.0);
    s3 = ser ? 0.0 : __builtin_fma(-Ec, P3, 1.0);
}

// Maclaurin coefficients of the modified functions: s1# = c t sum A1_n t^2n, s2# = c t^3 sum A2_n t^2n,
// s3# = c t^5 sum A3_n t^2n; from erf t = c sum E_n t^(2n+1), E_n = (-1)^n / (n! (2n+1)), and
// t^(2j+1) e^{-t^2} = sum X_m t^(2m+2j+1), X_m = (-1)^m / m!; the vanishing leading terms of s2#
// (one) and s3# (two) are left out.
struct SharpSeriesCoef {
    double a1[kSeriesN], a2[kSeriesN], a3[kSeriesN];
};
constexpr SharpSeriesCoef make_sharp_series()
{
    SharpSeriesCoef c{};
    double X[kSeriesN + 3] = {};
    X[0] = 1.0;
    for (int j = 1; j < kSeriesN + 3; ++j) X[j] = -X[j - 1] / j;
    for (int n = 0; n < kSeriesN + 2; ++n) {
        const double E = X[n] / (2 * n + 1);
        const double x1 = n >= 1 ? X[n - 1] : 0.0, x2 = n >= 2 ? X[n - 2] : 0.0;
        if (n < kSeriesN) c.a1[n] = E + (5.0 * X[n] - 2.0 * x1) / 3.0;
        if (n >= 1 && n - 1 < kSeriesN) c.a2[n - 1] = E - (3.0 * X[n] - 14.0 * x1 + 4.0 * x2) / 3.0;
        if (n >= 2 && n - 2 < kSeriesN) c.a3[n - 2] = E - (9.0 * X[n] + 6.0 * x1 - 4.0 * x2) / 9.0;
    }
    return c;
}
__constant__ constexpr SharpSeriesCoef kSharpSeries = make_sharp_series();

__device__ __forceinline__ void series3_sharp(double t, double &s1, double &s2, double &s3)
{
    const double t2 = t * t;
    double b1 = kSharpSeries.a1[kSeriesN - 1], b2 = kSharpSeries.a2[kSeriesN - 1], b3 = kSharpSeries.a3[kSeriesN - 1];
#pragma unroll 1
    for (int n = kSeriesN - 2; n >= 0; --n) {
        b1 = __builtin_fma(b1, t2, kSharpSeries.a1[n]);
        b2 = __builtin_fma(b2, t2, kSharpSeries.a2[n]);
        b3 = __builtin_fma(b3, t2, kSharpSeries.a3[n]);
    }
    const double ct = kTwoOverSqrtPi * t;
    s1 = ct * b1;
    s2 = ct * t2 * b2;
    s3 = ct * t2 * t2 * b3;
}

__device__ __forceinline__ double pick3(const double (&v)[3], int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }

struct Target {
    double y[3], x0[3], n[3], b, c, q0[3];
    double w[3];  // extrapolation weights (sorted-delta order), used when the sums are combined
};

struct Acc {
    double sl[3][3], dl[3][3];
};

// Adds one pair's contribution with smoothing factors s1, s2, s3 at sorted position J.
// COMB: the extrapolation weight w_J is applied here and every delta adds into slot 0 (one set of
// accumulators: sum_j w_j (far + near_j) = far + sum_j w_j near_j since the weights sum to 1).
template <int J, bool SL, bool DL, bool COMB>
__device__ __forceinline__ void add_delta(double s1, double s2, double s3, double ir, double ir3, double ir5,
                                          double dx, double dy, double dz, double gx, double gy, double gz,
                                          double dg, double t1x, double t1y, double t1z, double ex, double ey,
                                          double ez, double wJ, Acc &A)
{
    constexpr int K = COMB ? 0 : J;
    if (COMB) {
        s1 *= wJ;
        s2 *= wJ;
        s3 *= wJ;
    }
    if (SL) {
        const double k1 = s1 * ir, k2 = dg * s2 * ir3;
        A.sl[K][0] = __builtin_fma(dx, k2, __builtin_fma(gx, k1, A.sl[K][0]));
        A.sl[K][1] = __builtin_fma(dy, k2, __builtin_fma(gy, k1, A.sl[K][1]));
        A.sl[K][2] = __builtin_fma(dz, k2, __builtin_fma(gz, k1, A.sl[K][2]));
    }
    if (DL) {
        const double k2 = s2 * ir3, k3 = s3 * ir5;
        A.dl[K][0] = __builtin_fma(ex, k3, __builtin_fma(t1x, k2, A.dl[K][0]));
        A.dl[K][1] = __builtin_fma(ey, k3, __builtin_fma(t1y, k2, A.dl[K][1]));
        A.dl[K][2] = __builtin_fma(ez, k3, __builtin_fma(t1z, k2, A.dl[K][2]));
    }
}

template <int J, bool SL, bool DL, bool COMB, bool LO>
__device__ __forceinline__ void accumulate_delta(double r, double E, double ir, double ir3, double ir5, double dx,
                                                 double dy, double dz, double gx, double gy, double gz, double dg,
                                                 double t1x, double t1y, double t1z, double ex, double ey, double ez,
                                                 const DevParams &p, const Target &T, Acc &A)
{
    double s1, s2, s3;
    smoothing3<LO>(r * p.inv_delta[J], E, p.cutoff, s1, s2, s3);
    add_delta<J, SL, DL, COMB>(s1, s2, s3, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez,
                               T.w[J], A);
}

// The contributions that smoothing3 left out (t < kSeriesT), from the series.  Rarely executed: only
// pairs closer than kSeriesT times the largest delta reach it.
template <int J, bool SL, bool DL, bool COMB>
__device__ __forceinline__ void series_delta(double r, double ir, double ir3, double ir5, double dx, double dy,
                                             double dz, double gx, double gy, double gz, double dg, double t1x,
                                             double t1y, double t1z, double ex, double ey, double ez,
                                             const DevParams &p, const Target &T, Acc &A)
{
    const double t = r * p.inv_delta[J];
    if (t < kSeriesT) {
        double s1, s2, s3;
        series3(t, s1, s2, s3);
        add_delta<J, SL, DL, COMB>(s1, s2, s3, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez,
                                   T.w[J], A);
    }
}

// One near pair, accumulated at the three smoothing lengths (sorted-delta order).  SER = false: the
// closed-form smoothing factors, leaving out t < kSeriesT; returns whether some t is below kSeriesT
// (then the caller calls it again with SER = true, which adds just those terms from the series).
template <bool SL, bool DL, bool SER, bool P234, bool COMB, bool LO>
__device__ __forceinline__ bool near_pair(const SrcRec<double> &s, const Target &T, const DevParams &p, Acc &A)
{
    const double dx = T.y[0] - s.x, dy = T.y[1] - s.y, dz = T.y[2] - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) {
        if (SER) return false;
        // target on a quadrature point: limit of s1(r/delta)/r is 2/(sqrt(pi) delta); the d d s2/r^3
        // term and the whole double-layer term vanish
        if (SL) {
            const double gx = s.fw[0] - T.c * s.nw[0], gy = s.fw[1] - T.c * s.nw[1], gz = s.fw[2] - T.c * s.nw[2];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double l = kTwoOverSqrtPi * p.inv_delta[j] * (COMB ? T.w[j] : 1.0);
                const int k = COMB ? 0 : j;
                A.sl[k][0] += gx * l;
                A.sl[k][1] += gy * l;
                A.sl[k][2] += gz * l;
            }
        }
        return false;
    }
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    const double ir2 = ir * ir;
    const double ir3 = ir2 * ir;
    const double ir5 = ir3 * ir2;
    double gx = 0, gy = 0, gz = 0, dg = 0;
    if (SL) {
        gx = s.fw[0] - T.c * s.nw[0];
        gy = s.fw[1] - T.c * s.nw[1];
        gz = s.fw[2] - T.c * s.nw[2];
        dg = dx * gx + dy * gy + dz * gz;
    }
    double t1x = 0, t1y = 0, t1z = 0, ex = 0, ey = 0, ez = 0;
    if (DL) {
        const double nx = T.n[0], ny = T.n[1], nz = T.n[2], b = T.b;
        const double hx = s.x - T.x0[0], hy = s.y - T.x0[1], hz = s.z - T.x0[2];
        const double ax = s.q[0] - T.q0[0], ay = s.q[1] - T.q0[1], az = s.q[2] - T.q0[2];
        const double mx = s.nw[0], my = s.nw[1], mz = s.nw[2];
        const double na = nx * ax + ny * ay + nz * az;
        const double nm = nx * mx + ny * my + nz * mz;
        const double xa = hx * ax + hy * ay + hz * az;
        const double xm = hx * mx + hy * my + hz * mz;
        const double xn = hx * nx + hy * ny + hz * nz;
        const double xx = hx * hx + hy * hy + hz * hz;
        const double nanm = na * nm;
        const double c1n = b * nanm - xa * nm - na * xm;
        t1x = nx * c1n - hx * nanm;
        t1y = ny * c1n - hy * nanm;
        t1z = nz * c1n - hz * nanm;
        const double c2h = b * (xa * nm + na * xm) - xa * xm;
        const double c2n = b * xa * xm;
        const double rmb = xx - 2.0 * b * xn;  // r^2 - b^2
        ex = hx * c2h + nx * c2n - rmb * t1x;
        ey = hy * c2h + ny * c2n - rmb * t1y;
        ez = hz * c2h + nz * c2n - rmb * t1z;
    }
    if (SER) {
        series_delta<0, SL, DL, COMB>(r, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez, p, T, A);
        series_delta<1, SL, DL, COMB>(r, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez, p, T, A);
        series_delta<2, SL, DL, COMB>(r, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez, p, T, A);
        return false;
    }
    // e^{-t_j^2} for the three deltas.  P234 (sorted deltas in the ratio 2 : 3 : 4, the default rho):
    // B^36, B^16, B^9 of B = e^{-(t_0/6)^2}, one exponential and seven products (relative error ~50
    // ulp), taken in the order that keeps the fewest powers alive; otherwise three exponentials.
    if (P234) {
        const double tb = r * p.inv_delta[0] * (1.0 / 6.0);
        const double B = exp(-tb * tb);
        const double B4 = (B * B) * (B * B), B8 = B4 * B4;
        accumulate_delta<2, SL, DL, COMB, LO>(r, B8 * B, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez, p,
                                    T, A);
        const double B16 = B8 * B8;
        accumulate_delta<1, SL, DL, COMB, LO>(r, B16, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez, p,
                                    T, A);
        accumulate_delta<0, SL, DL, COMB, LO>(r, (B16 * B16) * B4, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex,
                                    ey, ez, p, T, A);
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double tj = r * p.inv_delta[j];
            const double Ej = exp(-tj * tj);
            if (j == 0)
                accumulate_delta<0, SL, DL, COMB, LO>(r, Ej, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez,
                                            p, T, A);
            else if (j == 1)
                accumulate_delta<1, SL, DL, COMB, LO>(r, Ej, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez,
                                            p, T, A);
            else
                accumulate_delta<2, SL, DL, COMB, LO>(r, Ej, ir, ir3, ir5, dx, dy, dz, gx, gy, gz, dg, t1x, t1y, t1z, ex, ey, ez,
                                            p, T, A);
        }
    }
    return r * p.inv_delta[2] < kSeriesT;  // inv_delta[2] is the smallest: t < kSeriesT for some delta
}

// A near pair: the closed-form pass, then (rarely) the series pass.  The empty asm hides that the
// second load reads the same record, so the record is not kept in registers across the first pass.
template <bool SL, bool DL, bool P234, bool COMB, bool LO>
__device__ __forceinline__ void near_pair_full(const SrcRec<double> *__restrict__ rec64, int k, const Target &T,
                                               const DevParams &p, Acc &A)
{
    if (near_pair<SL, DL, false, P234, COMB, LO>(rec64[k], T, p, A)) {
        int kk = k;
        asm volatile("" : "+v"(kk));
        near_pair<SL, DL, true, P234, COMB, LO>(rec64[kk], T, p, A);
    }
}

// Combined closed-form pass (COMB): the kernels are linear in (s1, s2, s3), so
// sum_j w_j K(s(t_j)) = K(S) with S_k = sum_j w_j s_k(t_j): the three smoothing lengths share one kernel
// evaluation and one set of accumulators.  Returns whether t < kSeriesT for some delta (then the
// series pass adds those terms).
template <bool SL, bool DL, bool P234, bool LO>
__device__ __forceinline__ bool near_pair_comb(const SrcRec<double> &s, const Target &T, const DevParams &p, Acc &A)
{
    const double dx = T.y[0] - s.x, dy = T.y[1] - s.y, dz = T.y[2] - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) {
        // target on a quadrature point: limit of s1(r/delta)/r is 2/(sqrt(pi) delta); the d d s2/r^3
        // term and the whole double-layer term vanish
        if (SL) {
            const double gx = s.fw[0] - T.c * s.nw[0], gy = s.fw[1] - T.c * s.nw[1], gz = s.fw[2] - T.c * s.nw[2];
            const double l = kTwoOverSqrtPi *
                             (T.w[0] * p.inv_delta[0] + T.w[1] * p.inv_delta[1] + T.w[2] * p.inv_delta[2]);
            A.sl[0][0] += gx * l;
            A.sl[0][1] += gy * l;
            A.sl[0][2] += gz * l;
        }
        return false;
    }
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    // e^{-t_j^2}: with P234 (sorted deltas in the ratio 2 : 3 : 4) B^9, B^16, B^36 of
    // B = e^{-(t_0/6)^2}, one exponential; otherwise one per delta
    double E0, E1, E2;
    if (P234) {
        const double tb = r * p.inv_delta[0] * (1.0 / 6.0);
        const double B = exp(-tb * tb);
        const double B4 = (B * B) * (B * B), B8 = B4 * B4, B16 = B8 * B8;
        E2 = B8 * B;
        E1 = B16;
        E0 = (B16 * B16) * B4;
    } else {
        const double t0 = r * p.inv_delta[0], t1 = r * p.inv_delta[1], t2 = r * p.inv_delta[2];
        E0 = exp(-t0 * t0);
        E1 = exp(-t1 * t1);
        E2 = exp(-t2 * t2);
    }
    double S1, S2, S3;
    {
        double a1, a2, a3;
        smoothing3<LO>(r * p.inv_delta[2], E2, p.cutoff, a1, a2, a3);
        S1 = T.w[2] * a1;
        S2 = T.w[2] * a2;
        S3 = T.w[2] * a3;
        // the two smaller deltas: when no pair of the wavefront's batch lies within their cut-off ball
        // (the candidates of a batch come from a few neighbouring cells, so about 40% of the batches
        // lie beyond cutoff * delta_0) their factors are 1 exactly and the evaluation is skipped
        const double t1 = r * p.inv_delta[1], t0 = r * p.inv_delta[0];
        if (__ballot(t1 <= p.cutoff)) {
            smoothing3<LO>(t1, E1, p.cutoff, a1, a2, a3);
            S1 = __builtin_fma(T.w[1], a1, S1);
            S2 = __builtin_fma(T.w[1], a2, S2);
            S3 = __builtin_fma(T.w[1], a3, S3);
        } else {
            S1 += T.w[1];
            S2 += T.w[1];
            S3 += T.w[1];
        }
        if (__ballot(t0 <= p.cutoff)) {
            smoothing3<LO>(t0, E0, p.cutoff, a1, a2, a3);
            S1 = __builtin_fma(T.w[0], a1, S1);
            S2 = __builtin_fma(T.w[0], a2, S2);
            S3 = __builtin_fma(T.w[0], a3, S3);
        } else {
            S1 += T.w[0];
            S2 += T.w[0];
            S3 += T.w[0];
        }
    }
    const double ir3 = (ir * ir) * ir;
    if (SL) {
        const double gx = s.fw[0] - T.c * s.nw[0], gy = s.fw[1] - T.c * s.nw[1], gz = s.fw[2] - T.c * s.nw[2];
        const double dg = dx * gx + dy * gy + dz * gz;
        const double k1 = S1 * ir, k2 = dg * S2 * ir3;
        A.sl[0][0] = __builtin_fma(dx, k2, __builtin_fma(gx, k1, A.sl[0][0]));
        A.sl[0][1] = __builtin_fma(dy, k2, __builtin_fma(gy, k1, A.sl[0][1]));
        A.sl[0][2] = __builtin_fma(dz, k2, __builtin_fma(gz, k1, A.sl[0][2]));
    }
    if (DL) {
        const double nx = T.n[0], ny = T.n[1], nz = T.n[2], b = T.b;
        const double hx = s.x - T.x0[0], hy = s.y - T.x0[1], hz = s.z - T.x0[2];
        const double ax = s.q[0] - T.q0[0], ay = s.q[1] - T.q0[1], az = s.q[2] - T.q0[2];
        const double mx = s.nw[0], my = s.nw[1], mz = s.nw[2];
        const double na = nx * ax + ny * ay + nz * az;
        const double nm = nx * mx + ny * my + nz * mz;
        const double xa = hx * ax + hy * ay + hz * az;
        const double xm = hx * mx + hy * my + hz * mz;
        const double xn = hx * nx + hy * ny + hz * nz;
        const double xx = hx * hx + hy * hy + hz * hz;
        const double nanm = na * nm;
        const double c1n = b * nanm - xa * nm - na * xm;
        const double t1x = nx * c1n - hx * nanm;
        const double t1y = ny * c1n - hy * nanm;
        const double t1z = nz * c1n - hz * nanm;
        const double c2h = b * (xa * nm + na * xm) - xa * xm;
        const double c2n = b * xa * xm;
        const double rmb = xx - 2.0 * b * xn;  // r^2 - b^2
        const double ex = hx * c2h + nx * c2n - rmb * t1x;
        const double ey = hy * c2h + ny * c2n - rmb * t1y;
        const double ez = hz * c2h + nz * c2n - rmb * t1z;
        const double k2 = S2 * ir3, k3 = S3 * (ir3 * (ir * ir));
        A.dl[0][0] = __builtin_fma(ex, k3, __builtin_fma(t1x, k2, A.dl[0][0]));
        A.dl[0][1] = __builtin_fma(ey, k3, __builtin_fma(t1y, k2, A.dl[0][1]));
        A.dl[0][2] = __builtin_fma(ez, k3, __builtin_fma(t1z, k2, A.dl[0][2]));
    }
    return r * p.inv_delta[2] < kSeriesT;  // inv_delta[2] is the smallest: t < kSeriesT for some delta
}

template <bool SL, bool DL, bool P234, bool LO>
__device__ __forceinline__ void near_pair_comb_full(const SrcRec<double> *__restrict__ rec64, int k, const Target &T,
                                                    const DevParams &p, Acc &A)
{
    if (near_pair_comb<SL, DL, P234, LO>(rec64[k], T, p, A)) {
        int kk = k;
        asm volatile("" : "+v"(kk));
        near_pair<SL, DL, true, P234, true, LO>(rec64[kk], T, p, A);
    }
}

// A near pair of a target on the surface evaluated with the modified smoothing at one delta
// (section 2.1): single layer with s1#, s2# (eq. (Sreg)); double layer with the stresslet's 1/r^5
// replaced by s3#/r^5, accumulated as sum d (d.a)(d.m) s3#/r^5 like the far-field channel.  Sums go to
// A.sl[0], A.dl[0].  SER as in near_pair.
template <bool SL, bool DL, bool SER, bool LO>
__device__ __forceinline__ bool near_pair_sharp(const SrcRec<double> &s, const Target &T, const DevParams &p,
                                                Acc &A)
{
    const double dx = T.y[0] - s.x, dy = T.y[1] - s.y, dz = T.y[2] - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    double gx = 0, gy = 0, gz = 0;
    if (SL) {
        gx = s.fw[0] - T.c * s.nw[0];
        gy = s.fw[1] - T.c * s.nw[1];
        gz = s.fw[2] - T.c * s.nw[2];
    }
    if (r2 == 0.0) {
        // limit of s1#(r/delta)/r: 16/(3 sqrt(pi) delta); the other terms vanish
        if (SL && !SER) {
            const double l = (8.0 / 3.0) * kTwoOverSqrtPi * p.inv_dsharp;
            A.sl[0][0] += gx * l;
            A.sl[0][1] += gy * l;
            A.sl[0][2] += gz * l;
        }
        return false;
    }
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    const double t = r * p.inv_dsharp;
    if (SER && !(t < kSeriesT)) return false;
    double s1, s2, s3;
    if (SER)
        series3_sharp(t, s1, s2, s3);
    else
        smoothing3_sharp<LO>(t, p.cutoff, s1, s2, s3);
    const double ir2 = ir * ir;
    const double ir3 = ir2 * ir;
    if (SL) {
        const double dg = dx * gx + dy * gy + dz * gz;
        const double k1 = s1 * ir, k2 = dg * s2 * ir3;
        A.sl[0][0] = __builtin_fma(dx, k2, __builtin_fma(gx, k1, A.sl[0][0]));
        A.sl[0][1] = __builtin_fma(dy, k2, __builtin_fma(gy, k1, A.sl[0][1]));
        A.sl[0][2] = __builtin_fma(dz, k2, __builtin_fma(gz, k1, A.sl[0][2]));
    }
    if (DL) {
        const double ax = s.q[0] - T.q0[0], ay = s.q[1] - T.q0[1], az = s.q[2] - T.q0[2];
        const double da = dx * ax + dy * ay + dz * az;
        const double dm = dx * s.nw[0] + dy * s.nw[1] + dz * s.nw[2];
        const double co = da * dm * s3 * (ir3 * ir2);
        A.dl[0][0] = __builtin_fma(dx, co, A.dl[0][0]);
        A.dl[0][1] = __builtin_fma(dy, co, A.dl[0][1]);
        A.dl[0][2] = __builtin_fma(dz, co, A.dl[0][2]);
    }
    return !SER && t < kSeriesT;
}

template <bool SL, bool DL, bool LO>
__device__ __forceinline__ void near_pair_sharp_full(const SrcRec<double> *__restrict__ rec64, int k,
                                                     const Target &T, const DevParams &p, Acc &A)
{
    if (near_pair_sharp<SL, DL, false, LO>(rec64[k], T, p, A)) {
        int kk = k;
        asm volatile("" : "+v"(kk));
        near_pair_sharp<SL, DL, true, LO>(rec64[kk], T, p, A);
    }
}

// Extrapolation weights of eq. (extrap_eqn) for a target at signed distance b (the same for the single and
// double layer and every component); far from the surface the smallest delta alone (w = 1, 0, 0).
__device__ __forceinline__ void extrap_weights(double b, const DevParams &p, double w[3])
{
    w[0] = 1.0;
    w[1] = 0.0;
    w[2] = 0.0;
    const double dmax = p.rho[2] * p.h;  // largest delta (sorted)
    if (fabs(b) < p.cutoff * dmax) {
        double al[3], be[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double lam = b * p.inv_delta[j];
            al[j] = p.rho[j] * I0f(lam);
            be[j] = p.rho[j] * p.rho[j] * p.rho[j] * I2f(lam);
        }
        const double C0 = al[1] * be[2] - al[2] * be[1];
        const double C1 = al[2] * be[0] - al[0] * be[2];
        const double C2 = al[0] * be[1] - al[1] * be[0];
        const double D = C0 + C1 + C2;
        w[0] = C0 / D;
        w[1] = C1 / D;
        w[2] = C2 / D;
    }
}

// Candidate steps of 64 loaded together: 4 with single-precision positions; 2 with double-precision
// ones, whose 4-deep batch costs enough registers to spill (both measured on MI355X).
template <typename TC>
constexpr int depth_for() { return sizeof(TC) == 4 ? 4 : 2; }
constexpr int kRing = 512;   // per-wave ring buffer of near pairs (power of two >= 63 + depth * 64)
static_assert(kRing >= kWave - 1 + 4 * kWave && (kRing & (kRing - 1)) == 0, "ring buffer size");

// LO: the degree-11 erfcx table of the mixed-precision path
template <bool SL, bool DL, bool SHARP, bool P234, bool COMB, bool LO>
__device__ __forceinline__ void eval_pair(const SrcRec<double> *__restrict__ rec64, int k, const Target &T,
                                          const DevParams &p, Acc &A)
{
    if (SHARP)
        near_pair_sharp_full<SL, DL, LO>(rec64, k, T, p, A);
    else if (COMB)
        near_pair_comb_full<SL, DL, P234, LO>(rec64, k, T, p, A);
    else
        near_pair_full<SL, DL, P234, false, LO>(rec64, k, T, p, A);
}

// COMB (only when no per-delta outputs are asked for): the weights are known before the pair loop and
// each pair adds K(S), S_k = sum_j w_j s_k(t_j), into one set of accumulators instead of three.
template <typename TC, bool SL, bool DL, bool SHARP, bool P234, bool COMB>
__global__ __launch_bounds__(kBlock, P234 ? 4 : 1) void near_finalize_kernel(const SrcRec<double> *__restrict__ rec64,
                                                               const Pos4<TC> *__restrict__ pos,
                                                               const int *__restrict__ cell_start, CellGrid grid,
                                                               EvalArgs a, DevParams p, TC rc2, TC rc2s,
                                                               const double *__restrict__ part, int nparts,
                                                               NearFlag *__restrict__ flag)
{
    // single-precision candidate test = the mixed-precision path: the degree-11 erfcx table
    constexpr bool kLo = std::is_same<TC, float>::value;
    __shared__ int queue_all[kBlock / kWave][kRing];
    // readfirstlane: tells the compiler the wave index (hence the target) is wavefront-uniform, so the
    // target's data live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int lane = (int)threadIdx.x % kWave;
    int *queue = queue_all[wave];
    const int64_t t = (int64_t)blockIdx.x * (kBlock / kWave) + wave;
    if (t >= a.m) return;  // wavefront-uniform exit

    Target T;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T.y[i] = a.y[3 * t + i];
        T.x0[i] = a.x0[3 * t + i];
        T.n[i] = a.n0[3 * t + i];
        T.q0[i] = DL ? a.q0[3 * t + i] : 0.0;
    }
    T.b = a.b[t];
    // a target on the surface with the modified smoothing selected: one delta, no extrapolation
    // (wavefront-uniform: one target per wavefront)
    // SHARP instances take exactly these targets, the others every other target, so that each
    // instance is compiled for one path (one register budget)
    const bool sharp = p.sharp && T.b == 0.0;
    if (sharp != SHARP) return;  // wavefront-uniform exit
    T.c = SL ? a.f0[3 * t] * T.n[0] + a.f0[3 * t + 1] * T.n[1] + a.f0[3 * t + 2] * T.n[2] : 0.0;
    if (COMB) extrap_weights(T.b, p, T.w);
    const TC tyx = (TC)(T.y[0] - a.org[0]), tyy = (TC)(T.y[1] - a.org[1]), tyz = (TC)(T.y[2] - a.org[2]);
    // the far rule of the extrapolation (w = (1, 0, 0)) asserts that no source is within
    // cutoff * max delta: checked against the candidates (wavefront-uniform)
    const bool farrule = !SHARP && fabs(T.b) >= p.cutoff * p.rho[2] * p.h;
    const TC rflag2 = (TC)(p.rflag * p.rflag);
    bool bad = false;

    int ci[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = floor((T.y[d] - grid.lo[d]) * grid.inv_side);
        u = fmin(fmax(u, -2.0), (double)grid.g[d] + 1.0);
        ci[d] = (int)u;
    }

    Acc A;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) A.sl[j][i] = A.dl[j][i] = 0.0;

    // Candidates are loaded kDepth steps of 64 at a time, so that kDepth loads are in flight per
    // wavefront instead of one (the scan is otherwise a chain of dependent load latencies); the near
    // ones go to a ring buffer in LDS (kRing >= 63 + kDepth * 64 entries) and every full 64 are evaluated.
    constexpr int kDepth = depth_for<TC>();
    int head = 0, cnt = 0;  // ring buffer start and length (wavefront-uniform)
    const int z0 = max(ci[2] - 1, 0), z1 = min(ci[2] + 1, grid.g[2] - 1);
    for (int ix = max(ci[0] - 1, 0); ix <= min(ci[0] + 1, grid.g[0] - 1); ++ix) {
        for (int iy = max(ci[1] - 1, 0); iy <= min(ci[1] + 1, grid.g[1] - 1); ++iy) {
            if (z0 > z1) continue;
            const int cb = (ix * grid.g[1] + iy) * grid.g[2];
            const int s0 = cell_start[cb + z0], s1 = cell_start[cb + z1 + 1];
            for (int base = s0; base < s1; base += kDepth * kWave) {
                Pos4<TC> q[kDepth];
#pragma unroll
                for (int u = 0; u < kDepth; ++u) {
                    const int k = base + u * kWave + lane;
                    if (k < s1) q[u] = pos[k];
                }
#pragma unroll
                for (int u = 0; u < kDepth; ++u) {
                    const int k = base + u * kWave + lane;
                    const TC r2c = pair_r2(tyx, tyy, tyz, q[u].x, q[u].y, q[u].z);
                    const bool nr = k < s1 && r2c <= (SHARP ? rc2s : rc2);
                    if (farrule) bad = bad || (nr && r2c < rflag2);
                    const uint64_t m = __ballot(nr);
                    if (nr) {
                        const int off = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        queue[(head + cnt + off) & (kRing - 1)] = k;
                    }
                    cnt += __popcll(m);
                }
                while (cnt >= kWave) {
                    wave_lds_sync();
                    const int k2 = queue[(head + lane) & (kRing - 1)];
                    wave_lds_sync();
                    head = (head + kWave) & (kRing - 1);
                    cnt -= kWave;
                    eval_pair<SL, DL, SHARP, P234, COMB, kLo>(rec64, k2, T, p, A);
                }
            }
        }
    }
    wave_lds_sync();
    if (lane < cnt) eval_pair<SL, DL, SHARP, P234, COMB, kLo>(rec64, queue[(head + lane) & (kRing - 1)], T, p, A);
    if (farrule && __ballot(bad) && lane == 0) {
        atomicOr(&flag->bits, kFlagFarRule);
        atomicMin(&flag->first, (unsigned long long)t);
    }

    constexpr int NJ = COMB ? 1 : 3;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (SL) A.sl[j][i] = wave_sum(A.sl[j][i]);
            if (DL) A.dl[j][i] = wave_sum(A.dl[j][i]);
        }

    const double b = T.b;
    const double chi = b < 0.0 ? 1.0 : (b > 0.0 ? 0.0 : 0.5);
    const double inv8pi = 1.0 / (8.0 * kPi);

    if (COMB) {
        if (lane < 3) {
            const int i = lane;
            if (SL) {
                double far = 0.0;
                for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + i) * (size_t)a.m + t];
                a.u[3 * t + i] = (far + pick3(A.sl[0], i)) * inv8pi;
            }
            if (DL) {
                double far = 0.0;
                for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + 3 + i) * (size_t)a.m + t];
                a.v[3 * t + i] = -6.0 * (far + pick3(A.dl[0], i)) * inv8pi + chi * pick3(T.q0, i);
            }
        }
        return;
    }

    double w0 = 1.0, w1 = 0.0, w2 = 0.0;
    if (!SHARP) {
        double w[3];
        extrap_weights(b, p, w);
        w0 = w[0];
        w1 = w[1];
        w2 = w[2];
    }

    if (lane < 3) {
        const int i = lane;
        if (SL) {
            double far = 0.0;
            for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + i) * (size_t)a.m + t];
            double uj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) uj[j] = (far + pick3(A.sl[j], i)) * inv8pi;
            a.u[3 * t + i] = w0 * uj[0] + w1 * uj[1] + w2 * uj[2];
            if (a.u_delta)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.u_delta[9 * t + 3 * p.ord[j] + i] = SHARP ? uj[0] : uj[j];
        }
        if (DL) {
            double far = 0.0;
            for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + 3 + i) * (size_t)a.m + t];
            double vj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) vj[j] = -6.0 * (far + pick3(A.dl[j], i)) * inv8pi;
            a.v[3 * t + i] = w0 * vj[0] + w1 * vj[1] + w2 * vj[2] + chi * pick3(T.q0, i);
            if (a.v_delta)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.v_delta[9 * t + 3 * p.ord[j] + i] = SHARP ? vj[0] : vj[j];
        }
    }
}

template <typename TC, bool SL, bool DL>
hipError_t launch_t(const SrcRec<double> *rec64, const Pos4<TC> *pos, const int *cell_start, const CellGrid &g,
                    const EvalArgs &a, const DevParams &p, TC rc2, const double *part, int nparts, NearFlag *flag,
                    hipStream_t s)
{
    const int per_block = kBlock / kWave;
    const int64_t blocks = (a.m + per_block - 1) / per_block;
    const bool comb = a.u_delta == nullptr && a.v_delta == nullptr;
    const TC rc2s = (TC)(p.rsharp * p.rsharp);  // near radius of the surface targets of the SHARP instance
    const dim3 grid((unsigned)blocks), block(kBlock);
    if (p.pow234 && comb)
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, false, true, true>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    else if (p.pow234)
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, false, true, false>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    else if (comb)
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, false, false, true>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    else
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, false, false, false>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !p.sharp) return e;
    hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, true, false, false>), grid, block, 0, s, rec64, pos,
                       cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    return hipGetLastError();
}

template <typename TC>
hipError_t dispatch(int layers, const SrcRec<double> *rec64, const Pos4<TC> *pos, const int *cell_start,
                    const CellGrid &g, const EvalArgs &a, const DevParams &p, TC rc2, const double *part,
                    int nparts, NearFlag *flag, hipStream_t s)
{
    if (layers == (SR_SL | SR_DL))
        return launch_t<TC, true, true>(rec64, pos, cell_start, g, a, p, rc2, part, nparts, flag, s);
    if (layers == SR_SL)
        return launch_t<TC, true, false>(rec64, pos, cell_start, g, a, p, rc2, part, nparts, flag, s);
    return launch_t<TC, false, true>(rec64, pos, cell_start, g, a, p, rc2, part, nparts, flag, s);
}

// Far field added to outputs that already hold the near sums, the extrapolation and the jump term
// (the near kernel run with no far partial sums, concurrently with the far-field kernel).  The
// extrapolation weights w = e_1^T A^{-1} of eq. (extrap_eqn) satisfy w A = e_1^T and the first column
// of A is all ones, so they sum to one (up to rounding) and the far sum shared by the three smoothing
// lengths enters once, unweighted: u += S_far / (8 pi), v += -6 T_far / (8 pi); a target with the
// modified smoothing has the single weight 1.  STORE: u = S_far / (8 pi), v = -6 T_far / (8 pi) (the
// plain sums at targets with no closest point).  One lane per (channel, target), channel-major, so
// that the partial sums part[split][channel][target] are read coalesced and the grid fills the chip.
template <bool SL, bool DL, bool STORE>
__global__ __launch_bounds__(kBlock) void far_add_kernel(const double *__restrict__ part, int nparts, int64_t m,
                                                         double *__restrict__ u, double *__restrict__ v)
{
    constexpr int c0 = SL ? 0 : 3, nch = (SL ? 3 : 0) + (DL ? 3 : 0);
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nch * m) return;
    const int c = c0 + (int)(e / m);  // channel 0..2 single layer, 3..5 double layer
    const int64_t t = e - (int64_t)(c - c0) * m;
    double far = 0.0;
    for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + c) * (size_t)m + t];
    const double inv8pi = 1.0 / (8.0 * kPi);
    double *o = c < 3 ? &u[3 * t + c] : &v[3 * t + c - 3];
    const double val = (c < 3 ? far : -6.0 * far) * inv8pi;
    *o = STORE ? val : *o + val;
}

__global__ void flag_clear_kernel(NearFlag *flag)
{
    if (threadIdx.x == 0) {
        flag->bits = 0u;
        flag->first = ~0ull;
    }
}

}  // namespace

template <bool STORE>
void launch_far_add_t(int layers, const double *part, int nparts, const EvalArgs &a, dim3 grid, hipStream_t s)
{
    const dim3 block(kBlock);
    if (layers == (SR_SL | SR_DL))
        hipLaunchKernelGGL((far_add_kernel<true, true, STORE>), grid, block, 0, s, part, nparts, a.m, a.u, a.v);
    else if (layers == SR_SL)
        hipLaunchKernelGGL((far_add_kernel<true, false, STORE>), grid, block, 0, s, part, nparts, a.m, a.u, a.v);
    else
        hipLaunchKernelGGL((far_add_kernel<false, true, STORE>), grid, block, 0, s, part, nparts, a.m, a.u, a.v);
}

hipError_t launch_far_add(int layers, const double *part, int nparts, const EvalArgs &a, bool store, hipStream_t s)
{
    const int64_t lanes = (layers == (SR_SL | SR_DL) ? 6 : 3) * a.m;
    const dim3 grid((unsigned)((lanes + kBlock - 1) / kBlock));
    if (store)
        launch_far_add_t<true>(layers, part, nparts, a, grid, s);
    else
        launch_far_add_t<false>(layers, part, nparts, a, grid, s);
    return hipGetLastError();
}

hipError_t launch_flag_clear(NearFlag *flag, hipStream_t s)
{
    hipLaunchKernelGGL(flag_clear_kernel, dim3(1), dim3(kWave), 0, s, flag);
    return hipGetLastError();
}

hipError_t launch_near_finalize(int precision, int layers, const SrcRec<double> *rec64,
                                const Pos4<double> *pos64, const Pos4<float> *pos32, const int *cell_start,
                                const CellGrid &grid, const EvalArgs &a, const DevParams &p, const double *part,
                                int nparts, NearFlag *flag, hipStream_t s)
{
    const double rc2 = p.rnear * p.rnear;
    if (precision == SR_MIXED)
        return dispatch<float>(layers, rec64, pos32, cell_start, grid, a, p, (float)rc2, part, nparts, flag, s);
    return dispatch<double>(layers, rec64, pos64, cell_start, grid, a, p, rc2, part, nparts, flag, s);
}

}  // namespace sr

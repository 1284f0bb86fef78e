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
// Work decomposition: one wavefront per target (4 per workgroup).  The cell grid's side is a third
// of the reach (the near radius plus its rounding margin), so the target's near pairs lie in the
// columns of cells within the reach: up to 7 x 7 columns, each a contiguous record range of the cells
// within the reach in z.  The lanes set up the columns in parallel (one per lane: the column is
// dropped when its xy-box lies beyond the reach, else its range is loaded), then the wavefront scans
// the live columns: the lanes test candidates 64 at a time (compact single- or double-precision
// positions; up to kDepth loads in flight, only the steps that hold candidates) and append the near
// ones to a per-wave ring buffer in LDS; each time it holds 64 pairs, all 64 lanes evaluate one pair
// each, so the FP64 regularized kernels run without idle lanes.
// Smoothing factors: s1 = 1 - E R, s2 = 1 - E P2, s2 - s3 = (4/(3 sqrt(pi))) t^3 E with E = e^{-t^2},
// R = erfcx(t) (sr_erfcx_table.h), P2 = R + (2/sqrt(pi)) t; with rho in the ratio 2 : 3 : 4 the three
// exponentials are powers of one.  When only the extrapolated values are asked for, the weights w_j
// are computed first and a pair adds K(S), S_k = sum_j w_j s_k(t_j), to one set of accumulators (the
// kernels are linear in the factors).  A batch of 64 pairs skips a smoothing length when none of its
// pairs lies within that length's cut-off ball (a wavefront-uniform test; beyond it the factors are 1).
// The double layer is summed as d (...) plus n0 (...), the n0 part as one scalar per target (see
// add_terms).  The closest pairs (r < kSeriesT max delta, the target's own point included) are left
// out of this pass and added by an exact pass (Maclaurin series of the factors where t < kSeriesT; the
// r -> 0 limits) run only on the lanes that hold them.
// Per-lane FP64 partial sums are combined by a butterfly wavefront reduction.
// A target whose |b| selects w = (1, 0, 0) lies, by its own b, at least cutoff * max delta from the
// surface; if a source is closer than that (less a rounding margin) the caller's b is wrong and the
// near regularization it skipped was needed: the scan reports it in the context's NearFlag.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include <type_traits>

#include "sr_erfcx_table.h"
#include "sr_internal.h"

namespace sr {

// The erfcx coefficients live in device variables with external linkage: the compiler cannot fold
// them into immediates, so the polynomial reads them with scalar loads into SGPRs instead of keeping
// 17 FP64 constants (34 VGPRs) live across the pair loop.  Two tables: degree 16 (|erfc error|
// ~6e-16) for the double-precision path, degree 11 (~2e-11) for the mixed-precision path, whose
// single-precision far field (relative error ~1e-7) dominates its error.

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

// acc * x + c as one fused multiply-add with the coefficient c in a scalar register.  Written out
// because the compiler otherwise keeps the polynomial coefficients in vector registers and, to use
// its two-address multiply-add, copies the coefficient into the destination before every step (one
// extra instruction per coefficient and about 50 more VGPRs for the kernel).
__device__ __forceinline__ double fma_coef(double acc, double x, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(x), "s"(c));
    return r;
}

// e^x for x <= 0 by Cody and Waite's reduction (W. J. Cody, W. Waite, Software Manual for the
// Elementary Functions, 1980): x = k ln2 + f with k = rint(x / ln2), |f| <= ln2/2, ln2 split into a
// 32-bit head (k ln2_hi exact for |k| < 2^21) and a tail; e^f by its Taylor polynomial of degree 13
// (remainder below 5e-18 relative), e^x = 2^k e^f (0 once 2^k underflows).  Written as plain Horner
// steps so that no coefficient register is overwritten (no copies), with no range checks: the callers'
// arguments are finite and non-positive.
struct ExpTaylor {
    double c[14];
};
constexpr ExpTaylor make_exp_taylor()
{
    ExpTaylor r{};
    double f = 1.0;
    for (int n = 0; n < 14; ++n) {
        r.c[n] = 1.0 / f;  // 1/n!, n! exact in double for n <= 18
        f *= (double)(n + 1);
    }
    return r;
}
constexpr ExpTaylor kExpTaylor = make_exp_taylor();
constexpr double kLn2Hi = 0.6931471803691238;      // ln 2 to 32 bits
constexpr double kLn2Lo = 1.9082149292705877e-10;  // ln 2 - kLn2Hi
constexpr double kLog2E = 1.4426950408889634;
__device__ __forceinline__ double exp_nonpos(double x)
{
    const double k = __builtin_rint(x * kLog2E);
    double f = __builtin_fma(-k, kLn2Hi, x);
    f = __builtin_fma(-k, kLn2Lo, f);
    double p = kExpTaylor.c[13];
#pragma unroll
    for (int n = 12; n >= 0; --n) p = fma_coef(p, f, kExpTaylor.c[n]);
    return __builtin_amdgcn_ldexp(p, (int)k);
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
// The table's coefficients times L, so that erfcx = inv * P_L(x) with one product.
template <class EP>
struct ErfcxCoefL {
    double c[EP::kDegree + 1];
};
template <class EP>
constexpr ErfcxCoefL<EP> make_erfcx_coef_l()
{
    ErfcxCoefL<EP> r{};
    for (int k = 0; k <= EP::kDegree; ++k) r.c[k] = EP::kL * EP::kC[k];
    return r;
}
__constant__ ErfcxCoefL<erfcx_poly::Fp64> g_erfcx_coef_l = make_erfcx_coef_l<erfcx_poly::Fp64>();
__constant__ ErfcxCoefL<erfcx_poly::Mixed> g_erfcx_coef_mixed_l = make_erfcx_coef_l<erfcx_poly::Mixed>();

// erfcx(t), t >= 0, from the interpolating polynomial of sr_erfcx_table.h in the variable
// x = A (t - L)/(t + L) + B = (A + B) - 2 A L inv, inv = 1/(t + L): erfcx = inv * sum_k (L C_k) x^k.
// The reciprocal is the hardware estimate refined by Newton steps y <- y + y (1 - den y): two for
// the degree-16 table (full double precision), one for the mixed path's degree-11 table (relative
// error ~1e-15, far below that table's 2e-11).  Accurate on [0, 6.25]; finite for every t >= 0.
template <bool LO>
__device__ __forceinline__ double erfcx_eval(double tc)
{
    using EP = std::conditional_t<LO, erfcx_poly::Mixed, erfcx_poly::Fp64>;
    const double den = tc + EP::kL;
    double inv = __builtin_amdgcn_rcp(den);
    double e = __builtin_fma(-den, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    if (!LO) {
        e = __builtin_fma(-den, inv, 1.0);
        inv = __builtin_fma(inv, e, inv);
    }
    const double x = __builtin_fma(-2.0 * EP::kA * EP::kL, inv, EP::kA + EP::kB);
    double pz;
    if constexpr (LO) {
        pz = g_erfcx_coef_mixed_l.c[EP::kDegree];
#pragma unroll
        for (int k = EP::kDegree - 1; k >= 0; --k) pz = fma_coef(pz, x, g_erfcx_coef_mixed_l.c[k]);
    } else {
        pz = g_erfcx_coef_l.c[EP::kDegree];
#pragma unroll
        for (int k = EP::kDegree - 1; k >= 0; --k) pz = fma_coef(pz, x, g_erfcx_coef_l.c[k]);
    }
    return inv * pz;
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
    const double E = exp_nonpos(-t * t);
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

// Target data used by the pair evaluation (wavefront-uniform values; see to_vgpr for where they are
// held).
struct TgtV {
    double y[3], n[3], q0[3], b, c;
    double w[3];  // extrapolation weights (sorted-delta order)
};

// Per-lane accumulators: slot 0 for the combined sums, slots 0..2 per delta otherwise.
template <int NJ>
struct AccN {
    double sl[NJ][3], dl[NJ][3];
    double dn[NJ];  // double layer: the scalar factor of n0 (see add_terms)
};

// s2 - s3 = (4 / (3 sqrt(pi))) t^3 e^{-t^2} (from P_3 = P_2 + (4 / (3 sqrt(pi))) t^3)
constexpr double kD3 = 2.0 / 3.0 * kTwoOverSqrtPi;

// 1/sqrt(v), v > 0 finite: hardware estimate and two Newton steps y <- y + (y/2)(1 - v y^2)
__device__ __forceinline__ double rsq64(double v)
{
    double y = __builtin_amdgcn_rsq(v);
    double e = __builtin_fma(-(v * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-(v * y), y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

// e^{-t_j^2} for the three sorted deltas: with P234 (deltas in the ratio 2 : 3 : 4) B^36, B^16, B^9 of
// B = e^{-(t_0/6)^2}, one exponential and seven products (relative error ~50 ulp); otherwise three
// exponentials.
template <bool P234>
__device__ __forceinline__ void exp3(double r, const DevParams &p, double &E0, double &E1, double &E2)
{
    if (P234) {
        const double tb = r * p.inv_delta[0] * (1.0 / 6.0);
        const double B = exp_nonpos(-tb * tb);
        const double B4 = (B * B) * (B * B), B8 = B4 * B4, B16 = B8 * B8;
        E2 = B8 * B;
        E1 = B16;
        E0 = (B16 * B16) * B4;
    } else {
        const double t0 = r * p.inv_delta[0], t1 = r * p.inv_delta[1], t2 = r * p.inv_delta[2];
        E0 = exp_nonpos(-t0 * t0);
        E1 = exp_nonpos(-t1 * t1);
        E2 = exp_nonpos(-t2 * t2);
    }
}

// One smoothing length's share of the combined factors.  With s1 = 1 - E R, s2 = 1 - E P2 and
// s2 - s3 = kD3 t^3 E (E = e^{-t^2}, R = erfcx(t), P2 = R + (2/sqrt(pi)) t; eqs. (s1)-(s3)) and weights
// summing to one:  S1 = sum_j w_j s1(t_j) = 1 - a1,  S2 = 1 - a2,  S2 - S3 = kD3 ad  with
// a1 = sum w_j E_j R_j,  a2 = sum w_j E_j P2_j,  ad = sum w_j E_j t_j^3;  beyond the cut-off the
// factors are 1 exactly (E taken as 0).
template <bool LO>
__device__ __forceinline__ void smooth_acc(double t, double E, double w, double cutoff, double &a1, double &a2,
                                           double &ad)
{
    // no clamp to the table's interval [0, 6.25]: beyond the cut-off E is taken as 0, and the
    // interpolant stays finite for every t >= 0 (its variable (t - L)/(t + L) lies in [-1, 1))
    const double R = erfcx_eval<LO>(t);
    const double P2 = __builtin_fma(kTwoOverSqrtPi, t, R);
    const double we = t > cutoff ? 0.0 : w * E;
    a1 = __builtin_fma(we, R, a1);
    a2 = __builtin_fma(we, P2, a2);
    ad = __builtin_fma(we * t, t * t, ad);
}

// The density factors of a pair, independent of the smoothing (eqs. (Stokes_SL1), (Stokes_DL1), (Tsplit)):
//   single layer: g = f w - c n w (c = f(x0).n0), dg = d.g;
//   double layer: with a = q - q0, m = n w, d = y - x = b n0 - xh (xh = x - x0):
//     t1 = n0 (b (n0.a)(n0.m) - (xh.a)(n0.m) - (n0.a)(xh.m)) - xh (n0.a)(n0.m) = n0 cn + d (n0.a)(n0.m),
//     cn = (d.a)(n0.m) + (n0.a)(d.m) - 2 b (n0.a)(n0.m),
//   and t2 - (r^2 - b^2) t1 = d (d.a)(d.m) - r^2 t1 (because t2 + b^2 t1 = d (d.a)(d.m)), so the
//   split stresslet's t1 s2/r^3 + (t2 - (r^2 - b^2) t1) s3/r^5 = t1 (s2 - s3)/r^3 + d (d.a)(d.m) s3/r^5
//   = n0 [cn (s2 - s3)/r^3] + d [(n0.a)(n0.m)(s2 - s3)/r^3 + (d.a)(d.m) s3/r^5]: the n0 part is a
//   scalar sum per target, multiplied by n0 once at the end.
struct PairGeo {
    double gx, gy, gz, dg;
    double cn, nanm, dadm;
};
template <bool SL, bool DL>
__device__ __forceinline__ PairGeo pair_geo(const SrcRec<double> &s, const TgtV &T, double dx, double dy, double dz)
{
    PairGeo G{};
    if (SL) {
        G.gx = __builtin_fma(-T.c, s.nw[0], s.fw[0]);
        G.gy = __builtin_fma(-T.c, s.nw[1], s.fw[1]);
        G.gz = __builtin_fma(-T.c, s.nw[2], s.fw[2]);
        G.dg = __builtin_fma(dz, G.gz, __builtin_fma(dy, G.gy, dx * G.gx));
    }
    if (DL) {
        const double ax = s.q[0] - T.q0[0], ay = s.q[1] - T.q0[1], az = s.q[2] - T.q0[2];
        const double na = __builtin_fma(T.n[2], az, __builtin_fma(T.n[1], ay, T.n[0] * ax));
        const double nm = __builtin_fma(T.n[2], s.nw[2], __builtin_fma(T.n[1], s.nw[1], T.n[0] * s.nw[0]));
        const double da = __builtin_fma(dz, az, __builtin_fma(dy, ay, dx * ax));
        const double dm = __builtin_fma(dz, s.nw[2], __builtin_fma(dy, s.nw[1], dx * s.nw[0]));
        G.nanm = na * nm;
        G.cn = __builtin_fma(-2.0 * T.b, G.nanm, __builtin_fma(da, nm, na * dm));
        G.dadm = da * dm;
    }
    return G;
}

// Adds K(S) for smoothing factors S1, S2, S3 = S2 - D: single layer g S1/r + d (d.g) S2/r^3
// (eq. (Sreg)) to sl; double layer d [(n0.a)(n0.m) D/r^3 + (d.a)(d.m) S3/r^5] to dl and cn D/r^3 to
// dn (the n0 part; the -6 is applied at the end).
template <bool SL, bool DL>
__device__ __forceinline__ void add_terms(double S1, double S2, double D, double ir, double dx, double dy, double dz,
                                          const PairGeo &G, double (&sl)[3], double (&dl)[3], double &dn)
{
    const double ir2 = ir * ir, ir3 = ir2 * ir;
    if (SL) {
        const double k1 = S1 * ir, k2 = G.dg * S2 * ir3;
        sl[0] = __builtin_fma(dx, k2, __builtin_fma(G.gx, k1, sl[0]));
        sl[1] = __builtin_fma(dy, k2, __builtin_fma(G.gy, k1, sl[1]));
        sl[2] = __builtin_fma(dz, k2, __builtin_fma(G.gz, k1, sl[2]));
    }
    if (DL) {
        const double k2 = D * ir3;
        const double kd = __builtin_fma(G.nanm, k2, (S2 - D) * (ir3 * ir2) * G.dadm);
        dl[0] = __builtin_fma(dx, kd, dl[0]);
        dl[1] = __builtin_fma(dy, kd, dl[1]);
        dl[2] = __builtin_fma(dz, kd, dl[2]);
        dn = __builtin_fma(G.cn, k2, dn);
    }
}

// Closed-form smoothing factors of one delta for t >= kSeriesT, or the series below it (eqs.
// (s1)-(s3)); 1 beyond the cut-off.  Returns s1, s2 and s2 - s3.
template <bool LO>
__device__ __forceinline__ void factors_one(double t, double cutoff, double &s1, double &s2, double &dd)
{
    if (t < kSeriesT) {
        double s3;
        series3(t, s1, s2, s3);
        dd = s2 - s3;
        return;
    }
    const double E = t > cutoff ? 0.0 : exp(-t * t);
    const double R = erfcx_eval<LO>(fmin(t, 6.25));
    s1 = __builtin_fma(-E, R, 1.0);
    s2 = __builtin_fma(-E, __builtin_fma(kTwoOverSqrtPi, t, R), 1.0);
    dd = kD3 * (E * t) * (t * t);
}

enum { kModeComb = 0, kModePerDelta = 1, kModeSharp = 2, kModeTab = 3 };

// The pairs the main pass leaves out (r below kSeriesT times the largest delta, r = 0 included):
// every factor from the series or the closed form as t requires; r = 0 adds the limit of s1/r,
// 2/(sqrt(pi) delta) (16/(3 sqrt(pi) delta) for s1#), the other terms vanish.  Rarely executed: the
// target's own point and its closest neighbours.
template <bool SL, bool DL, int MODE, bool LO, int NJ>
__device__ __forceinline__ void pair_exact(const SrcRec<double> &s, const TgtV &T, const DevParams &p, AccN<NJ> &A)
{
    const double dx = T.y[0] - s.x, dy = T.y[1] - s.y, dz = T.y[2] - s.z;
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    const PairGeo G = pair_geo<SL, DL>(s, T, dx, dy, dz);
    if (r2 == 0.0) {
        if (!SL) return;
        if (MODE == kModeSharp) {
            const double l = (8.0 / 3.0) * kTwoOverSqrtPi * p.inv_dsharp;
            A.sl[0][0] += G.gx * l;
            A.sl[0][1] += G.gy * l;
            A.sl[0][2] += G.gz * l;
            return;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double l = kTwoOverSqrtPi * p.inv_delta[j] * (MODE == kModeComb ? T.w[j] : 1.0);
            const int k = MODE == kModeComb ? 0 : j;
            A.sl[k][0] += G.gx * l;
            A.sl[k][1] += G.gy * l;
            A.sl[k][2] += G.gz * l;
        }
        return;
    }
    const double ir = rsq64(r2), r = r2 * ir;
    if (MODE == kModeSharp) {
        const double t = r * p.inv_dsharp;
        double s1, s2, s3;
        if (t < kSeriesT)
            series3_sharp(t, s1, s2, s3);
        else
            smoothing3_sharp<LO>(t, p.cutoff, s1, s2, s3);
        // the modified double layer is d (d.a)(d.m) s3#/r^5 alone: no t1 term
        add_terms<SL, DL>(s1, s2, s2 - s3, ir, dx, dy, dz, PairGeo{G.gx, G.gy, G.gz, G.dg, 0.0, 0.0, G.dadm},
                          A.sl[0], A.dl[0], A.dn[0]);
        return;
    }
    double S1 = 0.0, S2 = 0.0, D = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double s1, s2, dd;
        factors_one<LO>(r * p.inv_delta[j], p.cutoff, s1, s2, dd);
        if (MODE == kModeComb) {
            S1 = __builtin_fma(T.w[j], s1, S1);
            S2 = __builtin_fma(T.w[j], s2, S2);
            D = __builtin_fma(T.w[j], dd, D);
        } else {
            add_terms<SL, DL>(s1, s2, dd, ir, dx, dy, dz, G, A.sl[j], A.dl[j], A.dn[j]);
        }
    }
    if (MODE == kModeComb) add_terms<SL, DL>(S1, S2, D, ir, dx, dy, dz, G, A.sl[0], A.dl[0], A.dn[0]);
}

// One near pair in the main pass.  Lanes whose pair is closer than kSeriesT times the largest delta
// (`rare2`: some t below kSeriesT) contribute nothing here (1/r taken as 0, r2 as 1 so that every
// value stays finite) and go to pair_exact.
//   kModeComb: S_k = sum_j w_j s_k(t_j) (the kernels are linear in the factors, so the three smoothing
//     lengths share one kernel evaluation and one set of accumulators); a batch of 64 pairs skips a
//     smoothing length when none of its pairs lies within that length's cut-off ball (a
//     wavefront-uniform test: beyond it the factors are 1 and a1, a2, ad get nothing).
//   kModePerDelta: three sets of accumulators (the regularized values before extrapolation).
//   kModeSharp: the modified smoothing at one delta (section 2.1).
template <bool SL, bool DL, int MODE, bool P234, bool LO, int NJ>
__device__ __forceinline__ void near_pair(const SrcRec<double> &s, const TgtV &T, const DevParams &p, double rare2,
                                          AccN<NJ> &A, bool &rare)
{
    const double dx = T.y[0] - s.x, dy = T.y[1] - s.y, dz = T.y[2] - s.z;
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    rare = r2 < rare2;
    const double r2c = rare ? 1.0 : r2;
    double ir = rsq64(r2c);
    const double r = r2c * ir;
    ir = rare ? 0.0 : ir;
    if (MODE == kModeSharp) {
        double s1, s2, s3;
        smoothing3_sharp<LO>(r * p.inv_dsharp, p.cutoff, s1, s2, s3);
        const PairGeo G = pair_geo<SL, DL>(s, T, dx, dy, dz);
        add_terms<SL, DL>(s1, s2, s2 - s3, ir, dx, dy, dz, PairGeo{G.gx, G.gy, G.gz, G.dg, 0.0, 0.0, G.dadm},
                          A.sl[0], A.dl[0], A.dn[0]);
        return;
    }
    double E0, E1, E2;
    exp3<P234>(r, p, E0, E1, E2);
    if (MODE == kModeComb) {
        double a1 = 0.0, a2 = 0.0, ad = 0.0;
        smooth_acc<LO>(r * p.inv_delta[2], E2, T.w[2], p.cutoff, a1, a2, ad);
        const double t1 = r * p.inv_delta[1], t0 = r * p.inv_delta[0];
        if (__ballot(t1 <= p.cutoff)) smooth_acc<LO>(t1, E1, T.w[1], p.cutoff, a1, a2, ad);
        if (__ballot(t0 <= p.cutoff)) smooth_acc<LO>(t0, E0, T.w[0], p.cutoff, a1, a2, ad);
        const PairGeo G = pair_geo<SL, DL>(s, T, dx, dy, dz);
        add_terms<SL, DL>(1.0 - a1, 1.0 - a2, kD3 * ad, ir, dx, dy, dz, G, A.sl[0], A.dl[0], A.dn[0]);
    } else {
        const PairGeo G = pair_geo<SL, DL>(s, T, dx, dy, dz);
        const double E[3] = {E0, E1, E2};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double a1 = 0.0, a2 = 0.0, ad = 0.0;
            smooth_acc<LO>(r * p.inv_delta[j], E[j], 1.0, p.cutoff, a1, a2, ad);
            add_terms<SL, DL>(1.0 - a1, 1.0 - a2, kD3 * ad, ir, dx, dy, dz, G, A.sl[j], A.dl[j], A.dn[j]);
        }
    }
}

// One near pair of a target on the surface (b = 0) in the combined mode, from the smoothing table
// (NearTable: S1/r, S2/r^3 and S3/r^5 as polynomials on 160 intervals of r / h, held in LDS and read
// as coefficient pairs, 12 16-byte reads per pair;
// (S2 - S3)/r^3 = S2/r^3 - r^2 S3/r^5).  No closed forms, no exponential and no series: the table is
// smooth through r = 0 (the target's own point adds g S1/r at its limit), so every pair takes this one
// path.  r = r2 / sqrt(r2) from the hardware estimate and one Newton step (relative error ~4e-15);
// r = 0 exactly when r2 = 0.
template <bool SL, bool DL>
__device__ __forceinline__ void tab_pair(const SrcRec<double> &s, const TgtV &T, const DevParams &p,
                                         const double *__restrict__ tabs, AccN<1> &A)
{
    const double dx = T.y[0] - s.x, dy = T.y[1] - s.y, dz = T.y[2] - s.z;
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-((0.5 * r2) * y), y, 1.5);
    const double r = r2 > 0.0 ? r2 * (y * e) : 0.0;
    const double u = r * p.tab_scale;
    const int i = min((int)u, kTabIntervals - 1);
    const double sv = u - (double)i - 0.5;
    const double2 *c2 = reinterpret_cast<const double2 *>(tabs) + i;
    auto horner = [&](int f) {
        const double2 *q = c2 + f * (kTabCoef / 2) * kTabIntervals;
        double2 pr[kTabCoef / 2];
#pragma unroll
        for (int k = 0; k < kTabCoef / 2; ++k) pr[k] = q[k * kTabIntervals];
        double v = pr[kTabCoef / 2 - 1].y;
        v = __builtin_fma(v, sv, pr[kTabCoef / 2 - 1].x);
#pragma unroll
        for (int k = kTabCoef / 2 - 2; k >= 0; --k) {
            v = __builtin_fma(v, sv, pr[k].y);
            v = __builtin_fma(v, sv, pr[k].x);
        }
        return v;
    };
    const PairGeo G = pair_geo<SL, DL>(s, T, dx, dy, dz);
    const double g2 = horner(1) * p.ih3;
    if (SL) {
        const double k1 = horner(0) * p.ih, k2 = G.dg * g2;
        A.sl[0][0] = __builtin_fma(dx, k2, __builtin_fma(G.gx, k1, A.sl[0][0]));
        A.sl[0][1] = __builtin_fma(dy, k2, __builtin_fma(G.gy, k1, A.sl[0][1]));
        A.sl[0][2] = __builtin_fma(dz, k2, __builtin_fma(G.gz, k1, A.sl[0][2]));
    }
    if (DL) {
        const double g3 = horner(2) * p.ih5;
        const double k2 = __builtin_fma(-r2, g3, g2);  // (S2 - S3) / r^3
        const double kd = __builtin_fma(G.nanm, k2, g3 * G.dadm);
        A.dl[0][0] = __builtin_fma(dx, kd, A.dl[0][0]);
        A.dl[0][1] = __builtin_fma(dy, kd, A.dl[0][1]);
        A.dl[0][2] = __builtin_fma(dz, kd, A.dl[0][2]);
        A.dn[0] = __builtin_fma(G.cn, k2, A.dn[0]);
    }
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Extrapolation weights of eq. (extrap_eqn) for the wavefront's target at signed distance b (uniform;
// the same for the single and double layer and every component): w = e_1^T A^{-1} with rows
// A_j = [1, rho_j I0(lambda_j), rho_j^3 I2(lambda_j)], lambda_j = b / delta_j, by Cramer's rule, the three
// rows evaluated by lanes 0, 1, 2 side by side; far from the surface (|b| >= cutoff * max delta) the
// smallest delta alone, w = (1, 0, 0) (every pair is beyond the cut-off there and the matrix is
// numerically singular).
__device__ __forceinline__ void extrap_weights_wave(double b, const DevParams &p, int lane, double w[3])
{
    w[0] = 1.0;
    w[1] = 0.0;
    w[2] = 0.0;
    const double dmax = p.rho[2] * p.h;  // largest delta (sorted)
    if (fabs(b) < p.cutoff * dmax) {
        double al = 0.0, be = 0.0;
        if (lane < 3) {
            const double rho = lane == 0 ? p.rho[0] : (lane == 1 ? p.rho[1] : p.rho[2]);
            const double lam = b * (lane == 0 ? p.inv_delta[0] : (lane == 1 ? p.inv_delta[1] : p.inv_delta[2]));
            al = rho * I0f(lam);
            be = rho * rho * rho * I2f(lam);
        }
        const double al0 = readlane_f64(al, 0), al1 = readlane_f64(al, 1), al2 = readlane_f64(al, 2);
        const double be0 = readlane_f64(be, 0), be1 = readlane_f64(be, 1), be2 = readlane_f64(be, 2);
        const double C0 = al1 * be2 - al2 * be1;
        const double C1 = al2 * be0 - al0 * be2;
        const double C2 = al0 * be1 - al1 * be0;
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

// The pair of queue entry k: the main pass, then (if some lane's pair is one of the closest) the
// exact pass on those lanes.  The record is reloaded by the exact pass rather than kept.
template <bool SL, bool DL, int MODE, bool P234, bool LO, int NJ>
__device__ __forceinline__ void eval_pair(const SrcRec<double> *__restrict__ rec64, int k, const TgtV &T,
                                          const DevParams &p, double rare2, const double *__restrict__ tabs,
                                          AccN<NJ> &A)
{
    if constexpr (MODE == kModeTab) {
        tab_pair<SL, DL>(rec64[k], T, p, tabs, A);
        return;
    }
    bool rare;
    near_pair<SL, DL, MODE, P234, LO, NJ>(rec64[k], T, p, rare2, A, rare);
    if (__ballot(rare) && rare) {
        int kk = k;
        asm volatile("" : "+v"(kk));
        pair_exact<SL, DL, MODE, LO, NJ>(rec64[kk], T, p, A);
    }
}

// Pins a value to a vector register when PIN (see TgtV).  The double-precision path runs faster with
// its target data left to the compiler (scalar registers; near field at the 42k-source ellipsoid
// 2.47 -> 1.99 ms), the mixed path with them in vector registers (1.81 -> 1.76 ms).  The candidate
// test's coordinates and radius are always pinned: in single precision every operand of the test is
// then a vector register.
template <bool PIN, typename V>
__device__ __forceinline__ V to_vgpr(V v)
{
    if (PIN) asm volatile("" : "+v"(v));
    return v;
}

// MODE kModeComb: only the extrapolated values (weights known before the pair loop); kModePerDelta:
// also the per-delta values; kModeSharp: the targets on the surface under the modified smoothing.
template <typename TC, bool SL, bool DL, int MODE, bool P234>
__global__ __launch_bounds__(kBlock) void near_finalize_kernel(const SrcRec<double> *__restrict__ rec64,
                                                               const Pos4<TC> *__restrict__ pos,
                                                               const int *__restrict__ cell_start, CellGrid grid,
                                                               EvalArgs a, DevParams p, TC rc2, TC rc2s,
                                                               const double *__restrict__ part, int nparts,
                                                               NearFlag *__restrict__ flag)
{
    // single-precision candidate test = the mixed-precision path: the degree-11 erfcx table
    constexpr bool kLo = std::is_same<TC, float>::value;
    constexpr bool SHARP = MODE == kModeSharp;
    constexpr bool TAB = MODE == kModeTab;
    constexpr int NJ = MODE == kModePerDelta ? 3 : 1;
    __shared__ int queue_all[kBlock / kWave][kRing];
    __shared__ double2 tab_all[TAB ? kTabDoubles / 2 : 1];
    const double *tabs = reinterpret_cast<const double *>(tab_all);
    // readfirstlane: the wave index (hence the target) is wavefront-uniform
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int lane = (int)threadIdx.x % kWave;
    int *queue = queue_all[wave];
    // the target of this wavefront: slot-th in the target order (see DevParams::order)
    const int64_t slot = (int64_t)blockIdx.x * (kBlock / kWave) + wave;
    const int64_t t =
        (p.order != nullptr && slot < a.m) ? (int64_t)__builtin_amdgcn_readfirstlane(p.order[slot]) : slot;
    if constexpr (TAB) {
        // the workgroup copies the smoothing table into LDS if any of its targets is on the surface;
        // every wave reaches the barriers before leaving
        const bool mine = t < a.m && a.b[t] == 0.0;
        if (!__syncthreads_or(mine)) return;
        const double2 *src = reinterpret_cast<const double2 *>(p.tab);
        for (int k = (int)threadIdx.x; k < kTabDoubles / 2; k += kBlock) tab_all[k] = src[k];
        __syncthreads();
        if (!mine) return;
    }
    if (t >= a.m) return;  // wavefront-uniform exit

    double ty[3], tn[3], tq0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ty[i] = a.y[3 * t + i];
        tn[i] = a.n0[3 * t + i];
        tq0[i] = DL ? a.q0[3 * t + i] : 0.0;
    }
    const double tb = a.b[t];
    // a target on the surface with the modified smoothing selected: one delta, no extrapolation; the
    // SHARP instance takes exactly these targets, the others every other target (wavefront-uniform)
    const bool sharp = p.sharp && tb == 0.0;
    if (sharp != SHARP) return;
    // with the smoothing table the TAB instance takes the targets on the surface
    if (MODE == kModeComb && p.tab != nullptr && tb == 0.0) return;
    const double tc = SL ? a.f0[3 * t] * tn[0] + a.f0[3 * t + 1] * tn[1] + a.f0[3 * t + 2] * tn[2] : 0.0;
    double w[3] = {1.0, 0.0, 0.0};
    if (MODE == kModeComb) extrap_weights_wave(tb, p, lane, w);

    TgtV T;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T.y[i] = to_vgpr<kLo>(ty[i]);
        T.n[i] = to_vgpr<kLo>(tn[i]);
        T.q0[i] = to_vgpr<kLo>(tq0[i]);
        T.w[i] = to_vgpr<kLo>(w[i]);
    }
    T.b = to_vgpr<kLo>(tb);
    T.c = to_vgpr<kLo>(tc);
    const TC tyx = to_vgpr<true>((TC)(ty[0] - a.org[0])), tyy = to_vgpr<true>((TC)(ty[1] - a.org[1])),
             tyz = to_vgpr<true>((TC)(ty[2] - a.org[2]));
    const TC rcv = to_vgpr<true>(SHARP ? rc2s : rc2);
    // pairs closer than kSeriesT times the largest delta (the sharp delta for SHARP) go to pair_exact
    const double rare2 = SHARP ? (kSeriesT / p.inv_dsharp) * (kSeriesT / p.inv_dsharp)
                               : (kSeriesT / p.inv_delta[2]) * (kSeriesT / p.inv_delta[2]);
    // the far rule of the extrapolation (w = (1, 0, 0)) asserts that no source is within
    // cutoff * max delta: checked against the candidates (wavefront-uniform)
    const bool farrule = !SHARP && fabs(tb) >= p.cutoff * p.rho[2] * p.h;
    const TC rflag2 = (TC)(p.rflag * p.rflag);
    bool bad = false;

    // cells within the reach (near radius plus the rounding margin) of the target, per axis; in the
    // xy-plane a column of cells whose box lies farther than the reach is skipped
    const double R = SHARP ? p.reach_sharp : p.reach;
    int lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double l = floor((ty[d] - R - grid.lo[d]) * grid.inv_side);
        const double u = floor((ty[d] + R - grid.lo[d]) * grid.inv_side);
        lo[d] = (int)fmax(l, 0.0);
        hi[d] = (int)fmin(u, (double)grid.g[d] - 1.0);
    }

    AccN<NJ> A;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        A.dn[j] = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) A.sl[j][i] = A.dl[j][i] = 0.0;
    }

    // Candidates are loaded kDepth steps of 64 at a time, so that kDepth loads are in flight per
    // wavefront; the near ones go to a ring buffer in LDS (kRing >= 63 + kDepth * 64 entries) and every
    // full 64 are evaluated.  The columns of the block are set up in parallel, one per lane (up to 64
    // per pass): a column whose xy-box lies farther than the reach is dropped, the others load their
    // record range [cs, ce); the wavefront then scans the live columns in order.
    constexpr int kDepth = depth_for<TC>();
    int head = 0, cnt = 0;  // ring buffer start and length (wavefront-uniform)
    const double R2 = R * R;
    const int nyc = hi[1] - lo[1] + 1;
    const int ncol = (hi[0] >= lo[0] && hi[1] >= lo[1] && hi[2] >= lo[2]) ? (hi[0] - lo[0] + 1) * nyc : 0;
    for (int cb0 = 0; cb0 < ncol; cb0 += kWave) {
        int cs = 0, ce = 0;
        {
            const int j = cb0 + lane;
            if (j < ncol) {
                const int jx = j / nyc;
                const int ix = lo[0] + jx, iy = lo[1] + (j - jx * nyc);
                const double cx = grid.lo[0] + ix * grid.side, cy = grid.lo[1] + iy * grid.side;
                const double ex = fmax(0.0, fmax(cx - ty[0], ty[0] - (cx + grid.side)));
                const double ey = fmax(0.0, fmax(cy - ty[1], ty[1] - (cy + grid.side)));
                if (ex * ex + ey * ey <= R2) {
                    const int cb = (ix * grid.g[1] + iy) * grid.g[2];
                    cs = cell_start[cb + lo[2]];
                    ce = cell_start[cb + hi[2] + 1];
                }
            }
        }
        for (uint64_t live = __ballot(ce > cs); live; live &= live - 1) {
            const int jl = (int)__builtin_ctzll(live);
            const int s0 = __builtin_amdgcn_readlane(cs, jl), s1 = __builtin_amdgcn_readlane(ce, jl);
            for (int base = s0; base < s1; base += kDepth * kWave) {
                // only the steps of 64 that hold candidates (a wavefront-uniform count); the index is
                // clamped to the column so that every lane loads (no divergent branch)
                const int nsl = min(kDepth, (s1 - base + kWave - 1) / kWave);
                Pos4<TC> q[kDepth];
#pragma unroll
                for (int u = 0; u < kDepth; ++u)
                    if (u < nsl) q[u] = pos[min(base + u * kWave + lane, s1 - 1)];
#pragma unroll
                for (int u = 0; u < kDepth; ++u) {
                    if (u >= nsl) break;
                    const int k = base + u * kWave + lane;
                    const TC r2c = pair_r2(tyx, tyy, tyz, q[u].x, q[u].y, q[u].z);
                    const bool nr = k < s1 && r2c <= rcv;
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
                    eval_pair<SL, DL, MODE, P234, kLo, NJ>(rec64, k2, T, p, rare2, tabs, A);
                }
            }
        }
    }
    wave_lds_sync();
    if (lane < cnt)
        eval_pair<SL, DL, MODE, P234, kLo, NJ>(rec64, queue[(head + lane) & (kRing - 1)], T, p, rare2, tabs, A);
    if (farrule && __ballot(bad) && lane == 0) {
        atomicOr(&flag->bits, kFlagFarRule);
        atomicMin(&flag->first, (unsigned long long)t);
    }

#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (DL) A.dn[j] = wave_sum(A.dn[j]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (SL) A.sl[j][i] = wave_sum(A.sl[j][i]);
            if (DL) A.dl[j][i] = __builtin_fma(tn[i], A.dn[j], wave_sum(A.dl[j][i]));
        }
    }

    const double chi = tb < 0.0 ? 1.0 : (tb > 0.0 ? 0.0 : 0.5);
    const double inv8pi = 1.0 / (8.0 * kPi);

    if (MODE != kModePerDelta) {
        // combined (or single-delta) sums: u = (far + sum_j w_j near_j) / (8 pi)
        if (lane < 3) {
            const int i = lane;
            if (SL) {
                double far = 0.0;
                for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + i) * (size_t)a.m + t];
                a.u[3 * t + i] = (far + pick3(A.sl[0], i)) * inv8pi;
                if (a.u_delta)
#pragma unroll
                    for (int j = 0; j < 3; ++j) a.u_delta[9 * t + 3 * p.ord[j] + i] = a.u[3 * t + i];
            }
            if (DL) {
                double far = 0.0;
                for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + 3 + i) * (size_t)a.m + t];
                const double vv = -6.0 * (far + pick3(A.dl[0], i)) * inv8pi;
                a.v[3 * t + i] = vv + chi * pick3(tq0, i);
                if (a.v_delta)
#pragma unroll
                    for (int j = 0; j < 3; ++j) a.v_delta[9 * t + 3 * p.ord[j] + i] = vv;
            }
        }
        return;
    }

    double wx[3];
    extrap_weights_wave(tb, p, lane, wx);
    if (lane < 3) {
        const int i = lane;
        if (SL) {
            double far = 0.0;
            for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + i) * (size_t)a.m + t];
            double uj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) uj[j] = (far + pick3(A.sl[j], i)) * inv8pi;
            a.u[3 * t + i] = wx[0] * uj[0] + wx[1] * uj[1] + wx[2] * uj[2];
            if (a.u_delta)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.u_delta[9 * t + 3 * p.ord[j] + i] = uj[j];
        }
        if (DL) {
            double far = 0.0;
            for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + 3 + i) * (size_t)a.m + t];
            double vj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) vj[j] = -6.0 * (far + pick3(A.dl[j], i)) * inv8pi;
            a.v[3 * t + i] = wx[0] * vj[0] + wx[1] * vj[1] + wx[2] * vj[2] + chi * pick3(tq0, i);
            if (a.v_delta)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.v_delta[9 * t + 3 * p.ord[j] + i] = vj[j];
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
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, kModeComb, true>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    else if (p.pow234)
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, kModePerDelta, true>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    else if (comb)
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, kModeComb, false>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    else
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, kModePerDelta, false>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p.tab != nullptr) {  // set only for the combined mode without the modified smoothing
        hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, kModeTab, false>), grid, block, 0, s, rec64, pos,
                           cell_start, g, a, p, rc2, rc2s, part, nparts, flag);
        return hipGetLastError();
    }
    if (!p.sharp) return hipSuccess;
    hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL, kModeSharp, false>), grid, block, 0, s, rec64, pos,
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

__global__ void flag_clear_kernel(NearFlag *flag, int n)
{
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
        flag[i].bits = 0u;
        flag[i].first = ~0ull;
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

hipError_t launch_flag_clear(NearFlag *flag, int n, hipStream_t s)
{
    hipLaunchKernelGGL(flag_clear_kernel, dim3(1), dim3(kBlock), 0, s, flag, n);
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

// ---- the smoothing table of the targets on the surface (NearTable in sr_internal.h) ----
namespace {

// s1 / t, s2 / t^3, s3 / t^5 and e^{-t^2} at t >= 0 in long double (eqs. (s1)-(s3): s1 = erf t,
// s2 = erf t - (2/sqrt(pi)) t e^{-t^2}, s3 = s2 - (4/(3 sqrt(pi))) t^3 e^{-t^2}); Maclaurin series below
// t = 1 (the differences lose the relative accuracy of s2 ~ t^3 and s3 ~ t^5 there), closed forms above.
void smoothing_ratios_ld(long double t, long double &r1, long double &r2, long double &r3, long double &E)
{
    const long double c = 1.128379167095512573896158903121545172L;  // 2 / sqrt(pi)
    E = expl(-t * t);
    if (t < 1.0L) {
        const long double t2 = t * t;
        long double f = 1.0L, p = 1.0L, a1 = 0.0L, a2 = 0.0L, a3 = 0.0L;  // f = (-1)^n / n!, p = t^2n
        for (int n = 0; n < 40; ++n) {
            a1 += f * p / (2 * n + 1);
            a2 += 2.0L * f * p / (2 * n + 3);
            a3 += 4.0L * f * p / (3.0L * (2 * n + 5));
            f = -f / (n + 1);
            p *= t2;
        }
        r1 = c * a1;
        r2 = c * a2;
        r3 = c * a3;
        return;
    }
    const long double s1 = erfl(t);
    const long double s2 = s1 - c * t * E;
    const long double s3 = s2 - (2.0L / 3.0L) * c * t * t * t * E;
    r1 = s1 / t;
    r2 = s2 / (t * t * t);
    r3 = s3 / (t * t * t * t * t);
}

// g1, g2, g3 at x = r / h (see NearTable) for the weights w of the sorted ratios rho
void table_functions_ld(long double x, const long double rho[3], const long double w[3], long double cutoff,
                        long double g[kTabFuncs])
{
    g[0] = g[1] = g[2] = 0.0L;
    for (int j = 0; j < 3; ++j) {
        const long double t = x / rho[j];
        if (t > cutoff) {  // s_k = 1 beyond the cut-off (paper section 3.2); x > 0 here
            g[0] += w[j] / x;
            g[1] += w[j] / (x * x * x);
            g[2] += w[j] / (x * x * x * x * x);
            continue;
        }
        long double r1, r2, r3, E;
        smoothing_ratios_ld(t, r1, r2, r3, E);
        const long double p1 = rho[j], p3 = p1 * p1 * p1, p5 = p3 * p1 * p1;
        g[0] += w[j] * r1 / p1;
        g[1] += w[j] * r2 / p3;
        g[2] += w[j] * r3 / p5;
    }
}

}  // namespace

bool build_near_table(const double rho_d[3], double cutoff, double X, std::vector<double> &tab, double *maxerr)
{
    tab.clear();
    *maxerr = 0.0;
    long double rho[3], w[3];
    for (int j = 0; j < 3; ++j) rho[j] = rho_d[j];
    // extrapolation weights at b = 0 (eq. (extrap_eqn)): rows [1, rho_j I0(0), rho_j^3 I2(0)] with
    // I0(0) = 1/sqrt(pi), I2(0) = 1/(3 sqrt(pi)); w = e_1^T A^{-1} by Cramer's rule (the common factor
    // 1/sqrt(pi) cancels)
    long double al[3], be[3];
    for (int j = 0; j < 3; ++j) {
        al[j] = rho[j];
        be[j] = rho[j] * rho[j] * rho[j] / 3.0L;
    }
    const long double C0 = al[1] * be[2] - al[2] * be[1], C1 = al[2] * be[0] - al[0] * be[2],
                      C2 = al[0] * be[1] - al[1] * be[0];
    const long double D = C0 + C1 + C2;
    if (!(fabsl(D) > 0.0L) || !(X > 0.0)) return false;
    w[0] = C0 / D;
    w[1] = C1 / D;
    w[2] = C2 / D;
    const long double dx = (long double)X / kTabIntervals, pi = 3.141592653589793238462643383279502884L;
    std::vector<double> t((size_t)kTabDoubles);
    long double gmax[kTabFuncs] = {0.0L, 0.0L, 0.0L};
    // interpolation at the Chebyshev points of each interval, monomial coefficients in s
    for (int i = 0; i < kTabIntervals; ++i) {
        long double V[kTabCoef][kTabCoef], F[kTabFuncs][kTabCoef];
        for (int k = 0; k < kTabCoef; ++k) {
            const long double sk = 0.5L * cosl((2 * k + 1) * pi / (2 * kTabCoef));
            long double g[kTabFuncs];
            table_functions_ld(dx * (i + 0.5L + sk), rho, w, cutoff, g);
            long double pw = 1.0L;
            for (int e = 0; e < kTabCoef; ++e) {
                V[k][e] = pw;
                pw *= sk;
            }
            for (int f = 0; f < kTabFuncs; ++f) {
                F[f][k] = g[f];
                gmax[f] = std::max(gmax[f], fabsl(g[f]));
            }
        }
        // Gaussian elimination with partial pivoting, one right-hand side per function
        for (int col = 0; col < kTabCoef; ++col) {
            int piv = col;
            for (int r = col + 1; r < kTabCoef; ++r)
                if (fabsl(V[r][col]) > fabsl(V[piv][col])) piv = r;
            if (piv != col) {
                for (int e = 0; e < kTabCoef; ++e) std::swap(V[col][e], V[piv][e]);
                for (int f = 0; f < kTabFuncs; ++f) std::swap(F[f][col], F[f][piv]);
            }
            for (int r = col + 1; r < kTabCoef; ++r) {
                const long double m = V[r][col] / V[col][col];
                for (int e = col; e < kTabCoef; ++e) V[r][e] -= m * V[col][e];
                for (int f = 0; f < kTabFuncs; ++f) F[f][r] -= m * F[f][col];
            }
        }
        for (int f = 0; f < kTabFuncs; ++f)
            for (int r = kTabCoef - 1; r >= 0; --r) {
                long double acc = F[f][r];
                for (int e = r + 1; e < kTabCoef; ++e) acc -= V[r][e] * F[f][e];
                F[f][r] = acc / V[r][r];
                t[(((size_t)f * (kTabCoef / 2) + r / 2) * kTabIntervals + i) * 2 + (r & 1)] = (double)F[f][r];
            }
    }
    // check: the double-precision Horner evaluation the kernel performs against long double, at 17
    // points per interval (both ends included)
    long double err = 0.0L;
    for (int i = 0; i < kTabIntervals; ++i)
        for (int q = 0; q <= 16; ++q) {
            const double sv = -0.5 + q / 16.0;
            long double g[kTabFuncs];
            table_functions_ld(dx * (i + 0.5L + sv), rho, w, cutoff, g);
            for (int f = 0; f < kTabFuncs; ++f) {
                auto coef = [&](int e) { return t[(((size_t)f * (kTabCoef / 2) + e / 2) * kTabIntervals + i) * 2 + (e & 1)]; };
                double v = coef(kTabDegree);
                for (int e = kTabDegree - 1; e >= 0; --e) v = std::fma(v, sv, coef(e));
                err = std::max(err, fabsl((long double)v - g[f]) / gmax[f]);
            }
        }
    *maxerr = (double)err;
    if (!(err <= 5e-14L)) return false;
    tab.swap(t);
    return true;
}

}  // namespace sr

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
// The far-field partial sums are then added (eq. (near_far)) and the three values are combined by
// the 3x3 extrapolation of eq. (extrap_eqn): u = sum_j w_j u^{delta_j}, w = e_1^T A^{-1} with rows
// A_j = [1, rho_j I0(lambda_j), rho_j^3 I2(lambda_j)], lambda_j = b/delta_j, by Cramer's rule.
// If |b| >= cutoff * max delta every pair is beyond the cut-off for every delta, the three values
// coincide and w = (1, 0, 0) (the matrix is numerically singular there).
// Double layer: + chi q0 with chi = 1, 0, 1/2 for b < 0, b > 0, b == 0 (eq. (Stokes_DL1)).
//
// Work decomposition: one wavefront per target (4 per workgroup).  The target's cell and its
// neighbours in the uniform cell grid (side >= near radius) hold every near pair; with cells in
// z-fastest order, the 27 neighbour cells are 9 contiguous record ranges, read coalesced by the 64
// lanes.  Per-lane FP64 partial sums are combined by a butterfly wavefront reduction.
#include <math.h>

#include "sr_internal.h"

namespace sr {
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

template <typename TC, bool SL, bool DL>
__global__ __launch_bounds__(kBlock) void near_finalize_kernel(const SrcRec<double> *__restrict__ rec64,
                                                               const SrcRec<TC> *__restrict__ recc,
                                                               const int *__restrict__ cell_start, CellGrid grid,
                                                               EvalArgs a, DevParams p, TC rc2,
                                                               const double *__restrict__ part, int nparts)
{
    const int wave = (int)threadIdx.x / kWave;
    const int lane = (int)threadIdx.x % kWave;
    const int64_t t = (int64_t)blockIdx.x * (kBlock / kWave) + wave;
    if (t >= a.m) return;  // wavefront-uniform exit

    const double yx = a.y[3 * t], yy = a.y[3 * t + 1], yz = a.y[3 * t + 2];
    const double x0x = a.x0[3 * t], x0y = a.x0[3 * t + 1], x0z = a.x0[3 * t + 2];
    const double nx = a.n0[3 * t], ny = a.n0[3 * t + 1], nz = a.n0[3 * t + 2];
    const double b = a.b[t];
    double c = 0.0, q0x = 0.0, q0y = 0.0, q0z = 0.0;
    if (SL) c = a.f0[3 * t] * nx + a.f0[3 * t + 1] * ny + a.f0[3 * t + 2] * nz;
    if (DL) {
        q0x = a.q0[3 * t];
        q0y = a.q0[3 * t + 1];
        q0z = a.q0[3 * t + 2];
    }
    const TC tyx = (TC)yx, tyy = (TC)yy, tyz = (TC)yz;

    int ci[3];
    {
        const double yv[3] = {yx, yy, yz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double u = floor((yv[d] - grid.lo[d]) * grid.inv_side);
            u = fmin(fmax(u, -2.0), (double)grid.g[d] + 1.0);
            ci[d] = (int)u;
        }
    }

    double asl[3][3], adl[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) asl[j][i] = adl[j][i] = 0.0;

    const int z0 = max(ci[2] - 1, 0), z1 = min(ci[2] + 1, grid.g[2] - 1);
    for (int ix = max(ci[0] - 1, 0); ix <= min(ci[0] + 1, grid.g[0] - 1); ++ix) {
        for (int iy = max(ci[1] - 1, 0); iy <= min(ci[1] + 1, grid.g[1] - 1); ++iy) {
            if (z0 > z1) continue;
            const int cb = (ix * grid.g[1] + iy) * grid.g[2];
            const int s0 = cell_start[cb + z0], s1 = cell_start[cb + z1 + 1];
            for (int k = s0 + lane; k < s1; k += kWave) {
                const SrcRec<TC> &sc = recc[k];
                const TC r2c = pair_r2(tyx, tyy, tyz, sc.x, sc.y, sc.z);
                if (!(r2c <= rc2)) continue;
                const SrcRec<double> s = rec64[k];
                const double dx = yx - s.x, dy = yy - s.y, dz = yz - s.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) {
                    // target on a quadrature point: limit of s1(r/delta)/r is 2/(sqrt(pi) delta);
                    // the d d s2/r^3 term and the whole double-layer term vanish
                    if (SL) {
                        const double gx = s.fw[0] - c * s.nw[0], gy = s.fw[1] - c * s.nw[1],
                                     gz = s.fw[2] - c * s.nw[2];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            const double l = kTwoOverSqrtPi * p.inv_delta[j];
                            asl[j][0] += gx * l;
                            asl[j][1] += gy * l;
                            asl[j][2] += gz * l;
                        }
                    }
                    continue;
                }
                const double ir = rsqrt(r2);
                const double r = r2 * ir;
                const double ir3 = ir * ir * ir;
                const double ir5 = ir3 * ir * ir;
                double gx = 0, gy = 0, gz = 0, dg = 0;
                if (SL) {
                    gx = s.fw[0] - c * s.nw[0];
                    gy = s.fw[1] - c * s.nw[1];
                    gz = s.fw[2] - c * s.nw[2];
                    dg = dx * gx + dy * gy + dz * gz;
                }
                double t1x = 0, t1y = 0, t1z = 0, ex = 0, ey = 0, ez = 0;
                if (DL) {
                    const double hx = s.x - x0x, hy = s.y - x0y, hz = s.z - x0z;
                    const double ax = s.q[0] - q0x, ay = s.q[1] - q0y, az = s.q[2] - q0z;
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
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double tt = r * p.inv_delta[j];
                    double s1 = 1.0, s2 = 1.0, s3 = 1.0;
                    if (tt <= p.cutoff) {
                        const double e = exp(-tt * tt);
                        const double er = erf(tt);
                        const double ce = kTwoOverSqrtPi * tt * e;
                        s1 = er;
                        s2 = er - ce;
                        s3 = er - kTwoOverSqrtPi * (tt + (2.0 / 3.0) * tt * tt * tt) * e;
                    }
                    if (SL) {
                        const double k1 = s1 * ir, k2 = dg * s2 * ir3;
                        asl[j][0] += gx * k1 + dx * k2;
                        asl[j][1] += gy * k1 + dy * k2;
                        asl[j][2] += gz * k1 + dz * k2;
                    }
                    if (DL) {
                        const double k2 = s2 * ir3, k3 = s3 * ir5;
                        adl[j][0] += t1x * k2 + ex * k3;
                        adl[j][1] += t1y * k2 + ey * k3;
                        adl[j][2] += t1z * k2 + ez * k3;
                    }
                }
            }
        }
    }

#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (SL) asl[j][i] = wave_sum(asl[j][i]);
            if (DL) adl[j][i] = wave_sum(adl[j][i]);
        }

    // extrapolation weights (the same for the single and double layer and for every component)
    double w0 = 1.0, w1 = 0.0, w2 = 0.0;
    const double dmax = fmax(p.rho[0], fmax(p.rho[1], p.rho[2])) * p.h;
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
        w0 = C0 / D;
        w1 = C1 / D;
        w2 = C2 / D;
    }
    const double chi = b < 0.0 ? 1.0 : (b > 0.0 ? 0.0 : 0.5);
    const double inv8pi = 1.0 / (8.0 * kPi);

    if (lane < 3) {
        const int i = lane;
        if (SL) {
            double far = 0.0;
            for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + i) * (size_t)a.m + t];
            double uj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) uj[j] = (far + asl[j][i]) * inv8pi;
            a.u[3 * t + i] = w0 * uj[0] + w1 * uj[1] + w2 * uj[2];
            if (a.u_delta)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.u_delta[9 * t + 3 * j + i] = uj[j];
        }
        if (DL) {
            double far = 0.0;
            for (int sp = 0; sp < nparts; ++sp) far += part[((size_t)sp * 6 + 3 + i) * (size_t)a.m + t];
            double vj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) vj[j] = -6.0 * (far + adl[j][i]) * inv8pi;
            const double q0i = i == 0 ? q0x : (i == 1 ? q0y : q0z);
            a.v[3 * t + i] = w0 * vj[0] + w1 * vj[1] + w2 * vj[2] + chi * q0i;
            if (a.v_delta)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.v_delta[9 * t + 3 * j + i] = vj[j];
        }
    }
}

template <typename TC, bool SL, bool DL>
hipError_t launch_t(const SrcRec<double> *rec64, const SrcRec<TC> *recc, const int *cell_start, const CellGrid &g,
                    const EvalArgs &a, const DevParams &p, TC rc2, const double *part, int nparts, hipStream_t s)
{
    const int per_block = kBlock / kWave;
    const int64_t blocks = (a.m + per_block - 1) / per_block;
    hipLaunchKernelGGL((near_finalize_kernel<TC, SL, DL>), dim3((unsigned)blocks), dim3(kBlock), 0, s, rec64, recc,
                       cell_start, g, a, p, rc2, part, nparts);
    return hipGetLastError();
}

template <typename TC>
hipError_t dispatch(int layers, const SrcRec<double> *rec64, const SrcRec<TC> *recc, const int *cell_start,
                    const CellGrid &g, const EvalArgs &a, const DevParams &p, TC rc2, const double *part,
                    int nparts, hipStream_t s)
{
    if (layers == (SR_SL | SR_DL))
        return launch_t<TC, true, true>(rec64, recc, cell_start, g, a, p, rc2, part, nparts, s);
    if (layers == SR_SL) return launch_t<TC, true, false>(rec64, recc, cell_start, g, a, p, rc2, part, nparts, s);
    return launch_t<TC, false, true>(rec64, recc, cell_start, g, a, p, rc2, part, nparts, s);
}

}  // namespace

hipError_t launch_near_finalize(int precision, int layers, const SrcRec<double> *rec64,
                                const SrcRec<float> *rec32, const int *cell_start, const CellGrid &grid,
                                const EvalArgs &a, const DevParams &p, const double *part, int nparts,
                                hipStream_t s)
{
    const double rc2 = p.rnear * p.rnear;
    if (precision == SR_MIXED)
        return dispatch<float>(layers, rec64, rec32, cell_start, grid, a, p, (float)rc2, part, nparts, s);
    return dispatch<double>(layers, rec64, rec64, cell_start, grid, a, p, rc2, part, nparts, s);
}

}  // namespace sr

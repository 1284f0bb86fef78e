// Far-field direct sum of the extrapolated-regularization method (paper section 3.3, eq. (near_far)):
// for every target, the pairs farther than the near radius are summed ONCE with the original
// Stokeslet (eq. (Stokeslet)) and stresslet (eq. (Stresslet)) kernels, applied to the subtracted
// densities of eqs. (Stokes_SL1), (Stokes_DL1).  The result is shared by the three smoothing lengths.
//
// Work decomposition (MI355X, 256 CUs in 8 XCDs):
//   - each workgroup (256 lanes) owns a tile of targets and one of kFarSplits (16) contiguous source
//     ranges; blockIdx.x % 16 selects the range, so the round-robin dispatch over the 8 XCDs gives
//     every XCD's L2 two sixteenths of the source records;
//   - double precision (far_direct_kernel): two targets per lane; the source index is
//     wavefront-uniform, so each record is fetched once per wavefront through the scalar data cache
//     and feeds the VALU as scalar operands (double-precision instructions issue at one rate
//     whatever their operands): no LDS, no barriers;
//   - mixed precision (far_lds_kernel): pair arithmetic in FP32, one target per lane, every operand
//     in a vector register (see there), 32-pair FP32 partial sums promoted to FP64;
//   - near pairs (r^2 <= rc2 by the shared pair_r2 test) are selected out (not multiplied by zero:
//     r can be 0); rc2 is the target's: the smaller radius of the modified smoothing for targets on
//     the surface when it is selected, the near radius otherwise;
//   - output: per-split partial sums part[split][channel][target], channel 0..2 = single-layer
//     sum of S g, channel 3..5 = sum of d (d.a)(d.m) / r^5 (the -6 and 1/(8 pi) are applied
//     when the near-field kernel combines the parts).
// Targets with no closest point (PLAIN instance, sr_eval_far): g = f w and a = q, the plain sums of
// eqs. (Stokes_SL), (Stokes_DL) with no subtraction; a target that has a pair inside the near radius
// needs the near-field treatment (and x0) and is reported in the context's NearFlag.  Such targets
// may lie far from the single-precision origin, where rounding y - org to FP32 would move them by
// 2^-24 |y - org|: the instance keeps the rounding remainder y_lo and forms d = (y_hi - x) + y_lo.
#include <type_traits>

#include "sr_internal.h"

namespace sr {
namespace {

constexpr int kTile = 32;  // FP32 partial-sum length before promotion to FP64

struct Org3 {
    double v[3];
    __device__ double operator[](int i) const { return v[i]; }
};

// 1/r for a far pair, 0 for a near pair, without a branch (behind a select the compiler would put the
// double-precision rsqrt sequence in a divergent branch)
__device__ __forceinline__ float far_ir(float r2, float rc2) { return r2 > rc2 ? __builtin_amdgcn_rsqf(r2) : 0.0f; }
__device__ __forceinline__ double far_ir(double r2, double rc2)
{
    // hardware estimate (relative error ~5e-8 measured on MI355X) and one Newton step written as
    // y <- y (3/2 - (r2/2) y^2): the relative error becomes (3/2) eps^2 ~ 4e-15 plus a few roundings,
    // four instructions after the estimate (two steps of y + (y/2)(1 - r2 y^2) took eight and gained
    // nothing the 1e-10 bar of the double-precision path can see).  No handling of zero or infinite
    // arguments: a near pair (possibly r2 = 0, giving NaN here) is selected out.
    const double y = __builtin_amdgcn_rsq(r2);
    const double t = (0.5 * r2) * y;
    const double e = __builtin_fma(-t, y, 1.5);
    return r2 > rc2 ? y * e : 0.0;
}
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Double-precision far field (T = double).  PT: per-target near radius (the modified smoothing is on);
// otherwise rc2 for every target, in a scalar register.  PLAIN: no subtraction, near pairs reported in
// *flag.
template <typename T, bool SL, bool DL, int TPL, bool PT, bool PLAIN>
__global__ __launch_bounds__(kBlock) void far_direct_kernel(const SrcRec<T> *__restrict__ src, int n, int chunk,
                                                            const double *__restrict__ y,
                                                            const double *__restrict__ n0,
                                                            const double *__restrict__ f0,
                                                            const double *__restrict__ q0,
                                                            const double *__restrict__ bt, int m, T rc2, T rc2s,
                                                            Org3 org, NearFlag *__restrict__ flag,
                                                            double *__restrict__ part)
{
    const int split = blockIdx.x % kFarSplits;
    const int tile = blockIdx.x / kFarSplits;
    const int p0 = split * chunk;
    const int p1 = min(n, p0 + chunk);

    T ty[TPL][3], tc[TPL], tq[TPL][3], tr2[TPL];
    int tix[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = (tile * TPL + k) * kBlock + (int)threadIdx.x;
        tix[k] = t;
        const int tt = t < m ? t : m - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) ty[k][i] = (T)(y[3 * tt + i] - org[i]);
        tc[k] = 0;
        if (SL && !PLAIN)
            tc[k] = (T)(f0[3 * tt] * n0[3 * tt] + f0[3 * tt + 1] * n0[3 * tt + 1] + f0[3 * tt + 2] * n0[3 * tt + 2]);
#pragma unroll
        for (int i = 0; i < 3; ++i) tq[k][i] = (DL && !PLAIN) ? (T)q0[3 * tt + i] : (T)0;
        // a target on the surface under the modified smoothing has the smaller near radius
        tr2[k] = (PT && bt[tt] == 0.0) ? rc2s : rc2;
    }
    bool has_near[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) has_near[k] = false;

    double acc[TPL][6];
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[k][c] = 0.0;

    for (int pb = p0; pb < p1; pb += kTile) {
        const int pe = min(pb + kTile, p1);
        T a[TPL][6];
#pragma unroll
        for (int k = 0; k < TPL; ++k)
#pragma unroll
            for (int c = 0; c < 6; ++c) a[k][c] = 0;
#pragma unroll 2
        for (int p = pb; p < pe; ++p) {
            const SrcRec<T> s = src[p];
#pragma unroll
            for (int k = 0; k < TPL; ++k) {
                const T dx = ty[k][0] - s.x, dy = ty[k][1] - s.y, dz = ty[k][2] - s.z;
                const T r2 = pair_r2(ty[k][0], ty[k][1], ty[k][2], s.x, s.y, s.z);
                const T ir = far_ir(r2, tr2[k]);
                if (PLAIN) has_near[k] = has_near[k] || !(r2 > tr2[k]);
                const T ir2 = ir * ir;
                const T ir3 = ir2 * ir;
                if (SL) {
                    const T gx = s.fw[0] - tc[k] * s.nw[0];
                    const T gy = s.fw[1] - tc[k] * s.nw[1];
                    const T gz = s.fw[2] - tc[k] * s.nw[2];
                    const T sc = (dx * gx + dy * gy + dz * gz) * ir3;
                    // explicit chains: a += g/r + d s as two fused multiply-adds per component
                    a[k][0] = fma_t(dx, sc, fma_t(gx, ir, a[k][0]));
                    a[k][1] = fma_t(dy, sc, fma_t(gy, ir, a[k][1]));
                    a[k][2] = fma_t(dz, sc, fma_t(gz, ir, a[k][2]));
                }
                if (DL) {
                    const T ax = s.q[0] - tq[k][0], ay = s.q[1] - tq[k][1], az = s.q[2] - tq[k][2];
                    const T da = dx * ax + dy * ay + dz * az;
                    const T dm = dx * s.nw[0] + dy * s.nw[1] + dz * s.nw[2];
                    const T co = da * dm * (ir3 * ir2);
                    a[k][3] = fma_t(dx, co, a[k][3]);
                    a[k][4] = fma_t(dy, co, a[k][4]);
                    a[k][5] = fma_t(dz, co, a[k][5]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TPL; ++k)
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[k][c] += (double)a[k][c];
    }

    if (PLAIN) {
#pragma unroll
        for (int k = 0; k < TPL; ++k)
            if (tix[k] < m && has_near[k]) {
                atomicOr(&flag->bits, kFlagFarTarget);
                atomicMin(&flag->first, (unsigned long long)tix[k]);
            }
    }

#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        if (tix[k] < m) {
            const size_t base = (size_t)split * 6 * (size_t)m + (size_t)tix[k];
            if (SL)
#pragma unroll
                for (int c = 0; c < 3; ++c) part[base + (size_t)c * m] = acc[k][c];
            if (DL)
#pragma unroll
                for (int c = 3; c < 6; ++c) part[base + (size_t)c * m] = acc[k][c];
        }
    }
}

// Single-precision far field with the sources staged in LDS.  On gfx950 a single-precision VALU
// instruction whose operands are all vector registers issues at about twice the rate of one that reads
// a scalar register (measured: 62-72e12 lane operations per second at 8 or more wavefronts per SIMD,
// against 33-37e12; double precision runs at the lower rate either way), and the higher rate needs
// many wavefronts (52e12 at 5 per SIMD).  So every operand of the pair arithmetic lives in VGPRs:
// each workgroup copies kStage source records of its range into LDS, every lane reads the current
// record with a wavefront-uniform address (an LDS broadcast, about 1.5 clocks per 16-byte read per
// CU, measured), the uniform near radius is pinned to a VGPR, and one target per lane keeps the
// kernel at 53 VGPRs (9 wavefronts per SIMD).  The pair test is the shared pair_r2 on the same
// rounded operands as the near-field kernel's.
constexpr int kStage = 512;  // records per LDS stage (24 KB)
template <bool SL, bool DL, int TPL, bool PT, bool PLAIN>
__global__ __launch_bounds__(kBlock) void far_lds_kernel(const SrcRec<float> *__restrict__ src, int n, int chunk,
                                                         const double *__restrict__ y,
                                                         const double *__restrict__ n0,
                                                         const double *__restrict__ f0,
                                                         const double *__restrict__ q0,
                                                         const double *__restrict__ bt, int m, float rc2,
                                                         float rc2s, Org3 org, NearFlag *__restrict__ flag,
                                                         double *__restrict__ part)
{
    __shared__ float4 st[kStage * 3];
    const int split = blockIdx.x % kFarSplits;
    const int tile = blockIdx.x / kFarSplits;
    const int p0 = split * chunk;
    const int p1 = min(n, p0 + chunk);

    float ty[TPL][3], tc[TPL], tq[TPL][3], tr2[TPL], tlo[TPL][3];
    int tix[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        const int t = (tile * TPL + k) * kBlock + (int)threadIdx.x;
        tix[k] = t;
        const int tt = t < m ? t : m - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double yr = y[3 * tt + i] - org[i];
            ty[k][i] = (float)yr;
            tlo[k][i] = (float)(yr - (double)ty[k][i]);
        }
        tc[k] = 0.0f;
        if (SL && !PLAIN)
            tc[k] = (float)(f0[3 * tt] * n0[3 * tt] + f0[3 * tt + 1] * n0[3 * tt + 1] + f0[3 * tt + 2] * n0[3 * tt + 2]);
#pragma unroll
        for (int i = 0; i < 3; ++i) tq[k][i] = (DL && !PLAIN) ? (float)q0[3 * tt + i] : 0.0f;
        tr2[k] = (PT && bt[tt] == 0.0) ? rc2s : rc2;
        // a uniform radius would otherwise sit in a scalar register and halve the compare's issue rate
        asm volatile("" : "+v"(tr2[k]));
    }
    bool has_near[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) has_near[k] = false;

    double acc[TPL][6];
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[k][c] = 0.0;

    const float4 *g4 = reinterpret_cast<const float4 *>(src);
    for (int sb = p0; sb < p1; sb += kStage) {
        const int cnt = min(kStage, p1 - sb);
        __syncthreads();  // every wave is done with the previous stage
        for (int i = (int)threadIdx.x; i < 3 * cnt; i += kBlock) st[i] = g4[3 * (size_t)sb + i];
        __syncthreads();
        for (int pb = 0; pb < cnt; pb += kTile) {
            const int pe = min(pb + kTile, cnt);
            float a[TPL][6];
#pragma unroll
            for (int k = 0; k < TPL; ++k)
#pragma unroll
                for (int c = 0; c < 6; ++c) a[k][c] = 0.0f;
            // the record index as a VGPR value: the broadcast reads then use a vector address with
            // immediate offsets instead of a scalar index moved into a VGPR per record
            int vp = 3 * pb;
            asm volatile("" : "+v"(vp));
#pragma unroll 4
            for (int p = 0; p < pe - pb; ++p) {
                const float4 A = st[vp + 3 * p], B = st[vp + 3 * p + 1], Cq = st[vp + 3 * p + 2];
                const float sx = A.x, sy = A.y, sz = A.z;
                const float fw0 = A.w, fw1 = B.x, fw2 = B.y, nw0 = B.z, nw1 = B.w, nw2 = Cq.x;
                const float qq0 = Cq.y, qq1 = Cq.z, qq2 = Cq.w;
#pragma unroll
                for (int k = 0; k < TPL; ++k) {
                    float dx = ty[k][0] - sx, dy = ty[k][1] - sy, dz = ty[k][2] - sz;
                    float r2;
                    if (PLAIN) {
                        dx += tlo[k][0];
                        dy += tlo[k][1];
                        dz += tlo[k][2];
                        r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                    } else {
                        r2 = pair_r2(ty[k][0], ty[k][1], ty[k][2], sx, sy, sz);
                    }
                    const float ir = far_ir(r2, tr2[k]);
                    if (PLAIN) has_near[k] = has_near[k] || !(r2 > tr2[k]);
                    const float ir2 = ir * ir;
                    const float ir3 = ir2 * ir;
                    if (SL) {
                        const float gx = fw0 - tc[k] * nw0;
                        const float gy = fw1 - tc[k] * nw1;
                        const float gz = fw2 - tc[k] * nw2;
                        const float sc = (dx * gx + dy * gy + dz * gz) * ir3;
                        a[k][0] = __builtin_fmaf(dx, sc, __builtin_fmaf(gx, ir, a[k][0]));
                        a[k][1] = __builtin_fmaf(dy, sc, __builtin_fmaf(gy, ir, a[k][1]));
                        a[k][2] = __builtin_fmaf(dz, sc, __builtin_fmaf(gz, ir, a[k][2]));
                    }
                    if (DL) {
                        const float ax = qq0 - tq[k][0], ay = qq1 - tq[k][1], az = qq2 - tq[k][2];
                        const float da = dx * ax + dy * ay + dz * az;
                        const float dm = dx * nw0 + dy * nw1 + dz * nw2;
                        const float co = da * dm * (ir3 * ir2);
                        a[k][3] = __builtin_fmaf(dx, co, a[k][3]);
                        a[k][4] = __builtin_fmaf(dy, co, a[k][4]);
                        a[k][5] = __builtin_fmaf(dz, co, a[k][5]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < TPL; ++k)
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[k][c] += (double)a[k][c];
        }
    }

    if (PLAIN) {
#pragma unroll
        for (int k = 0; k < TPL; ++k)
            if (tix[k] < m && has_near[k]) {
                atomicOr(&flag->bits, kFlagFarTarget);
                atomicMin(&flag->first, (unsigned long long)tix[k]);
            }
    }

#pragma unroll
    for (int k = 0; k < TPL; ++k) {
        if (tix[k] < m) {
            const size_t base = (size_t)split * 6 * (size_t)m + (size_t)tix[k];
            if (SL)
#pragma unroll
                for (int c = 0; c < 3; ++c) part[base + (size_t)c * m] = acc[k][c];
            if (DL)
#pragma unroll
                for (int c = 3; c < 6; ++c) part[base + (size_t)c * m] = acc[k][c];
        }
    }
}

template <typename T, bool SL, bool DL, bool PLAIN>
hipError_t launch_t(const SrcRec<T> *rec, int64_t n, const EvalArgs &a, T rc2, T rc2s, int sharp, NearFlag *flag,
                    double *part, hipStream_t s)
{
    // one target per lane in single precision (53 VGPRs, 9 wavefronts per SIMD, against 86 and 5 with
    // two: far field at the 42k-source ellipsoid 2.25 -> 1.97 ms), two in double precision
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr int TPL = kF32 ? 1 : 2;
    const int m = (int)a.m;
    const int tiles = (m + kBlock * TPL - 1) / (kBlock * TPL);
    const int chunk = (int)((n + kFarSplits - 1) / kFarSplits);
    const dim3 grid(tiles * kFarSplits), block(kBlock);
    const Org3 org{a.org[0], a.org[1], a.org[2]};
    if constexpr (kF32) {
        if (PLAIN)
            hipLaunchKernelGGL((far_lds_kernel<SL, DL, TPL, false, true>), grid, block, 0, s, rec, (int)n, chunk, a.y,
                               a.n0, a.f0, a.q0, a.b, m, rc2, rc2s, org, flag, part);
        else if (sharp)
            hipLaunchKernelGGL((far_lds_kernel<SL, DL, TPL, true, false>), grid, block, 0, s, rec, (int)n, chunk, a.y,
                               a.n0, a.f0, a.q0, a.b, m, rc2, rc2s, org, flag, part);
        else
            hipLaunchKernelGGL((far_lds_kernel<SL, DL, TPL, false, false>), grid, block, 0, s, rec, (int)n, chunk, a.y,
                               a.n0, a.f0, a.q0, a.b, m, rc2, rc2s, org, flag, part);
    } else {
        if (PLAIN)
            hipLaunchKernelGGL((far_direct_kernel<T, SL, DL, TPL, false, true>), grid, block, 0, s, rec, (int)n, chunk,
                               a.y, a.n0, a.f0, a.q0, a.b, m, rc2, rc2s, org, flag, part);
        else if (sharp)
            hipLaunchKernelGGL((far_direct_kernel<T, SL, DL, TPL, true, false>), grid, block, 0, s, rec, (int)n, chunk,
                               a.y, a.n0, a.f0, a.q0, a.b, m, rc2, rc2s, org, flag, part);
        else
            hipLaunchKernelGGL((far_direct_kernel<T, SL, DL, TPL, false, false>), grid, block, 0, s, rec, (int)n,
                               chunk, a.y, a.n0, a.f0, a.q0, a.b, m, rc2, rc2s, org, flag, part);
    }
    return hipGetLastError();
}

template <typename T, bool PLAIN>
hipError_t dispatch(int layers, const SrcRec<T> *rec, int64_t n, const EvalArgs &a, T rc2, T rc2s, int sharp,
                    NearFlag *flag, double *part, hipStream_t s)
{
    if (layers == (SR_SL | SR_DL)) return launch_t<T, true, true, PLAIN>(rec, n, a, rc2, rc2s, sharp, flag, part, s);
    if (layers == SR_SL) return launch_t<T, true, false, PLAIN>(rec, n, a, rc2, rc2s, sharp, flag, part, s);
    return launch_t<T, false, true, PLAIN>(rec, n, a, rc2, rc2s, sharp, flag, part, s);
}

}  // namespace

hipError_t launch_far_direct(int precision, int layers, const SrcRec<double> *rec64, const SrcRec<float> *rec32,
                             int64_t n, const EvalArgs &a, double rnear, double rsharp, int sharp, double *part,
                             hipStream_t s)
{
    const double rc2 = rnear * rnear, rc2s = rsharp * rsharp;
    if (precision == SR_MIXED)
        return dispatch<float, false>(layers, rec32, n, a, (float)rc2, (float)rc2s, sharp, nullptr, part, s);
    return dispatch<double, false>(layers, rec64, n, a, rc2, rc2s, sharp, nullptr, part, s);
}

hipError_t launch_far_plain(int precision, int layers, const SrcRec<double> *rec64, const SrcRec<float> *rec32,
                            int64_t n, const EvalArgs &a, double rnear, NearFlag *flag, double *part, hipStream_t s)
{
    const double rc2 = rnear * rnear;
    if (precision == SR_MIXED)
        return dispatch<float, true>(layers, rec32, n, a, (float)rc2, (float)rc2, 0, flag, part, s);
    return dispatch<double, true>(layers, rec64, n, a, rc2, rc2, 0, flag, part, s);
}

}  // namespace sr

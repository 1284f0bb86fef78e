// Rigid spheres in Stokes flow: the completed double-layer equation solved by GMRES, every integral
// evaluated with the extrapolated-regularization evaluator of this library (sr_eval, double layer).
//
//   (A q)(x) = -1/2 q(x) + sum_m DL_m[q_m](x) + sum_m C_m(x) = U_b + Omega_b x (x - c_b),  x on sphere b
//
//   DL_m     double layer of sphere m: on-surface for the sphere's own points (b = 0, chi = 1/2, the
//            principal value, paper eq. (Stokes_DL1)), nearly singular exterior evaluation for the other
//            spheres' points (x0 = closest point of sphere m, q(x0) interpolated);
//   C_m(x)   (1/8 pi) [ S(x - c_m) F_m + L_m x (x - c_m) / |x - c_m|^3 ],
//            F_m = sum_p q_p w_p, L_m = sum_p (x_p - c_m) x q_p w_p over sphere m (the completion that
//            removes the rigid-motion null space of -1/2 I + DL; Power & Miranda 1987).
//
// q(x0): tensor Lagrange interpolation on the grid of one quadrature family (paper section 2.2): the
// first of widths 6, 5, 4, 3, 2 points per axis (6 x 6: O(h^6)) and, per width, the families in
// decreasing |n_i(x0)| order whose stencil points all exist, on the sheet sign(n_i(x0)).  Stencils
// depend on the geometry only and are built on the host once; kStencil slots per target, unused ones
// with weight 0.
//
// GMRES(restart): Arnoldi with classical Gram-Schmidt applied twice (one block dot product and one
// block update per pass), Givens rotations on the host, residual estimate from the rotated right-hand
// side; the final relative residual is recomputed with one more matrix-vector product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sr_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kRed = 256;       // threads per reduction block
constexpr int kRedBlocks = 512;  // blocks of the first reduction pass

thread_local std::string g_rerr;

sr_status rfail(sr_status st, const char *msg)
{
    g_rerr = msg;
    return st;
}

#define RHIP(call)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) {                                                                       \
            g_rerr = std::string(#call) + " failed: " + hipGetErrorString(e_);                        \
            return e_ == hipErrorOutOfMemory ? SR_ENOMEM : SR_EHIP;                                   \
        }                                                                                             \
    } while (0)

#define RSR(call)                                                                                     \
    do {                                                                                              \
        sr_status s_ = (call);                                                                        \
        if (s_ != SR_OK) {                                                                            \
            g_rerr = std::string(#call) + ": " + sr_last_error();                                     \
            return s_;                                                                                \
        }                                                                                             \
    } while (0)

template <typename T>
struct Buf {
    T *p = nullptr;
    size_t n = 0;
    hipError_t alloc(size_t k)
    {
        if (p && n >= k) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void **)&p, std::max<size_t>(k, 1) * sizeof(T));
        if (e == hipSuccess) n = k;
        return e;
    }
    ~Buf()
    {
        if (p) (void)hipFree(p);
    }
};

// ---------------------------------------------------------------- kernels

constexpr int kStencilWidth = 6;
constexpr int kStencil = kStencilWidth * kStencilWidth;

// q0 of sphere m at every target: the density itself for the sphere's own points (targets
// [own0, own1), whose density sits at the same index), the interpolated density at the closest point
// otherwise (stencil indices relative to the sphere's first point soff).
__global__ void gather_q0_kernel(const double *__restrict__ q, int64_t nt, int64_t own0, int64_t own1,
                                 int64_t soff, const int *__restrict__ idx, const double *__restrict__ wts,
                                 double *__restrict__ q0)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double v[3] = {0.0, 0.0, 0.0};
    if (t >= own0 && t < own1) {
        for (int c = 0; c < 3; ++c) v[c] = q[3 * t + c];
    } else {
        for (int s = 0; s < kStencil; ++s) {
            const double wv = wts[(int64_t)kStencil * t + s];
            const int64_t p = soff + idx[(int64_t)kStencil * t + s];
            for (int c = 0; c < 3; ++c) v[c] += wv * q[3 * p + c];
        }
    }
    for (int c = 0; c < 3; ++c) q0[3 * t + c] = v[c];
}

__global__ void zero_kernel(double *__restrict__ y, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = 0.0;
}

// first pass of the completion strengths of one sphere: 6 sums (F, L) per block
__global__ __launch_bounds__(kRed) void strengths_kernel(const double *__restrict__ q, const double *__restrict__ x,
                                                         const double *__restrict__ w, int64_t off, int64_t nm,
                                                         double cx, double cy, double cz, double *__restrict__ part)
{
    __shared__ double sh[6][kRed];
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x; i < nm; i += (int64_t)gridDim.x * kRed) {
        const int64_t p = off + i;
        const double qx = q[3 * p] * w[p], qy = q[3 * p + 1] * w[p], qz = q[3 * p + 2] * w[p];
        const double rx = x[3 * p] - cx, ry = x[3 * p + 1] - cy, rz = x[3 * p + 2] - cz;
        a[0] += qx;
        a[1] += qy;
        a[2] += qz;
        a[3] += ry * qz - rz * qy;
        a[4] += rz * qx - rx * qz;
        a[5] += rx * qy - ry * qx;
    }
    for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int s = kRed / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 6; ++c) part[6 * blockIdx.x + c] = sh[c][0];
}

// fixed-order sum of the kRed values in sh (a binary tree); the result is in sh[0]
__device__ __forceinline__ void block_tree_sum(double *sh)
{
    __syncthreads();
    for (int st = kRed / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
}

// second pass of the strengths: FL[m][c] = sum over the blocks' partial sums; one workgroup per
// (m, c), each thread a fixed strided subset, then a fixed-order tree (reproducible)
__global__ __launch_bounds__(kRed) void strengths_final_kernel(const double *__restrict__ part, int nsph, int nblk,
                                                               double *__restrict__ FL)
{
    __shared__ double sh[kRed];
    const int i = (int)blockIdx.x;  // m * 6 + c
    const int m = i / 6, c = i % 6;
    double a = 0.0;
    for (int b = (int)threadIdx.x; b < nblk; b += kRed) a += part[((size_t)m * nblk + b) * 6 + c];
    sh[threadIdx.x] = a;
    block_tree_sum(sh);
    if (threadIdx.x == 0) FL[i] = sh[0];
}

// out = [-1/2 q] + sum_m v_m + sum_m C_m(y), FL[m] = (F_m, L_m)
// out = a_id q + a_dl sum_m v_m (+ the completion terms when `completion`)
__global__ void assemble_kernel(const double *__restrict__ q, const double *__restrict__ y, int64_t nt, int nsph,
                                const double *__restrict__ v, const double *__restrict__ centers,
                                const double *__restrict__ FLs, double *__restrict__ out, double a_id, double a_dl,
                                int completion)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double o[3] = {0.0, 0.0, 0.0};
    if (a_id != 0.0) {
        for (int c = 0; c < 3; ++c) o[c] = a_id * q[3 * t + c];
    }
    const double k = 1.0 / (8.0 * kPi);
    for (int m = 0; m < nsph; ++m) {
        for (int c = 0; c < 3; ++c) o[c] += a_dl * v[((size_t)m * nt + t) * 3 + c];
        if (!completion) continue;
        const double *FL = FLs + 6 * m;
        const double dx = y[3 * t] - centers[3 * m], dy = y[3 * t + 1] - centers[3 * m + 1],
                     dz = y[3 * t + 2] - centers[3 * m + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ir = 1.0 / sqrt(r2), ir3 = ir * ir * ir;
        const double dF = dx * FL[0] + dy * FL[1] + dz * FL[2];
        const double Lx = FL[3], Ly = FL[4], Lz = FL[5];
        o[0] += k * (FL[0] * ir + dx * dF * ir3 + (Ly * dz - Lz * dy) * ir3);
        o[1] += k * (FL[1] * ir + dy * dF * ir3 + (Lz * dx - Lx * dz) * ir3);
        o[2] += k * (FL[2] * ir + dz * dF * ir3 + (Lx * dy - Ly * dx) * ir3);
    }
    for (int c = 0; c < 3; ++c) out[3 * t + c] = o[c];
}

// block dot products: part[b][k] = sum over block b's range of V[k] . w, k < K
__global__ __launch_bounds__(kRed) void mdot_kernel(const double *__restrict__ V, size_t ld, int K,
                                                    const double *__restrict__ w, size_t n,
                                                    double *__restrict__ part)
{
    __shared__ double sh[kRed];
    for (int k = 0; k < K; ++k) {
        double a = 0.0;
        for (size_t i = (size_t)blockIdx.x * kRed + threadIdx.x; i < n; i += (size_t)gridDim.x * kRed)
            a += V[k * ld + i] * w[i];
        sh[threadIdx.x] = a;
        __syncthreads();
        for (int s = kRed / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * K + k] = sh[0];
        __syncthreads();
    }
}

// second pass: res[k] = sum_b part[b][k]; one workgroup per k, each thread a fixed strided subset of
// the blocks, then a fixed-order tree (reproducible)
__global__ __launch_bounds__(kRed) void mdot_final_kernel(const double *__restrict__ part, int nblk, int K,
                                                          double *__restrict__ res)
{
    __shared__ double sh[kRed];
    const int k = (int)blockIdx.x;
    double a = 0.0;
    for (int b = (int)threadIdx.x; b < nblk; b += kRed) a += part[(size_t)b * K + k];
    sh[threadIdx.x] = a;
    block_tree_sum(sh);
    if (threadIdx.x == 0) res[k] = sh[0];
}

// w -= sum_k V[k] c[k]   (c on the device)
__global__ void mupdate_kernel(const double *__restrict__ V, size_t ld, int K, const double *__restrict__ c,
                               double *__restrict__ w, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = w[i];
    for (int k = 0; k < K; ++k) a -= V[k * ld + i] * c[k];
    w[i] = a;
}

// y = alpha x + beta y
__global__ void axpby_kernel(double alpha, const double *__restrict__ x, double beta, double *__restrict__ y, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = alpha * x[i] + beta * y[i];
}

// right-hand side U_b + Omega_b x (x - c_b)
__global__ void rhs_kernel(const double *__restrict__ x, int64_t ntot, const int64_t *__restrict__ sph_of,
                           const double *__restrict__ centers, const double *__restrict__ motion,
                           double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntot) return;
    const int64_t m = sph_of[t];
    const double *U = motion + 6 * m, *O = U + 3;
    const double rx = x[3 * t] - centers[3 * m], ry = x[3 * t + 1] - centers[3 * m + 1],
                 rz = x[3 * t + 2] - centers[3 * m + 2];
    out[3 * t] = U[0] + O[1] * rz - O[2] * ry;
    out[3 * t + 1] = U[1] + O[2] * rx - O[0] * rz;
    out[3 * t + 2] = U[2] + O[0] * ry - O[1] * rx;
}

unsigned nblocks(size_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- host: interpolation stencils

struct Key {
    int i, s;
    int64_t j, k;
    bool operator==(const Key &o) const { return i == o.i && s == o.s && j == o.j && k == o.k; }
};
struct KeyHash {
    size_t operator()(const Key &a) const
    {
        return std::hash<int64_t>()(((a.j * 1000003LL + a.k) * 7 + a.i) * 3 + a.s + 1);
    }
};

double lagrange(double s, int a, int wdt)
{
    double L = 1.0;
    for (int b = 0; b < wdt; ++b)
        if (b != a) L *= (s - b) / (double)(a - b);
    return L;
}

using KeyMap = std::unordered_map<Key, int, KeyHash>;

// Family/grid keys of one sphere's quadrature points (local index within the sphere).
KeyMap sphere_keys(const double *hx, const double *hn, int64_t nm, const double *c, double h)
{
#pragma clang fp contract(off)
    const double cth = std::cos(70.0 * kPi / 180.0);
    KeyMap keys;
    for (int64_t p = 0; p < nm; ++p) {
        const double *xp = hx + 3 * p, *np_ = hn + 3 * p;
        for (int i = 0; i < 3; ++i) {
            if (std::fabs(np_[i]) < cth) continue;
            const int j = (i + 1) % 3 < (i + 2) % 3 ? (i + 1) % 3 : (i + 2) % 3;
            const int k = 3 - i - j;
            const double aj = (xp[j] - c[j]) / h, ak = (xp[k] - c[k]) / h;
            if (std::fabs(aj - std::round(aj)) < 1e-9 && std::fabs(ak - std::round(ak)) < 1e-9)
                keys[Key{i, xp[i] - c[i] > 0 ? 1 : -1, (int64_t)std::llround(aj), (int64_t)std::llround(ak)}] = (int)p;
        }
    }
    return keys;
}

// Closest-point data and interpolation stencils of sphere (c, a) for targets hy[0..nt); targets in
// [own0, own1) are the sphere's own points (normals hn_own, indexed from own0).  Returns false if a
// stencil cannot be formed.
bool sphere_targets(const KeyMap &keys, const double *c, double a, double h, const double *hy, int64_t nt,
                    int64_t own0, int64_t own1, const double *hn_own, std::vector<double> &x0,
                    std::vector<double> &n0, std::vector<double> &b, std::vector<int> &idx, std::vector<double> &wts)
{
#pragma clang fp contract(off)
    x0.assign(3 * nt, 0.0);
    n0.assign(3 * nt, 0.0);
    b.assign(nt, 0.0);
    idx.assign(kStencil * nt, 0);
    wts.assign(kStencil * nt, 0.0);
    for (int64_t t = 0; t < nt; ++t) {
        if (t >= own0 && t < own1) {
            for (int d = 0; d < 3; ++d) {
                x0[3 * t + d] = hy[3 * t + d];
                n0[3 * t + d] = hn_own[3 * (t - own0) + d];
            }
            continue;
        }
        double d[3], r2 = 0.0;
        for (int e = 0; e < 3; ++e) {
            d[e] = hy[3 * t + e] - c[e];
            r2 = r2 + d[e] * d[e];
        }
        const double r = std::sqrt(r2);
        double loc[3];
        for (int e = 0; e < 3; ++e) {
            n0[3 * t + e] = d[e] / r;
            x0[3 * t + e] = c[e] + a * n0[3 * t + e];
            loc[e] = x0[3 * t + e] - c[e];
        }
        b[t] = r - a;
        // widths 6 .. 2; for each, families in decreasing |n_i| (ties: lower index first)
        int fam[3] = {0, 1, 2};
        std::stable_sort(fam, fam + 3, [&](int u, int v2) { return std::fabs(loc[u]) > std::fabs(loc[v2]); });
        bool done = false;
        for (int wdt = kStencilWidth; wdt >= 2 && !done; --wdt) {
            for (int fi = 0; fi < 3 && !done; ++fi) {
                const int i = fam[fi];
                const int j = (i + 1) % 3 < (i + 2) % 3 ? (i + 1) % 3 : (i + 2) % 3;
                const int k = 3 - i - j;
                const int sg = loc[i] > 0 ? 1 : -1;
                const int64_t j0 = (int64_t)std::floor(loc[j] / h) - (wdt - 1) / 2;
                const int64_t k0 = (int64_t)std::floor(loc[k] / h) - (wdt - 1) / 2;
                int ids[kStencil];
                bool ok = true;
                for (int aa = 0; aa < wdt && ok; ++aa)
                    for (int bb = 0; bb < wdt && ok; ++bb) {
                        auto it = keys.find(Key{i, sg, j0 + aa, k0 + bb});
                        if (it == keys.end())
                            ok = false;
                        else
                            ids[aa * wdt + bb] = it->second;
                    }
                if (!ok) continue;
                const double sj = loc[j] / h - (double)j0, sk = loc[k] / h - (double)k0;
                for (int aa = 0; aa < wdt; ++aa)
                    for (int bb = 0; bb < wdt; ++bb) {
                        idx[kStencil * t + aa * wdt + bb] = ids[aa * wdt + bb];
                        wts[kStencil * t + aa * wdt + bb] = lagrange(sj, aa, wdt) * lagrange(sk, bb, wdt);
                    }
                done = true;
            }
        }
        if (!done) return false;
    }
    return true;
}

}  // namespace

struct sr_rigid {
    int device = 0;
    sr_params prm{};
    bool have_params = false;
    int nsph = 0;
    int64_t ntot = 0;
    std::vector<int64_t> off;              // nsph + 1
    std::vector<double> centers, radii;    // host
    std::vector<KeyMap> keys;              // per sphere: family grid keys
    std::vector<double> hnrm;              // host copy of the normals
    std::vector<sr_ctx *> ctx;             // one evaluator per sphere
    std::vector<sr_ctx *> ctx64;           // FP64 evaluators for the refined solve (made on first use)
    Buf<double> x, nrm, w, dcenters;       // all points (ntot)
    Buf<int64_t> sph_of;
    std::vector<Buf<double>> x0, n0, b, q0, v;  // per sphere, over all targets
    std::vector<Buf<int>> sidx;
    std::vector<Buf<double>> swts;
    Buf<double> vall;                      // nsph * ntot * 3 (the v_m contiguous)
    Buf<double> part;                      // strengths partials
    Buf<double> FL;                        // completion strengths (F, L) per sphere
    // GMRES work
    Buf<double> V, wv, tmp, red, coef, r;
    Buf<double> rr, dd;                    // refined solve: outer residual and correction
    // operator a_id q + a_dl sum_m DL_m[q] (+ completion): -1/2, 1, on for rigid spheres
    double a_id = -0.5, a_dl = 1.0;
    bool completion = true;
    bool ready = false;
};

namespace {

sr_status rigid_matvec(sr_rigid *R, const std::vector<sr_ctx *> &ctx, const double *q, double *out, hipStream_t s)
{
    const int64_t N = R->ntot;
    RHIP(R->vall.alloc((size_t)R->nsph * N * 3));
    RHIP(R->part.alloc((size_t)R->nsph * kRedBlocks * 6));
    RHIP(R->FL.alloc((size_t)R->nsph * 6));
    for (int m = 0; m < R->nsph; ++m) {
        const int64_t o = R->off[m], nm = R->off[m + 1] - o;
        hipLaunchKernelGGL(gather_q0_kernel, dim3(nblocks(N)), dim3(256), 0, s, q, N, o, o + nm, o, R->sidx[m].p,
                           R->swts[m].p, R->q0[m].p);
        RHIP(hipGetLastError());
        RSR(sr_set_density(ctx[m], SR_DL, q + 3 * o, s));
        RSR(sr_eval(ctx[m], SR_DL, N, R->x.p, R->x0[m].p, R->n0[m].p, R->b[m].p, nullptr, R->q0[m].p, nullptr,
                    R->vall.p + (size_t)m * N * 3, nullptr, nullptr, s));
        if (R->completion) {
            hipLaunchKernelGGL(strengths_kernel, dim3(kRedBlocks), dim3(kRed), 0, s, q, R->x.p, R->w.p, o, nm,
                               R->centers[3 * m], R->centers[3 * m + 1], R->centers[3 * m + 2],
                               R->part.p + (size_t)m * kRedBlocks * 6);
            RHIP(hipGetLastError());
        }
    }
    if (R->completion) {
        hipLaunchKernelGGL(strengths_final_kernel, dim3(6 * R->nsph), dim3(kRed), 0, s, R->part.p, R->nsph, kRedBlocks,
                           R->FL.p);
        RHIP(hipGetLastError());
    }
    hipLaunchKernelGGL(assemble_kernel, dim3(nblocks(N)), dim3(256), 0, s, q, R->x.p, N, R->nsph, R->vall.p,
                       R->dcenters.p, R->FL.p, out, R->a_id, R->a_dl, R->completion ? 1 : 0);
    RHIP(hipGetLastError());
    return SR_OK;
}

// res[0..K-1] = V[0..K-1] . w (on the device, into R->coef); copies to host if hres
sr_status mdot(sr_rigid *R, const double *V, size_t ld, int K, const double *w, size_t n, double *hres, hipStream_t s)
{
    RHIP(R->red.alloc((size_t)kRedBlocks * K));
    hipLaunchKernelGGL(mdot_kernel, dim3(kRedBlocks), dim3(kRed), 0, s, V, ld, K, w, n, R->red.p);
    RHIP(hipGetLastError());
    hipLaunchKernelGGL(mdot_final_kernel, dim3(K), dim3(kRed), 0, s, R->red.p, kRedBlocks, K, R->coef.p);
    RHIP(hipGetLastError());
    if (hres) {
        RHIP(hipMemcpyAsync(hres, R->coef.p, K * sizeof(double), hipMemcpyDeviceToHost, s));
        RHIP(hipStreamSynchronize(s));
    }
    return SR_OK;
}

}  // namespace

extern "C" {

sr_status sr_rigid_create(sr_rigid **out, int device)
{
    g_rerr.clear();
    if (!out) return rfail(SR_EINVAL, "sr_rigid_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || device < 0 || device >= count)
        return rfail(SR_ENODEV, "sr_rigid_create: no such HIP device");
    sr_rigid *R = new (std::nothrow) sr_rigid();
    if (!R) return rfail(SR_ENOMEM, "sr_rigid_create: out of host memory");
    R->device = device;
    sr_default_params(&R->prm);
    *out = R;
    return SR_OK;
}

sr_status sr_rigid_destroy(sr_rigid *R)
{
    g_rerr.clear();
    if (!R) return SR_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(R->device);
    (void)hipDeviceSynchronize();
    for (sr_ctx *c : R->ctx) sr_destroy(c);
    for (sr_ctx *c : R->ctx64) sr_destroy(c);
    delete R;
    if (prev >= 0) (void)hipSetDevice(prev);
    return SR_OK;
}

sr_status sr_rigid_set_params(sr_rigid *R, const sr_params *p)
{
    g_rerr.clear();
    if (!R || !p) return rfail(SR_EINVAL, "sr_rigid_set_params: NULL argument");
    for (sr_ctx *c : R->ctx) RSR(sr_set_params(c, p));
    for (sr_ctx *c : R->ctx64) sr_destroy(c);
    R->ctx64.clear();
    R->prm = *p;
    R->have_params = true;
    return SR_OK;
}

sr_status sr_rigid_set_spheres(sr_rigid *R, int nsph, const double *centers, const double *radii,
                               const int64_t *counts, const double *x, const double *nrm, const double *w,
                               void *stream)
{
    g_rerr.clear();
    if (!R || !centers || !radii || !counts || !x || !nrm || !w) return rfail(SR_EINVAL, "sr_rigid_set_spheres: NULL argument");
    if (nsph < 1 || nsph > 64) return rfail(SR_EINVAL, "sr_rigid_set_spheres: nsph must be in 1..64");
    if (!R->have_params) return rfail(SR_ESTATE, "sr_rigid_set_spheres: set the parameters first");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(R->device) != hipSuccess) return rfail(SR_ENODEV, "sr_rigid_set_spheres: cannot select device");
    struct Restore {
        int d;
        ~Restore()
        {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev};
    hipStream_t s = (hipStream_t)stream;
    R->ready = false;
    for (sr_ctx *c : R->ctx) sr_destroy(c);
    R->ctx.clear();
    for (sr_ctx *c : R->ctx64) sr_destroy(c);
    R->ctx64.clear();
    R->nsph = nsph;
    R->off.assign(nsph + 1, 0);
    for (int m = 0; m < nsph; ++m) {
        if (counts[m] < 1 || !(radii[m] > 0.0)) return rfail(SR_EINVAL, "sr_rigid_set_spheres: bad count or radius");
        R->off[m + 1] = R->off[m] + counts[m];
    }
    const int64_t N = R->off[nsph];
    R->ntot = N;
    R->centers.assign(centers, centers + 3 * nsph);
    R->radii.assign(radii, radii + nsph);
    std::vector<double> hx(3 * N), hn(3 * N), hw(N);
    RHIP(hipMemcpyAsync(hx.data(), x, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipMemcpyAsync(hn.data(), nrm, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipMemcpyAsync(hw.data(), w, N * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipStreamSynchronize(s));
    RHIP(R->x.alloc(3 * N));
    RHIP(R->nrm.alloc(3 * N));
    RHIP(R->w.alloc(N));
    RHIP(R->dcenters.alloc(3 * nsph));
    RHIP(R->sph_of.alloc(N));
    RHIP(hipMemcpyAsync(R->x.p, x, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    RHIP(hipMemcpyAsync(R->nrm.p, nrm, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    RHIP(hipMemcpyAsync(R->w.p, w, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<int64_t> hsph(N);
    for (int m = 0; m < nsph; ++m)
        for (int64_t t = R->off[m]; t < R->off[m + 1]; ++t) hsph[t] = m;
    RHIP(hipMemcpyAsync(R->sph_of.p, hsph.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, s));
    RHIP(hipMemcpyAsync(R->dcenters.p, R->centers.data(), 3 * nsph * sizeof(double), hipMemcpyHostToDevice, s));

    const double h = R->prm.h;
    R->x0.clear();
    R->n0.clear();
    R->b.clear();
    R->q0.clear();
    R->sidx.clear();
    R->swts.clear();
    R->keys.clear();
    R->x0.resize(nsph);
    R->n0.resize(nsph);
    R->b.resize(nsph);
    R->q0.resize(nsph);
    R->sidx.resize(nsph);
    R->swts.resize(nsph);
    R->hnrm = hn;
    for (int m = 0; m < nsph; ++m) {
        const double *c = &R->centers[3 * m];
        const double a = R->radii[m];
        const int64_t o = R->off[m], nm = counts[m];
        R->keys.push_back(sphere_keys(&hx[3 * o], &hn[3 * o], nm, c, h));
        std::vector<double> hx0, hn0, hb, hwts;
        std::vector<int> hidx;
        if (!sphere_targets(R->keys[m], c, a, h, hx.data(), N, o, o + nm, &hn[3 * o], hx0, hn0, hb, hidx, hwts))
            return rfail(SR_EINVAL, "sr_rigid_set_spheres: no interpolation stencil (are the points the grid-line "
                                    "quadrature of spheres with the parameters' h?)");
        RHIP(R->x0[m].alloc(3 * N));
        RHIP(R->n0[m].alloc(3 * N));
        RHIP(R->b[m].alloc(N));
        RHIP(R->q0[m].alloc(3 * N));
        RHIP(R->sidx[m].alloc(kStencil * N));
        RHIP(R->swts[m].alloc(kStencil * N));
        RHIP(hipMemcpyAsync(R->x0[m].p, hx0.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(R->n0[m].p, hn0.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(R->b[m].p, hb.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(R->sidx[m].p, hidx.data(), kStencil * N * sizeof(int), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(R->swts[m].p, hwts.data(), kStencil * N * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipStreamSynchronize(s));
        sr_ctx *c2 = nullptr;
        RSR(sr_create(&c2, R->device));
        R->ctx.push_back(c2);
        RSR(sr_set_params(c2, &R->prm));
        RSR(sr_set_surface(c2, nm, x + 3 * o, nrm + 3 * o, w + o, stream));
    }
    R->ready = true;
    return SR_OK;
}

sr_status sr_rigid_rhs(sr_rigid *R, const double *motion, double *rhs, void *stream)
{
    g_rerr.clear();
    if (!R || !motion || !rhs) return rfail(SR_EINVAL, "sr_rigid_rhs: NULL argument");
    if (!R->ready) return rfail(SR_ESTATE, "sr_rigid_rhs: set the spheres first");
    hipStream_t s = (hipStream_t)stream;
    Buf<double> dm;
    RHIP(dm.alloc(6 * R->nsph));
    RHIP(hipMemcpyAsync(dm.p, motion, 6 * R->nsph * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(rhs_kernel, dim3(nblocks(R->ntot)), dim3(256), 0, s, R->x.p, R->ntot, R->sph_of.p,
                       R->dcenters.p, dm.p, rhs);
    RHIP(hipGetLastError());
    RHIP(hipStreamSynchronize(s));  // dm dies at return
    return SR_OK;
}

sr_status sr_rigid_matvec(sr_rigid *R, const double *q, double *out, void *stream)
{
    g_rerr.clear();
    if (!R || !q || !out) return rfail(SR_EINVAL, "sr_rigid_matvec: NULL argument");
    if (!R->ready) return rfail(SR_ESTATE, "sr_rigid_matvec: set the spheres first");
    return rigid_matvec(R, R->ctx, q, out, (hipStream_t)stream);
}

sr_status sr_rigid_set_operator(sr_rigid *R, double a_id, double a_dl, int completion)
{
    g_rerr.clear();
    if (!R) return rfail(SR_EINVAL, "sr_rigid_set_operator: NULL argument");
    if (!std::isfinite(a_id) || !std::isfinite(a_dl)) return rfail(SR_EINVAL, "sr_rigid_set_operator: not finite");
    R->a_id = a_id;
    R->a_dl = a_dl;
    R->completion = completion != 0;
    return SR_OK;
}

sr_status sr_rigid_single_layer(sr_rigid *R, const double *f, double *out, void *stream)
{
    g_rerr.clear();
    if (!R || !f || !out) return rfail(SR_EINVAL, "sr_rigid_single_layer: NULL argument");
    if (!R->ready) return rfail(SR_ESTATE, "sr_rigid_single_layer: set the spheres first");
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = R->ntot;
    RHIP(R->vall.alloc((size_t)R->nsph * N * 3));
    for (int m = 0; m < R->nsph; ++m) {
        const int64_t o = R->off[m], nm = R->off[m + 1] - o;
        // f(x0): the sphere's own values at its points, the stencil interpolation elsewhere
        hipLaunchKernelGGL(gather_q0_kernel, dim3(nblocks(N)), dim3(256), 0, s, f, N, o, o + nm, o, R->sidx[m].p,
                           R->swts[m].p, R->q0[m].p);
        RHIP(hipGetLastError());
        RSR(sr_set_density(R->ctx[m], SR_SL, f + 3 * o, s));
        RSR(sr_eval(R->ctx[m], SR_SL, N, R->x.p, R->x0[m].p, R->n0[m].p, R->b[m].p, R->q0[m].p, nullptr,
                    R->vall.p + (size_t)m * N * 3, nullptr, nullptr, nullptr, s));
    }
    hipLaunchKernelGGL(assemble_kernel, dim3(nblocks(N)), dim3(256), 0, s, f, R->x.p, N, R->nsph, R->vall.p,
                       R->dcenters.p, R->FL.p, out, 0.0, 1.0, 0);
    RHIP(hipGetLastError());
    return SR_OK;
}

sr_status sr_rigid_velocity(sr_rigid *R, const double *q, int64_t m, const double *y, double *u, void *stream)
{
    g_rerr.clear();
    if (!R || !q || !y || !u) return rfail(SR_EINVAL, "sr_rigid_velocity: NULL argument");
    if (!R->ready) return rfail(SR_ESTATE, "sr_rigid_velocity: set the spheres first");
    if (m < 1) return m == 0 ? SR_OK : rfail(SR_EINVAL, "sr_rigid_velocity: m < 0");
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> hy(3 * m);
    RHIP(hipMemcpyAsync(hy.data(), y, 3 * m * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipStreamSynchronize(s));
    for (int64_t t = 0; t < m; ++t)
        for (int k = 0; k < R->nsph; ++k) {
            double r2 = 0.0;
            for (int e = 0; e < 3; ++e) {
                const double d = hy[3 * t + e] - R->centers[3 * k + e];
                r2 += d * d;
            }
            if (!(r2 > R->radii[k] * R->radii[k]))
                return rfail(SR_EINVAL, "sr_rigid_velocity: a point is not outside every sphere");
        }
    Buf<double> vv, part, dx0, dn0, db, dq0, dw;
    Buf<int> di;
    RHIP(vv.alloc((size_t)R->nsph * m * 3));
    RHIP(part.alloc((size_t)R->nsph * kRedBlocks * 6));
    RHIP(dx0.alloc(3 * m));
    RHIP(dn0.alloc(3 * m));
    RHIP(db.alloc(m));
    RHIP(dq0.alloc(3 * m));
    RHIP(dw.alloc(kStencil * m));
    RHIP(di.alloc(kStencil * m));
    for (int k = 0; k < R->nsph; ++k) {
        const int64_t o = R->off[k], nm = R->off[k + 1] - o;
        std::vector<double> hx0, hn0, hb, hwts;
        std::vector<int> hidx;
        if (!sphere_targets(R->keys[k], &R->centers[3 * k], R->radii[k], R->prm.h, hy.data(), m, 0, 0, nullptr, hx0,
                            hn0, hb, hidx, hwts))
            return rfail(SR_EINVAL, "sr_rigid_velocity: no interpolation stencil");
        RHIP(hipMemcpyAsync(dx0.p, hx0.data(), 3 * m * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(dn0.p, hn0.data(), 3 * m * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(db.p, hb.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(di.p, hidx.data(), kStencil * m * sizeof(int), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(dw.p, hwts.data(), kStencil * m * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_q0_kernel, dim3(nblocks(m)), dim3(256), 0, s, q, m, (int64_t)0, (int64_t)0, o, di.p,
                           dw.p, dq0.p);
        RHIP(hipGetLastError());
        RSR(sr_set_density(R->ctx[k], SR_DL, q + 3 * o, s));
        RSR(sr_eval(R->ctx[k], SR_DL, m, y, dx0.p, dn0.p, db.p, nullptr, dq0.p, nullptr, vv.p + (size_t)k * m * 3,
                    nullptr, nullptr, s));
        hipLaunchKernelGGL(strengths_kernel, dim3(kRedBlocks), dim3(kRed), 0, s, q, R->x.p, R->w.p, o, nm,
                           R->centers[3 * k], R->centers[3 * k + 1], R->centers[3 * k + 2],
                           part.p + (size_t)k * kRedBlocks * 6);
        RHIP(hipGetLastError());
        RHIP(hipStreamSynchronize(s));  // host staging vectors die at the end of the iteration
    }
    Buf<double> FL;
    RHIP(FL.alloc((size_t)R->nsph * 6));
    hipLaunchKernelGGL(strengths_final_kernel, dim3(6 * R->nsph), dim3(kRed), 0, s, part.p, R->nsph, kRedBlocks,
                       FL.p);
    RHIP(hipGetLastError());
    hipLaunchKernelGGL(assemble_kernel, dim3(nblocks(m)), dim3(256), 0, s, q, y, m, R->nsph, vv.p, R->dcenters.p,
                       FL.p, u, 0.0, 1.0, 1);
    RHIP(hipGetLastError());
    RHIP(hipStreamSynchronize(s));  // temporaries die at return
    return SR_OK;
}

}  // extern "C"

namespace {

// Restarted GMRES on A x = rhs with the operator of the evaluators `ctx` (classical Gram-Schmidt
// applied twice; Givens rotations on the host).  *iters = Arnoldi products, *relres = recomputed true
// relative residual, *converged = whether the estimate reached tol.
sr_status gmres_solve(sr_rigid *R, const std::vector<sr_ctx *> &ctx, const double *rhs, double *x, bool x_is_guess,
                      double tol, int maxit, int restart, int *iters, double *relres, bool *converged_out,
                      hipStream_t s)
{
    const size_t n = (size_t)R->ntot * 3;
    const int mr = restart;
    RHIP(R->V.alloc((size_t)(mr + 1) * n));
    RHIP(R->wv.alloc(n));
    RHIP(R->r.alloc(n));
    RHIP(R->coef.alloc(mr + 2));
    if (!x_is_guess) {
        hipLaunchKernelGGL(zero_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, n);
        RHIP(hipGetLastError());
    }
    double bn2 = 0.0;
    RSR(mdot(R, rhs, n, 1, rhs, n, &bn2, s));
    const double bn = std::sqrt(bn2);
    if (bn == 0.0) {
        hipLaunchKernelGGL(zero_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, n);
        RHIP(hipGetLastError());
        *iters = 0;
        *relres = 0.0;
        *converged_out = true;
        return SR_OK;
    }
    int total = 0;
    double est = 1.0;
    std::vector<double> H((size_t)(mr + 1) * mr), cs(mr), sn(mr), g(mr + 1), hcol(mr + 1), h2(mr + 1), yv(mr);
    bool converged = false;
    while (total < maxit && !converged) {
        // r = b - A x
        RSR(rigid_matvec(R, ctx, x, R->r.p, s));
        hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, 1.0, rhs, -1.0, R->r.p, n);
        RHIP(hipGetLastError());
        double beta2 = 0.0;
        RSR(mdot(R, R->r.p, n, 1, R->r.p, n, &beta2, s));
        const double beta = std::sqrt(beta2);
        est = beta / bn;
        if (est <= tol) {
            converged = true;
            break;
        }
        hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, 1.0 / beta, R->r.p, 0.0, R->V.p, n);
        RHIP(hipGetLastError());
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (; k < mr && total < maxit; ++k) {
            double *vk = R->V.p + (size_t)k * n, *vk1 = R->V.p + (size_t)(k + 1) * n;
            RSR(rigid_matvec(R, ctx, vk, R->wv.p, s));
            ++total;
            // classical Gram-Schmidt, twice
            std::fill(hcol.begin(), hcol.end(), 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                RSR(mdot(R, R->V.p, n, k + 1, R->wv.p, n, h2.data(), s));
                hipLaunchKernelGGL(mupdate_kernel, dim3(nblocks(n)), dim3(256), 0, s, R->V.p, n, k + 1, R->coef.p,
                                   R->wv.p, n);
                RHIP(hipGetLastError());
                for (int i = 0; i <= k; ++i) hcol[i] += h2[i];
            }
            double hn2 = 0.0;
            RSR(mdot(R, R->wv.p, n, 1, R->wv.p, n, &hn2, s));
            hcol[k + 1] = std::sqrt(hn2);
            if (hcol[k + 1] > 0.0) {
                hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, 1.0 / hcol[k + 1], R->wv.p, 0.0,
                                   vk1, n);
                RHIP(hipGetLastError());
            }
            for (int i = 0; i < k; ++i) {
                const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
                hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
                hcol[i] = t;
            }
            const double d = std::hypot(hcol[k], hcol[k + 1]);
            cs[k] = hcol[k] / d;
            sn[k] = hcol[k + 1] / d;
            hcol[k] = d;
            hcol[k + 1] = 0.0;
            for (int i = 0; i <= k; ++i) H[(size_t)i * mr + k] = hcol[i];
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            est = std::fabs(g[k + 1]) / bn;
            if (est <= tol) {
                ++k;
                converged = true;
                break;
            }
        }
        // y = H^{-1} g, x += V y
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int j = i + 1; j < k; ++j) t -= H[(size_t)i * mr + j] * yv[j];
            yv[i] = t / H[(size_t)i * mr + i];
        }
        for (int i = 0; i < k; ++i) {
            hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, yv[i], R->V.p + (size_t)i * n, 1.0,
                               x, n);
            RHIP(hipGetLastError());
        }
    }
    // true relative residual
    RSR(rigid_matvec(R, ctx, x, R->r.p, s));
    hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, 1.0, rhs, -1.0, R->r.p, n);
    RHIP(hipGetLastError());
    double rr2 = 0.0;
    RSR(mdot(R, R->r.p, n, 1, R->r.p, n, &rr2, s));
    *iters = total;
    *relres = std::sqrt(rr2) / bn;
    *converged_out = converged || *relres <= tol;
    return SR_OK;
}

sr_status check_solve_args(sr_rigid *R, const double *rhs, const double *x, double tol, int maxit, int restart,
                           const char *who)
{
    if (!R || !rhs || !x) return rfail(SR_EINVAL, (std::string(who) + ": NULL argument").c_str());
    if (!R->ready) return rfail(SR_ESTATE, (std::string(who) + ": set the spheres first").c_str());
    if (!(tol > 0.0) || maxit < 1 || restart < 1 || restart > 512)
        return rfail(SR_EINVAL, (std::string(who) + ": need tol > 0, maxit >= 1, 1 <= restart <= 512").c_str());
    return SR_OK;
}

}  // namespace

extern "C" {

sr_status sr_rigid_solve(sr_rigid *R, const double *rhs, double *x, int x_is_guess, double tol, int maxit,
                         int restart, int *iters, double *relres, void *stream)
{
    g_rerr.clear();
    RSR(check_solve_args(R, rhs, x, tol, maxit, restart, "sr_rigid_solve"));
    int it = 0;
    double rel = 0.0;
    bool conv = false;
    RSR(gmres_solve(R, R->ctx, rhs, x, x_is_guess != 0, tol, maxit, restart, &it, &rel, &conv, (hipStream_t)stream));
    if (iters) *iters = it;
    if (relres) *relres = rel;
    if (!conv) return rfail(SR_ENOCONV, "sr_rigid_solve: no convergence");
    return SR_OK;
}

sr_status sr_rigid_solve_refined(sr_rigid *R, const double *rhs, double *x, int x_is_guess, double tol,
                                 double inner_tol, int maxit, int restart, int *iters, int *outer, double *relres,
                                 void *stream)
{
    g_rerr.clear();
    RSR(check_solve_args(R, rhs, x, tol, maxit, restart, "sr_rigid_solve_refined"));
    if (!(inner_tol > 0.0 && inner_tol < 1.0)) return rfail(SR_EINVAL, "sr_rigid_solve_refined: need 0 < inner_tol < 1");
    hipStream_t s = (hipStream_t)stream;
    if (R->ctx64.empty()) {
        sr_params p64 = R->prm;
        p64.precision = SR_FP64;
        p64.far_method = SR_DIRECT;  // the residual is measured with the exact operator, whatever the inner one
        for (int m = 0; m < R->nsph; ++m) {
            sr_ctx *c = nullptr;
            RSR(sr_create(&c, R->device));
            R->ctx64.push_back(c);
            RSR(sr_set_params(c, &p64));
            const int64_t o = R->off[m];
            RSR(sr_set_surface(c, R->off[m + 1] - o, R->x.p + 3 * o, R->nrm.p + 3 * o, R->w.p + o, stream));
        }
    }
    const size_t n = (size_t)R->ntot * 3;
    RHIP(R->rr.alloc(n));
    RHIP(R->dd.alloc(n));
    RHIP(R->coef.alloc(restart + 2));
    if (!x_is_guess) {
        hipLaunchKernelGGL(zero_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, n);
        RHIP(hipGetLastError());
    }
    double bn2 = 0.0;
    RSR(mdot(R, rhs, n, 1, rhs, n, &bn2, s));
    const double bn = std::sqrt(bn2);
    int total = 0, nout = 0;
    double rel = 0.0;
    bool conv = bn == 0.0;
    if (conv) {
        hipLaunchKernelGGL(zero_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, n);
        RHIP(hipGetLastError());
    }
    bool first = true;
    while (!conv) {
        // outer residual with the FP64 operator
        RSR(rigid_matvec(R, R->ctx64, x, R->rr.p, s));
        hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, 1.0, rhs, -1.0, R->rr.p, n);
        RHIP(hipGetLastError());
        double r2 = 0.0;
        RSR(mdot(R, R->rr.p, n, 1, R->rr.p, n, &r2, s));
        rel = std::sqrt(r2) / bn;
        if (first && x_is_guess && !(rel < 1.0)) {
            // a guess no better than zero (or not finite): start from zero instead
            hipLaunchKernelGGL(zero_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, n);
            RHIP(hipGetLastError());
            first = false;
            continue;
        }
        first = false;
        if (rel <= tol) {
            conv = true;
            break;
        }
        if (total >= maxit) break;
        // correction from the working-precision operator: reduce the residual by inner_tol, or only
        // as far as the outer tolerance needs (with a factor 2 of margin), whichever is less work
        const double eta = std::min(0.5, std::max(inner_tol, 0.5 * tol / rel));
        int it = 0;
        double irel = 0.0;
        bool iconv = false;
        RSR(gmres_solve(R, R->ctx, R->rr.p, R->dd.p, false, eta, maxit - total, restart, &it, &irel, &iconv, s));
        total += it;
        ++nout;
        hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, s, 1.0, R->dd.p, 1.0, x, n);
        RHIP(hipGetLastError());
    }
    RHIP(hipStreamSynchronize(s));
    if (iters) *iters = total;
    if (outer) *outer = nout;
    if (relres) *relres = rel;
    if (!conv) return rfail(SR_ENOCONV, "sr_rigid_solve_refined: no convergence");
    return SR_OK;
}


// ---- coarse-to-fine interpolation of densities on spheres ----

struct sr_prolong {
    int device = 0;
    int nsph = 0;
    std::vector<int64_t> offc, offf;
    std::vector<Buf<int>> idx;
    std::vector<Buf<double>> wts;
};

sr_status sr_prolong_create(sr_prolong **out, int device, int nsph, const double *centers, const double *radii,
                            double hc, const int64_t *counts_c, const double *xc, const double *nc,
                            const int64_t *counts_f, const double *xf, void *stream)
{
    g_rerr.clear();
    if (!out || !centers || !radii || !counts_c || !xc || !nc || !counts_f || !xf)
        return rfail(SR_EINVAL, "sr_prolong_create: NULL argument");
    *out = nullptr;
    if (nsph < 1 || nsph > 64) return rfail(SR_EINVAL, "sr_prolong_create: nsph must be in 1..64");
    if (!(hc > 0.0)) return rfail(SR_EINVAL, "sr_prolong_create: hc must be > 0");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return rfail(SR_ENODEV, "sr_prolong_create: cannot select device");
    struct Restore {
        int d;
        ~Restore()
        {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev};
    hipStream_t s = (hipStream_t)stream;
    sr_prolong *P = new (std::nothrow) sr_prolong();
    if (!P) return rfail(SR_ENOMEM, "sr_prolong_create: out of host memory");
    std::unique_ptr<sr_prolong> guard(P);
    P->device = device;
    P->nsph = nsph;
    P->offc.assign(nsph + 1, 0);
    P->offf.assign(nsph + 1, 0);
    for (int m = 0; m < nsph; ++m) {
        if (counts_c[m] < 1 || counts_f[m] < 1 || !(radii[m] > 0.0))
            return rfail(SR_EINVAL, "sr_prolong_create: bad count or radius");
        P->offc[m + 1] = P->offc[m] + counts_c[m];
        P->offf[m + 1] = P->offf[m] + counts_f[m];
    }
    const int64_t NC = P->offc[nsph], NF = P->offf[nsph];
    std::vector<double> hxc(3 * NC), hnc(3 * NC), hxf(3 * NF);
    RHIP(hipMemcpyAsync(hxc.data(), xc, 3 * NC * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipMemcpyAsync(hnc.data(), nc, 3 * NC * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipMemcpyAsync(hxf.data(), xf, 3 * NF * sizeof(double), hipMemcpyDeviceToHost, s));
    RHIP(hipStreamSynchronize(s));
    P->idx.resize(nsph);
    P->wts.resize(nsph);
    for (int m = 0; m < nsph; ++m) {
        const double *c = centers + 3 * m;
        const int64_t oc = P->offc[m], nf = counts_f[m];
        KeyMap keys = sphere_keys(&hxc[3 * oc], &hnc[3 * oc], counts_c[m], c, hc);
        std::vector<double> x0, n0, b, w;
        std::vector<int> id;
        if (!sphere_targets(keys, c, radii[m], hc, &hxf[3 * P->offf[m]], nf, 0, 0, nullptr, x0, n0, b, id, w))
            return rfail(SR_EINVAL, "sr_prolong_create: no interpolation stencil (is the coarse set the grid-line "
                                    "quadrature of the spheres with spacing hc?)");
        RHIP(P->idx[m].alloc(kStencil * nf));
        RHIP(P->wts[m].alloc(kStencil * nf));
        RHIP(hipMemcpyAsync(P->idx[m].p, id.data(), kStencil * nf * sizeof(int), hipMemcpyHostToDevice, s));
        RHIP(hipMemcpyAsync(P->wts[m].p, w.data(), kStencil * nf * sizeof(double), hipMemcpyHostToDevice, s));
        RHIP(hipStreamSynchronize(s));  // host staging vectors die at the end of the iteration
    }
    *out = guard.release();
    return SR_OK;
}

sr_status sr_prolong_apply(sr_prolong *P, const double *qc, double *qf, void *stream)
{
    g_rerr.clear();
    if (!P || !qc || !qf) return rfail(SR_EINVAL, "sr_prolong_apply: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    for (int m = 0; m < P->nsph; ++m) {
        const int64_t nf = P->offf[m + 1] - P->offf[m];
        hipLaunchKernelGGL(gather_q0_kernel, dim3(nblocks(nf)), dim3(256), 0, s, qc, nf, (int64_t)0, (int64_t)0,
                           P->offc[m], P->idx[m].p, P->wts[m].p, qf + 3 * P->offf[m]);
        RHIP(hipGetLastError());
    }
    return SR_OK;
}

sr_status sr_prolong_destroy(sr_prolong *P)
{
    g_rerr.clear();
    if (!P) return SR_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    delete P;
    if (prev >= 0) (void)hipSetDevice(prev);
    return SR_OK;
}

const char *sr_rigid_last_error(void) { return g_rerr.c_str(); }

}  // extern "C"

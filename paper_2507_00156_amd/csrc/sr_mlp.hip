// Warm-start network for the two-sphere solve: training and inference on BF16 matrix cores.
//
// The network (exactly linear in the 12 rigid-motion parameters m, because the density solves a
// linear equation whose right-hand side is linear in m):
//   gt = (ln g - g_mid) / g_half (near contact the flow varies like log(gap))
//   h1 = tanh(W1 gt + b1), h2 = tanh(W2 h1 + b2), h3 = tanh(W3 h2 + b3)      (width W)
//   a4 = W4 h3 + b4 (12 W), C[w][k] = a4[12 w + k], z = C m                  (width W)
//   o  = Wh z (P outputs, standardized), density q = s o with a per-output scale s
// loss = mean over the batch and the P outputs of (o - y / s)^2; Adam (Kingma & Ba 2015).
//
// Matrix products: one kernel, C = A B^T with both operands stored K-contiguous as BF16, on
// mfma_f32_16x16x32_bf16 with FP32 accumulation.  Each FP32 operand is carried as hi + lo + lo2, three
// BF16 numbers (hi = bf16(x), lo = bf16(x - hi), lo2 = bf16(x - hi - lo): together the whole FP32
// significand); with passes = 3 the product sums hi*hi, hi*lo and lo*hi (all on BF16 MFMA), which keeps
// about 16 significant bits instead of 8; passes = 6 adds lo*lo, hi*lo2 and lo2*hi (about 24 bits, the
// precision of the FP32 operands, at twice the matrix-core work); passes = 1 uses hi*hi
// only.  Operands that a product needs transposed are kept as transposed BF16 copies, written by a
// tiled LDS transpose as they are produced.  Leading dimensions and padded extents are multiples
// of 32, padding is zero, so every fragment load is an aligned 16-byte load.
//
// Work decomposition of the product: a workgroup of 4 wavefronts owns a 64 x 64 tile of C, each
// wavefront a 32 x 32 block (2 x 2 MFMA tiles of 16 x 16); K advances 32 per step.  Long
// contractions (over the P outputs) are split over blockIdx.z into partial tiles that an epilogue
// sums in a fixed order (no atomics: results are reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "stokesreg.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kNMot = 12;     // rigid-motion parameters (translation + rotation of two spheres)
constexpr int kPad = 32;      // padding unit of extents and leading dimensions (MFMA K step)
constexpr int kMaxSplit = 256;

thread_local std::string g_merr;

sr_status mfail(sr_status st, const std::string &msg)
{
    g_merr = msg;
    return st;
}

#define MHIP(call)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return mfail(SR_EHIP, std::string("HIP: ") + hipGetErrorString(e_));  \
    } while (0)
#define MSR(call)                                                                                     \
    do {                                                                                              \
        sr_status s_ = (call);                                                                        \
        if (s_ != SR_OK) return s_;                                                                   \
    } while (0)

inline int64_t pad_up(int64_t x) { return (x + kPad - 1) / kPad * kPad; }
inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------------------------
// BF16 conversion (round to nearest even)

__device__ __forceinline__ u16 bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_f(u16 b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------------------------
// C (M x N, ldc) = A (M x K) B^T (N x K), K-contiguous BF16 hi/lo operands, FP32 result.
// blockIdx.z = split index: contracts K range [z kchunk, min(Kpad, (z+1) kchunk)) into
// C + z * split_stride.  Rows beyond M / N are clamped for loads and not stored.

template <int PASSES>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const u16 *__restrict__ Ahi, const u16 *__restrict__ Alo,
                                                      const u16 *__restrict__ Alo2, int64_t lda,
                                                      const u16 *__restrict__ Bhi, const u16 *__restrict__ Blo,
                                                      const u16 *__restrict__ Blo2, int64_t ldb, int M, int N,
                                                      int Kpad, int kchunk, float *__restrict__ C, int64_t ldc,
                                                      int64_t split_stride)
{
    const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const int m0 = (int)blockIdx.x * 64 + (wave >> 1) * 32;
    const int n0 = (int)blockIdx.y * 64 + (wave & 1) * 32;
    const int kb = (int)blockIdx.z * kchunk;
    const int ke = min(Kpad, kb + kchunk);
    const int r = lane % 16, kq = 8 * (lane / 16);
    int64_t oa[2], ob[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        oa[i] = (int64_t)min(m0 + 16 * i + r, M - 1) * lda + kq;
        ob[i] = (int64_t)min(n0 + 16 * i + r, N - 1) * ldb + kq;
    }
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the operands of step k + kPad are loaded while step k's products run (register double buffer)
    bf16x8 ah[2], bh[2], al[2], bl[2], a2[2], b2[2];
    auto load = [&](int k) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = *(const bf16x8 *)(Ahi + oa[i] + k);
            bh[i] = *(const bf16x8 *)(Bhi + ob[i] + k);
            if (PASSES >= 3) {
                al[i] = *(const bf16x8 *)(Alo + oa[i] + k);
                bl[i] = *(const bf16x8 *)(Blo + ob[i] + k);
            }
            if (PASSES == 6) {
                a2[i] = *(const bf16x8 *)(Alo2 + oa[i] + k);
                b2[i] = *(const bf16x8 *)(Blo2 + ob[i] + k);
            }
        }
    };
    if (kb < ke) load(kb);
    for (int k = kb; k < ke; k += kPad) {
        const bf16x8 ch[2] = {ah[0], ah[1]}, dh[2] = {bh[0], bh[1]};
        bf16x8 cl[2], dl[2], c2[2], d2[2];
        if (PASSES >= 3) {
            cl[0] = al[0];
            cl[1] = al[1];
            dl[0] = bl[0];
            dl[1] = bl[1];
        }
        if (PASSES == 6) {
            c2[0] = a2[0];
            c2[1] = a2[1];
            d2[0] = b2[0];
            d2[1] = b2[1];
        }
        if (k + kPad < ke) load(k + kPad);
        // smallest terms first
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (PASSES == 6) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c2[i], dh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[i], d2[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl[i], dl[j], acc[i][j], 0, 0, 0);
                }
                if (PASSES >= 3) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl[i], dh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[i], dl[j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[i], dh[j], acc[i][j], 0, 0, 0);
            }
    }
    float *Cz = C + (int64_t)blockIdx.z * split_stride;
    // result layout: lane l, element v holds row 4 (l / 16) + v, column l % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + 16 * i + 4 * (lane / 16) + v, col = n0 + 16 * j + r;
                if (row < M && col < N) Cz[(int64_t)row * ldc + col] = acc[i][j][v];
            }
}

// out = act(sum over S splits of part + bias[col]); act 1 = tanh.  out may alias part when S == 1.
__global__ __launch_bounds__(256) void epilogue_kernel(const float *part, int S, int64_t sstride, int M, int N,
                                                       int64_t ldp, const float *__restrict__ bias, int act,
                                                       float *out, int64_t ldo)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    // M N < 2^31 (checked by the caller): 32-bit division
    const unsigned iu = (unsigned)i, row = iu / (unsigned)N, col = iu - row * (unsigned)N;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * sstride + (int64_t)row * ldp + col];
    if (bias) s += bias[col];
    if (act) s = tanhf(s);
    out[(int64_t)row * ldo + col] = s;
}

// X (R x Cc, FP32, ldx) -> hi/lo/lo2 (rows < Rp, columns < Cp, ldh) and/or the transposes
// hiT/loT/lo2T (rows < Cp, columns < Rp, ldt; lo2 / lo2T may be null); entries outside R x Cc are
// written as zero.  32 x 32
// tiles through LDS so that both the row-major and the transposed stores are coalesced.  x - hi and
// x - hi - lo are exact in FP32 (each difference has at most 16 significant bits).
__global__ __launch_bounds__(256) void convert_kernel(const float *__restrict__ X, int R, int Cc, int64_t ldx, int Rp,
                                                      int Cp, u16 *__restrict__ hi, u16 *__restrict__ lo,
                                                      u16 *__restrict__ lo2, int64_t ldh, u16 *__restrict__ hiT,
                                                      u16 *__restrict__ loT, u16 *__restrict__ lo2T, int64_t ldt)
{
    __shared__ float tile[32][33];
    const int c0 = (int)blockIdx.x * 32, r0 = (int)blockIdx.y * 32;
    const int tx = (int)threadIdx.x % 32, ty = (int)threadIdx.x / 32;
    for (int k = ty; k < 32; k += 8) {
        const int rr = r0 + k, cc = c0 + tx;
        const float v = (rr < R && cc < Cc) ? X[(int64_t)rr * ldx + cc] : 0.f;
        tile[k][tx] = v;
        if (hi && rr < Rp && cc < Cp) {
            const u16 h = bf16_rne(v);
            const float r1 = v - bf16_f(h);
            const u16 l = bf16_rne(r1);
            hi[(int64_t)rr * ldh + cc] = h;
            lo[(int64_t)rr * ldh + cc] = l;
            if (lo2) lo2[(int64_t)rr * ldh + cc] = bf16_rne(r1 - bf16_f(l));
        }
    }
    if (hiT) {  // uniform over the block
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int cc = c0 + k, rr = r0 + tx;
            if (cc < Cp && rr < Rp) {
                const float v = tile[tx][k];
                const u16 h = bf16_rne(v);
                const float r1 = v - bf16_f(h);
                const u16 l = bf16_rne(r1);
                hiT[(int64_t)cc * ldt + rr] = h;
                loT[(int64_t)cc * ldt + rr] = l;
                if (lo2T) lo2T[(int64_t)cc * ldt + rr] = bf16_rne(r1 - bf16_f(l));
            }
        }
    }
}

__device__ __forceinline__ int64_t row_of(const int64_t *idx, int n) { return idx ? idx[n] : (int64_t)n; }

// gap layer: gt[n] and h1[n][w] = tanh(W1[w] gt[n] + b1[w]); padding rows use gt = 0
__global__ __launch_bounds__(256) void l1_forward_kernel(int B, int Bp, const int64_t *__restrict__ idx,
                                                         const double *__restrict__ g, double gmid, double ghalf,
                                                         const float *__restrict__ W1, const float *__restrict__ b1,
                                                         int W, float *__restrict__ gt, float *__restrict__ h1)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)Bp * W) return;
    const int n = (int)(i / W), w = (int)(i % W);
    const float t = n < B ? (float)((log(g[row_of(idx, n)]) - gmid) / ghalf) : 0.f;
    if (w == 0) gt[n] = t;
    h1[i] = tanhf(fmaf(W1[w], t, b1[w]));
}

// z[n][w] = sum_k a4[n][12 w + k] m[n][k]; padding rows 0
__global__ __launch_bounds__(256) void contract_kernel(int B, int Bp, const int64_t *__restrict__ idx,
                                                       const double *__restrict__ mot, const float *__restrict__ a4,
                                                       int W, float *__restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)Bp * W) return;
    const int n = (int)(i / W), w = (int)(i % W);
    float s = 0.f;
    if (n < B) {
        const double *mm = mot + kNMot * row_of(idx, n);
        const float *a = a4 + (int64_t)n * kNMot * W + (int64_t)kNMot * w;
#pragma unroll
        for (int k = 0; k < kNMot; ++k) s = fmaf(a[k], (float)mm[k], s);
    }
    z[i] = s;
}

// da4[n][12 w + k] = dz[n][w] m[n][k]; padding rows 0
__global__ __launch_bounds__(256) void contract_back_kernel(int B, int Bp, const int64_t *__restrict__ idx,
                                                            const double *__restrict__ mot,
                                                            const float *__restrict__ dz, int W,
                                                            float *__restrict__ da4)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t K = (int64_t)kNMot * W;
    if (i >= (int64_t)Bp * K) return;
    const int n = (int)(i / K);
    const int j = (int)(i % K), w = j / kNMot, k = j % kNMot;
    da4[i] = n < B ? dz[(int64_t)n * W + w] * (float)mot[kNMot * row_of(idx, n) + k] : 0.f;
}

// d = o - y / s (FP64); dout = 2 d / (B P) for rows < B, 0 for padding rows; per-block sums of d^2.
// Grid (kLossCols, Bp): block (x, n) covers the columns x * 256 + t, strided by kLossCols * 256, of row n;
// its sum goes to partial[n kLossCols + x].
constexpr int kLossCols = 16;
__global__ __launch_bounds__(256) void loss_kernel(int B, int64_t P, const int64_t *__restrict__ idx,
                                                   const double *__restrict__ y, int64_t ldy,
                                                   const double *__restrict__ s, const float *__restrict__ o,
                                                   int64_t ldo, float *__restrict__ dout, int64_t ldd,
                                                   double *__restrict__ partial)
{
    __shared__ double red[256];
    const int n = (int)blockIdx.y;
    const double scale = 2.0 / ((double)B * (double)P);
    double acc = 0.0;
    const float *on = o + (int64_t)n * ldo;
    float *dn = dout + (int64_t)n * ldd;
    if (n < B) {
        const double *yn = y + row_of(idx, n) * ldy;
        for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)kLossCols * 256) {
            const double d = (double)on[p] - yn[p] / s[p];
            acc += d * d;
            dn[p] = (float)(scale * d);
        }
    } else {
        for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)kLossCols * 256) dn[p] = 0.f;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)n * kLossCols + blockIdx.x] = red[0];
}

// one block of 256: each thread sums a fixed strided subset, then a fixed-order tree (reproducible)
__global__ __launch_bounds__(256) void loss_final_kernel(const double *__restrict__ partial, int nb, double inv_count,
                                                         double *__restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = (int)threadIdx.x; b < nb; b += 256) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * inv_count;
}

// d = dh (1 - h^2)
__global__ __launch_bounds__(256) void tanh_back_kernel(int64_t n, const float *__restrict__ dh,
                                                        const float *__restrict__ h, float *__restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float hv = h[i];
    d[i] = dh[i] * (1.f - hv * hv);
}

// out[c] = sum over rows r < R of X[r][c], rows in order (one thread per column)
__global__ __launch_bounds__(256) void colsum_kernel(int R, int N, const float *__restrict__ X, int64_t ldx,
                                                     float *__restrict__ out)
{
    const int c = (int)(blockIdx.x * 256 + threadIdx.x);
    if (c >= N) return;
    float s = 0.f;
#pragma unroll 8
    for (int r = 0; r < R; ++r) s += X[(int64_t)r * ldx + c];
    out[c] = s;
}

// dW1[w] = sum_n d1[n][w] gt[n], db1[w] = sum_n d1[n][w]
__global__ __launch_bounds__(256) void l1_back_kernel(int B, int W, const float *__restrict__ d1,
                                                      const float *__restrict__ gt, float *__restrict__ dW1,
                                                      float *__restrict__ db1)
{
    const int w = (int)(blockIdx.x * 256 + threadIdx.x);
    if (w >= W) return;
    float a = 0.f, b = 0.f;
#pragma unroll 8
    for (int n = 0; n < B; ++n) {
        const float d = d1[(int64_t)n * W + w];
        a = fmaf(d, gt[n], a);
        b += d;
    }
    dW1[w] = a;
    db1[w] = b;
}

__global__ __launch_bounds__(256) void adam_kernel(int64_t n, float *__restrict__ th, float *__restrict__ m1,
                                                   float *__restrict__ m2, const float *__restrict__ g, float lr,
                                                   float beta1, float beta2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = beta1 * m1[i] + (1.f - beta1) * gi;
    const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    th[i] -= lr * (a * c1) / (sqrtf(b * c2) + eps);
}

// s[p] = sqrt(mean_n y[n][p]^2) (1 where that is 0)
__global__ __launch_bounds__(256) void rms_kernel(int64_t nrow, int64_t P, const double *__restrict__ y, int64_t ldy,
                                                  double *__restrict__ s)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double a = 0.0;
    for (int64_t n = 0; n < nrow; ++n) {
        const double v = y[n * ldy + p];
        a += v * v;
    }
    const double r = sqrt(a / (double)nrow);
    s[p] = r > 0.0 ? r : 1.0;
}

// q[n][p] = s[p] o[n][p]
__global__ __launch_bounds__(256) void predict_kernel(int B, int64_t P, const float *__restrict__ o, int64_t ldo,
                                                      const double *__restrict__ s, double *__restrict__ q)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)B * P) return;
    const int n = (int)(i / P);
    const int64_t p = i % P;
    q[i] = s[p] * (double)o[(int64_t)n * ldo + p];
}

__global__ __launch_bounds__(256) void fill_u16_kernel(int64_t n, u16 *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------------------------

struct Bf {  // one FP32 matrix as BF16 hi/lo/lo2, row-major, and optionally its transpose
    u16 *hi = nullptr, *lo = nullptr, *lo2 = nullptr, *hiT = nullptr, *loT = nullptr, *lo2T = nullptr;
    int64_t ld = 0, ldT = 0;
};

// one GEMM operand: the three BF16 pieces of a K-contiguous matrix and its leading dimension
struct Op {
    const u16 *hi, *lo, *lo2;
    int64_t ld;
};
inline Op rows_of(const Bf &b) { return Op{b.hi, b.lo, b.lo2, b.ld}; }
inline Op cols_of(const Bf &b) { return Op{b.hiT, b.loT, b.lo2T, b.ldT}; }

}  // namespace

struct sr_mlp {
    int device = 0;
    int W = 0;
    int64_t P = 0, Pp = 0;
    int Bmax = 0, Bpm = 0;
    int passes = 3;
    double gmid = -2.760730458931123, ghalf = 1.151292546497023;  // ln 0.02 .. ln 0.2 -> -1 .. 1
    int64_t off[9] = {}, sz[9] = {}, nparam = 0;
    int64_t step = 0;
    bool have_params = false, have_scale = false;
    std::vector<void *> allocs;
    float *theta = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr;
    double *scale = nullptr;
    Bf w2, w3, w4, wh;
    // activations (FP32, Bpm rows) and their BF16 forms
    float *gt = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *a4 = nullptr, *z = nullptr, *o = nullptr;
    float *dout = nullptr, *dz = nullptr, *da4 = nullptr, *dh = nullptr, *d3 = nullptr, *d2 = nullptr,
          *d1 = nullptr;
    float *part = nullptr;
    double *lpart = nullptr, *lval = nullptr;
    Bf bh1, bh2, bh3, bz, bdout, bda4, bd3, bd2;
    // profiling of training steps: 5 events per step (start, forward, backward, Adam, weight copies)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool, ev_rec;

    template <typename T>
    hipError_t alloc(T **p, int64_t n)
    {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
        if (e != hipSuccess) return e;
        allocs.push_back(q);
        *p = (T *)q;
        return hipSuccess;
    }
};

namespace {

// hi/lo/lo2 buffers (rows x ld) and transposes (cols x ldT), zero-filled
sr_status alloc_bf(sr_mlp *M, Bf &b, int64_t rows, int64_t ld, int64_t cols, int64_t ldT, hipStream_t s)
{
    b.ld = ld;
    b.ldT = ldT;
    if (rows > 0) {
        for (u16 **q : {&b.hi, &b.lo, &b.lo2}) {
            MHIP(M->alloc(q, rows * ld));
            hipLaunchKernelGGL(fill_u16_kernel, dim3(nblk(rows * ld)), dim3(256), 0, s, rows * ld, *q);
        }
    }
    if (cols > 0) {
        for (u16 **q : {&b.hiT, &b.loT, &b.lo2T}) {
            MHIP(M->alloc(q, cols * ldT));
            hipLaunchKernelGGL(fill_u16_kernel, dim3(nblk(cols * ldT)), dim3(256), 0, s, cols * ldT, *q);
        }
    }
    MHIP(hipGetLastError());
    return SR_OK;
}

// X (R x Cc) -> b.hi/lo/lo2 over Rp x Cp and b.hiT/loT/lo2T over Cp x Rp (those present)
// third: also the lo2 pieces (read by the six-product matrix products only)
sr_status convert(const float *X, int64_t R, int64_t Cc, int64_t ldx, int64_t Rp, int64_t Cp, const Bf &b,
                  bool rowmajor, bool transposed, bool third, hipStream_t s)
{
    dim3 grid((unsigned)((Cp + 31) / 32), (unsigned)((Rp + 31) / 32));
    hipLaunchKernelGGL(convert_kernel, grid, dim3(256), 0, s, X, (int)R, (int)Cc, ldx, (int)Rp, (int)Cp,
                       rowmajor ? b.hi : nullptr, rowmajor ? b.lo : nullptr, rowmajor && third ? b.lo2 : nullptr,
                       b.ld, transposed ? b.hiT : nullptr, transposed ? b.loT : nullptr,
                       transposed && third ? b.lo2T : nullptr, b.ldT);
    MHIP(hipGetLastError());
    return SR_OK;
}

// C (M x N) = A (M x Kpad) B^T (N x Kpad): A and B row-major with K contiguous.
// S > 1 splits K into S ranges written to M->part and summed by the epilogue.
sr_status gemm(sr_mlp *Mo, const Op &A, const Op &B, int M, int N, int64_t Kpad, float *C, int64_t ldc,
               const float *bias, int act, int S, hipStream_t s)
{
    const int64_t lda = A.ld, ldb = B.ld;
    if (Kpad % kPad != 0 || lda % 8 != 0 || ldb % 8 != 0 || M < 1 || N < 1 || (int64_t)M * N >= ((int64_t)1 << 31))
        return mfail(SR_EINVAL, "internal: gemm operand shapes");
    const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
    if (S == 1 && tiles < 128 && Mo->part) {
        // few output tiles (batch x width products): split K so that the machine has work, at least
        // two K steps per split; the partial products are summed by the epilogue in a fixed order
        const int64_t want = (256 + tiles - 1) / tiles, most = std::max<int64_t>(1, Kpad / (2 * kPad));
        const int64_t room = (int64_t)Mo->Bpm * Mo->W * kMaxSplit / ((int64_t)M * N);  // split buffer capacity
        S = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, most), std::min<int64_t>(room, kMaxSplit)));
    }
    int64_t kchunk = pad_up((Kpad + S - 1) / S);
    S = (int)((Kpad + kchunk - 1) / kchunk);
    float *dst = S == 1 ? C : Mo->part;
    const int64_t ldd = S == 1 ? ldc : N;
    const int64_t sstride = (int64_t)M * N;
    if (S > 1 && (!Mo->part || sstride * S > (int64_t)Mo->Bpm * Mo->W * kMaxSplit))
        return mfail(SR_EINVAL, "internal: split buffer");
    dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64), (unsigned)S);
    if (Mo->passes == 6)
        hipLaunchKernelGGL(gemm_nt_kernel<6>, grid, dim3(256), 0, s, A.hi, A.lo, A.lo2, lda, B.hi, B.lo, B.lo2, ldb,
                           M, N, (int)Kpad, (int)kchunk, dst, ldd, sstride);
    else if (Mo->passes == 3)
        hipLaunchKernelGGL(gemm_nt_kernel<3>, grid, dim3(256), 0, s, A.hi, A.lo, A.lo2, lda, B.hi, B.lo, B.lo2, ldb,
                           M, N, (int)Kpad, (int)kchunk, dst, ldd, sstride);
    else
        hipLaunchKernelGGL(gemm_nt_kernel<1>, grid, dim3(256), 0, s, A.hi, A.lo, A.lo2, lda, B.hi, B.lo, B.lo2, ldb,
                           M, N, (int)Kpad, (int)kchunk, dst, ldd, sstride);
    MHIP(hipGetLastError());
    if (S > 1 || bias || act) {
        hipLaunchKernelGGL(epilogue_kernel, dim3(nblk((int64_t)M * N)), dim3(256), 0, s, dst, S, sstride, M, N, ldd,
                           bias, act, C, ldc);
        MHIP(hipGetLastError());
    }
    return SR_OK;
}

float *blk(sr_mlp *M, float *base, int b) { return base + M->off[b]; }
enum { PW1 = 0, PB1, PW2, PB2, PW3, PB3, PW4, PB4, PWH };

// BF16 copies of the weight matrices (row-major for the forward products, transposed for the
// backward ones)
sr_status refresh_weights(sr_mlp *M, hipStream_t s)
{
    const int W = M->W;
    MSR(convert(blk(M, M->theta, PW2), W, W, W, W, W, M->w2, true, true, M->passes == 6, s));
    MSR(convert(blk(M, M->theta, PW3), W, W, W, W, W, M->w3, true, true, M->passes == 6, s));
    MSR(convert(blk(M, M->theta, PW4), (int64_t)kNMot * W, W, W, (int64_t)kNMot * W, W, M->w4, true, true, M->passes == 6, s));
    MSR(convert(blk(M, M->theta, PWH), M->P, W, W, M->Pp, W, M->wh, true, true, M->passes == 6, s));
    return SR_OK;
}

sr_status forward(sr_mlp *M, int B, const int64_t *idx, const double *g, const double *mot, hipStream_t s)
{
    const int W = M->W, Bp = (int)pad_up(B), K4 = kNMot * W;
    hipLaunchKernelGGL(l1_forward_kernel, dim3(nblk((int64_t)Bp * W)), dim3(256), 0, s, B, Bp, idx, g, M->gmid,
                       M->ghalf, blk(M, M->theta, PW1), blk(M, M->theta, PB1), W, M->gt, M->h1);
    MHIP(hipGetLastError());
    MSR(convert(M->h1, Bp, W, W, Bp, W, M->bh1, true, true, M->passes == 6, s));
    MSR(gemm(M, rows_of(M->bh1), rows_of(M->w2), Bp, W, W, M->h2, W, blk(M, M->theta, PB2), 1, 1, s));
    MSR(convert(M->h2, Bp, W, W, Bp, W, M->bh2, true, true, M->passes == 6, s));
    MSR(gemm(M, rows_of(M->bh2), rows_of(M->w3), Bp, W, W, M->h3, W, blk(M, M->theta, PB3), 1, 1, s));
    MSR(convert(M->h3, Bp, W, W, Bp, W, M->bh3, true, true, M->passes == 6, s));
    MSR(gemm(M, rows_of(M->bh3), rows_of(M->w4), Bp, K4, W, M->a4, K4, blk(M, M->theta, PB4), 0, 1, s));
    hipLaunchKernelGGL(contract_kernel, dim3(nblk((int64_t)Bp * W)), dim3(256), 0, s, B, Bp, idx, mot, M->a4, W, M->z);
    MHIP(hipGetLastError());
    MSR(convert(M->z, Bp, W, W, Bp, W, M->bz, true, true, M->passes == 6, s));
    MSR(gemm(M, rows_of(M->bz), rows_of(M->wh), Bp, (int)M->P, W, M->o, M->Pp, nullptr, 0, 1, s));
    return SR_OK;
}

// gradients of the loss into M->grad, loss into M->lval (device)
sr_status backward(sr_mlp *M, int B, const int64_t *idx, const double *mot, const double *y, hipStream_t s)
{
    const int W = M->W, Bp = (int)pad_up(B), K4 = kNMot * W;
    const int64_t P = M->P, Pp = M->Pp;
    hipLaunchKernelGGL(loss_kernel, dim3(kLossCols, (unsigned)Bp), dim3(256), 0, s, B, P, idx, y, P, M->scale, M->o, Pp,
                       M->dout, Pp, M->lpart);
    MHIP(hipGetLastError());
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, M->lpart, Bp * kLossCols,
                       1.0 / ((double)B * (double)P), M->lval);
    MHIP(hipGetLastError());
    MSR(convert(M->dout, Bp, P, Pp, Bp, Pp, M->bdout, true, true, M->passes == 6, s));
    // head: dWh = dout^T z, dz = dout Wh
    MSR(gemm(M, cols_of(M->bdout), cols_of(M->bz), (int)P, W, Bp, blk(M, M->grad, PWH), W, nullptr, 0, 1, s));
    const int S = (int)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1, Pp / 512));
    MSR(gemm(M, rows_of(M->bdout), cols_of(M->wh), Bp, W, Pp, M->dz, W, nullptr, 0, S, s));
    hipLaunchKernelGGL(contract_back_kernel, dim3(nblk((int64_t)Bp * K4)), dim3(256), 0, s, B, Bp, idx, mot, M->dz, W,
                       M->da4);
    MHIP(hipGetLastError());
    MSR(convert(M->da4, Bp, K4, K4, Bp, K4, M->bda4, true, true, M->passes == 6, s));
    // layer 4
    MSR(gemm(M, cols_of(M->bda4), cols_of(M->bh3), K4, W, Bp, blk(M, M->grad, PW4), W, nullptr, 0, 1, s));
    hipLaunchKernelGGL(colsum_kernel, dim3(nblk(K4)), dim3(256), 0, s, B, K4, M->da4, (int64_t)K4, blk(M, M->grad, PB4));
    MHIP(hipGetLastError());
    MSR(gemm(M, rows_of(M->bda4), cols_of(M->w4), Bp, W, K4, M->dh, W, nullptr, 0, 1, s));
    // layer 3
    hipLaunchKernelGGL(tanh_back_kernel, dim3(nblk((int64_t)Bp * W)), dim3(256), 0, s, (int64_t)Bp * W, M->dh, M->h3,
                       M->d3);
    MHIP(hipGetLastError());
    MSR(convert(M->d3, Bp, W, W, Bp, W, M->bd3, true, true, M->passes == 6, s));
    MSR(gemm(M, cols_of(M->bd3), cols_of(M->bh2), W, W, Bp, blk(M, M->grad, PW3), W, nullptr, 0, 1, s));
    hipLaunchKernelGGL(colsum_kernel, dim3(nblk(W)), dim3(256), 0, s, B, W, M->d3, (int64_t)W, blk(M, M->grad, PB3));
    MHIP(hipGetLastError());
    MSR(gemm(M, rows_of(M->bd3), cols_of(M->w3), Bp, W, W, M->dh, W, nullptr, 0, 1, s));
    // layer 2
    hipLaunchKernelGGL(tanh_back_kernel, dim3(nblk((int64_t)Bp * W)), dim3(256), 0, s, (int64_t)Bp * W, M->dh, M->h2,
                       M->d2);
    MHIP(hipGetLastError());
    MSR(convert(M->d2, Bp, W, W, Bp, W, M->bd2, true, true, M->passes == 6, s));
    MSR(gemm(M, cols_of(M->bd2), cols_of(M->bh1), W, W, Bp, blk(M, M->grad, PW2), W, nullptr, 0, 1, s));
    hipLaunchKernelGGL(colsum_kernel, dim3(nblk(W)), dim3(256), 0, s, B, W, M->d2, (int64_t)W, blk(M, M->grad, PB2));
    MHIP(hipGetLastError());
    MSR(gemm(M, rows_of(M->bd2), cols_of(M->w2), Bp, W, W, M->dh, W, nullptr, 0, 1, s));
    // layer 1 (the gap layer)
    hipLaunchKernelGGL(tanh_back_kernel, dim3(nblk((int64_t)Bp * W)), dim3(256), 0, s, (int64_t)Bp * W, M->dh, M->h1,
                       M->d1);
    MHIP(hipGetLastError());
    hipLaunchKernelGGL(l1_back_kernel, dim3(nblk(W)), dim3(256), 0, s, B, W, M->d1, M->gt, blk(M, M->grad, PW1),
                       blk(M, M->grad, PB1));
    MHIP(hipGetLastError());
    return SR_OK;
}

struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int d)
    {
        (void)hipGetDevice(&prev);
        ok = hipSetDevice(d) == hipSuccess;
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

sr_status mark(sr_mlp *M, hipStream_t s)
{
    if (!M->profiling) return SR_OK;
    hipEvent_t e;
    if (!M->ev_pool.empty()) {
        e = M->ev_pool.back();
        M->ev_pool.pop_back();
    } else {
        MHIP(hipEventCreate(&e));
    }
    M->ev_rec.push_back(e);
    MHIP(hipEventRecord(e, s));
    return SR_OK;
}

sr_status check_batch(sr_mlp *M, int B, const char *who)
{
    if (!M) return mfail(SR_EINVAL, std::string(who) + ": NULL network");
    if (B < 1 || B > M->Bmax) return mfail(SR_EINVAL, std::string(who) + ": batch must be in 1..max_batch");
    if (!M->have_params) return mfail(SR_ESTATE, std::string(who) + ": set the parameters first");
    return SR_OK;
}

// every selected row must exist: idx (device, B values) in [0, nrows), or B <= nrows without idx
sr_status check_rows(const int64_t *idx, int B, int64_t nrows, hipStream_t s, const char *who)
{
    if (!idx) {
        if (nrows < B) return mfail(SR_EINVAL, std::string(who) + ": nrows < batch");
        return SR_OK;
    }
    std::vector<int64_t> h(B);
    MHIP(hipMemcpyAsync(h.data(), idx, B * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MHIP(hipStreamSynchronize(s));
    for (int i = 0; i < B; ++i)
        if (h[i] < 0 || h[i] >= nrows) return mfail(SR_EINVAL, std::string(who) + ": idx out of range");
    return SR_OK;
}

}  // namespace

extern "C" {

int64_t sr_mlp_num_params(int width, int64_t nout)
{
    const int64_t W = width;
    return W + W + W * W + W + W * W + W + kNMot * W * W + kNMot * W + nout * W;
}

sr_status sr_mlp_create(sr_mlp **out, int device, int width, int64_t nout, int max_batch)
{
    g_merr.clear();
    if (!out) return mfail(SR_EINVAL, "sr_mlp_create: out is NULL");
    *out = nullptr;
    if (width < 32 || width > 4096 || width % 32 != 0) return mfail(SR_EINVAL, "sr_mlp_create: width must be a multiple of 32 in 32..4096");
    if (nout < 1 || nout > (int64_t(1) << 28)) return mfail(SR_EINVAL, "sr_mlp_create: nout out of range");
    if (max_batch < 1 || max_batch > 4096) return mfail(SR_EINVAL, "sr_mlp_create: max_batch must be in 1..4096");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || device < 0 || device >= count)
        return mfail(SR_ENODEV, "sr_mlp_create: no such HIP device");
    DevGuard g(device);
    if (!g.ok) return mfail(SR_ENODEV, "sr_mlp_create: cannot select device");
    sr_mlp *M = new (std::nothrow) sr_mlp();
    if (!M) return mfail(SR_ENOMEM, "sr_mlp_create: out of host memory");
    M->device = device;
    M->W = width;
    M->P = nout;
    M->Pp = pad_up(nout);
    M->Bmax = max_batch;
    M->Bpm = (int)pad_up(max_batch);
    const int64_t W = width, K4 = kNMot * W, Bpm = M->Bpm, P = nout, Pp = M->Pp;
    const int64_t sizes[9] = {W, W, W * W, W, W * W, W, K4 * W, K4, P * W};
    int64_t o = 0;
    for (int b = 0; b < 9; ++b) {
        M->off[b] = o;
        M->sz[b] = sizes[b];
        o += sizes[b];
    }
    M->nparam = o;
    hipStream_t s = nullptr;
    auto fail_free = [&](sr_status st) {
        for (void *p : M->allocs) (void)hipFree(p);
        delete M;
        return st;
    };
#define MC(call)                                                                                      \
    do {                                                                                              \
        if ((call) != hipSuccess) return fail_free(mfail(SR_ENOMEM, "sr_mlp_create: device allocation failed")); \
    } while (0)
#define MCS(call)                                                                                     \
    do {                                                                                              \
        sr_status s_ = (call);                                                                        \
        if (s_ != SR_OK) return fail_free(s_);                                                        \
    } while (0)
    MC(M->alloc(&M->theta, o));
    MC(M->alloc(&M->mom, o));
    MC(M->alloc(&M->vel, o));
    MC(M->alloc(&M->grad, o));
    MC(M->alloc(&M->scale, P));
    MC(M->alloc(&M->gt, Bpm));
    MC(M->alloc(&M->h1, Bpm * W));
    MC(M->alloc(&M->h2, Bpm * W));
    MC(M->alloc(&M->h3, Bpm * W));
    MC(M->alloc(&M->a4, Bpm * K4));
    MC(M->alloc(&M->z, Bpm * W));
    MC(M->alloc(&M->o, Bpm * Pp));
    MC(M->alloc(&M->dout, Bpm * Pp));
    MC(M->alloc(&M->dz, Bpm * W));
    MC(M->alloc(&M->da4, Bpm * K4));
    MC(M->alloc(&M->dh, Bpm * W));
    MC(M->alloc(&M->d3, Bpm * W));
    MC(M->alloc(&M->d2, Bpm * W));
    MC(M->alloc(&M->d1, Bpm * W));
    MC(M->alloc(&M->part, Bpm * W * kMaxSplit));
    MC(M->alloc(&M->lpart, (int64_t)Bpm * kLossCols));
    MC(M->alloc(&M->lval, 1));
    MCS(alloc_bf(M, M->w2, W, W, W, W, s));
    MCS(alloc_bf(M, M->w3, W, W, W, W, s));
    MCS(alloc_bf(M, M->w4, K4, W, W, K4, s));
    MCS(alloc_bf(M, M->wh, Pp, W, W, Pp, s));
    MCS(alloc_bf(M, M->bh1, Bpm, W, W, Bpm, s));
    MCS(alloc_bf(M, M->bh2, Bpm, W, W, Bpm, s));
    MCS(alloc_bf(M, M->bh3, Bpm, W, W, Bpm, s));
    MCS(alloc_bf(M, M->bz, Bpm, W, W, Bpm, s));
    MCS(alloc_bf(M, M->bdout, Bpm, Pp, Pp, Bpm, s));
    MCS(alloc_bf(M, M->bda4, Bpm, K4, K4, Bpm, s));
    MCS(alloc_bf(M, M->bd3, Bpm, W, W, Bpm, s));
    MCS(alloc_bf(M, M->bd2, Bpm, W, W, Bpm, s));
#undef MC
#undef MCS
    if (hipStreamSynchronize(s) != hipSuccess) return fail_free(mfail(SR_EHIP, "sr_mlp_create: initialization failed"));
    *out = M;
    return SR_OK;
}

sr_status sr_mlp_destroy(sr_mlp *M)
{
    g_merr.clear();
    if (!M) return SR_OK;
    DevGuard g(M->device);
    (void)hipDeviceSynchronize();
    for (void *p : M->allocs) (void)hipFree(p);
    for (hipEvent_t e : M->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : M->ev_rec) (void)hipEventDestroy(e);
    delete M;
    return SR_OK;
}

sr_status sr_mlp_set_options(sr_mlp *M, int passes, double g_mid, double g_half)
{
    g_merr.clear();
    if (!M) return mfail(SR_EINVAL, "sr_mlp_set_options: NULL network");
    if (passes != 1 && passes != 3 && passes != 6) return mfail(SR_EINVAL, "sr_mlp_set_options: passes must be 1, 3 or 6");
    if (!std::isfinite(g_mid) || !(g_half > 0.0) || !std::isfinite(g_half))
        return mfail(SR_EINVAL, "sr_mlp_set_options: need finite g_mid and g_half > 0");
    const bool redo = passes == 6 && M->passes != 6 && M->have_params;
    M->passes = passes;
    M->gmid = g_mid;
    M->ghalf = g_half;
    if (redo) {  // the weights' lo2 pieces are written only for the six-product mode
        DevGuard g(M->device);
        MSR(refresh_weights(M, nullptr));
        MHIP(hipStreamSynchronize(nullptr));
    }
    return SR_OK;
}

sr_status sr_mlp_set_params(sr_mlp *M, const float *params)
{
    g_merr.clear();
    if (!M || !params) return mfail(SR_EINVAL, "sr_mlp_set_params: NULL argument");
    for (int64_t i = 0; i < M->nparam; ++i)
        if (!std::isfinite(params[i])) return mfail(SR_EINVAL, "sr_mlp_set_params: parameter not finite");
    DevGuard g(M->device);
    if (!g.ok) return mfail(SR_ENODEV, "sr_mlp_set_params: cannot select device");
    hipStream_t s = nullptr;
    MHIP(hipMemcpy(M->theta, params, M->nparam * sizeof(float), hipMemcpyHostToDevice));
    MHIP(hipMemset(M->mom, 0, M->nparam * sizeof(float)));
    MHIP(hipMemset(M->vel, 0, M->nparam * sizeof(float)));
    MSR(refresh_weights(M, s));
    MHIP(hipStreamSynchronize(s));
    M->step = 0;
    M->have_params = true;
    if (!M->have_scale) {
        std::vector<double> one(M->P, 1.0);
        MHIP(hipMemcpy(M->scale, one.data(), M->P * sizeof(double), hipMemcpyHostToDevice));
        M->have_scale = true;
    }
    return SR_OK;
}

sr_status sr_mlp_get_params(sr_mlp *M, float *params)
{
    g_merr.clear();
    if (!M || !params) return mfail(SR_EINVAL, "sr_mlp_get_params: NULL argument");
    if (!M->have_params) return mfail(SR_ESTATE, "sr_mlp_get_params: no parameters set");
    DevGuard g(M->device);
    MHIP(hipDeviceSynchronize());
    MHIP(hipMemcpy(params, M->theta, M->nparam * sizeof(float), hipMemcpyDeviceToHost));
    return SR_OK;
}

sr_status sr_mlp_set_output_scale(sr_mlp *M, const double *s_dev, void *stream)
{
    g_merr.clear();
    if (!M || !s_dev) return mfail(SR_EINVAL, "sr_mlp_set_output_scale: NULL argument");
    DevGuard g(M->device);
    MHIP(hipMemcpyAsync(M->scale, s_dev, M->P * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    M->have_scale = true;
    return SR_OK;
}

sr_status sr_mlp_fit_output_scale(sr_mlp *M, int64_t n, const double *y, void *stream)
{
    g_merr.clear();
    if (!M || !y) return mfail(SR_EINVAL, "sr_mlp_fit_output_scale: NULL argument");
    if (n < 1) return mfail(SR_EINVAL, "sr_mlp_fit_output_scale: n < 1");
    DevGuard g(M->device);
    hipLaunchKernelGGL(rms_kernel, dim3(nblk(M->P)), dim3(256), 0, (hipStream_t)stream, n, M->P, y, M->P, M->scale);
    MHIP(hipGetLastError());
    M->have_scale = true;
    return SR_OK;
}

sr_status sr_mlp_get_output_scale(sr_mlp *M, double *s_dev, void *stream)
{
    g_merr.clear();
    if (!M || !s_dev) return mfail(SR_EINVAL, "sr_mlp_get_output_scale: NULL argument");
    DevGuard g(M->device);
    MHIP(hipMemcpyAsync(s_dev, M->scale, M->P * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SR_OK;
}

sr_status sr_mlp_forward(sr_mlp *M, int B, const double *gap, const double *motion, float *out, void *stream)
{
    g_merr.clear();
    MSR(check_batch(M, B, "sr_mlp_forward"));
    if (!gap || !motion || !out) return mfail(SR_EINVAL, "sr_mlp_forward: NULL argument");
    DevGuard g(M->device);
    hipStream_t s = (hipStream_t)stream;
    MSR(forward(M, B, nullptr, gap, motion, s));
    MHIP(hipMemcpy2DAsync(out, M->P * sizeof(float), M->o, M->Pp * sizeof(float), M->P * sizeof(float), B,
                          hipMemcpyDeviceToDevice, s));
    return SR_OK;
}

sr_status sr_mlp_predict(sr_mlp *M, int B, const double *gap, const double *motion, double *q, void *stream)
{
    g_merr.clear();
    MSR(check_batch(M, B, "sr_mlp_predict"));
    if (!gap || !motion || !q) return mfail(SR_EINVAL, "sr_mlp_predict: NULL argument");
    DevGuard g(M->device);
    hipStream_t s = (hipStream_t)stream;
    MSR(forward(M, B, nullptr, gap, motion, s));
    hipLaunchKernelGGL(predict_kernel, dim3(nblk((int64_t)B * M->P)), dim3(256), 0, s, B, M->P, M->o, M->Pp, M->scale, q);
    MHIP(hipGetLastError());
    return SR_OK;
}

sr_status sr_mlp_gradients(sr_mlp *M, int B, const int64_t *idx, int64_t nrows, const double *gap,
                           const double *motion, const double *y, float *grad, double *loss, void *stream)
{
    g_merr.clear();
    MSR(check_batch(M, B, "sr_mlp_gradients"));
    if (!gap || !motion || !y || !grad) return mfail(SR_EINVAL, "sr_mlp_gradients: NULL argument");
    DevGuard g(M->device);
    hipStream_t s = (hipStream_t)stream;
    MSR(check_rows(idx, B, nrows, s, "sr_mlp_gradients"));
    MSR(forward(M, B, idx, gap, motion, s));
    MSR(backward(M, B, idx, motion, y, s));
    MHIP(hipMemcpyAsync(grad, M->grad, M->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (loss) {
        MHIP(hipMemcpyAsync(loss, M->lval, sizeof(double), hipMemcpyDeviceToHost, s));
        MHIP(hipStreamSynchronize(s));
    }
    return SR_OK;
}

sr_status sr_mlp_train_step(sr_mlp *M, int B, const int64_t *idx, int64_t nrows, const double *gap,
                            const double *motion, const double *y, float lr, double *loss, void *stream)
{
    g_merr.clear();
    MSR(check_batch(M, B, "sr_mlp_train_step"));
    if (!gap || !motion || !y) return mfail(SR_EINVAL, "sr_mlp_train_step: NULL argument");
    if (!(lr > 0.f) || !std::isfinite(lr)) return mfail(SR_EINVAL, "sr_mlp_train_step: need lr > 0");
    DevGuard g(M->device);
    hipStream_t s = (hipStream_t)stream;
    MSR(check_rows(idx, B, nrows, s, "sr_mlp_train_step"));
    MSR(mark(M, s));
    MSR(forward(M, B, idx, gap, motion, s));
    MSR(mark(M, s));
    MSR(backward(M, B, idx, motion, y, s));
    MSR(mark(M, s));
    const double b1 = 0.9, b2 = 0.999;
    M->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)M->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)M->step)));
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(M->nparam)), dim3(256), 0, s, M->nparam, M->theta, M->mom, M->vel, M->grad,
                       lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    MHIP(hipGetLastError());
    MSR(mark(M, s));
    MSR(refresh_weights(M, s));
    MSR(mark(M, s));
    if (loss) {
        MHIP(hipMemcpyAsync(loss, M->lval, sizeof(double), hipMemcpyDeviceToHost, s));
        MHIP(hipStreamSynchronize(s));
    }
    return SR_OK;
}

sr_status sr_mlp_set_profiling(sr_mlp *M, int on)
{
    g_merr.clear();
    if (!M) return mfail(SR_EINVAL, "sr_mlp_set_profiling: NULL network");
    M->profiling = on != 0;
    return SR_OK;
}

sr_status sr_mlp_get_profile(sr_mlp *M, double *ms, int64_t *steps)
{
    g_merr.clear();
    if (!M || !ms || !steps) return mfail(SR_EINVAL, "sr_mlp_get_profile: NULL argument");
    DevGuard g(M->device);
    for (int k = 0; k < SR_MLP_NPHASES; ++k) ms[k] = 0.0;
    *steps = 0;
    const size_t per = SR_MLP_NPHASES + 1;
    for (size_t i = 0; i + per <= M->ev_rec.size(); i += per) {
        MHIP(hipEventSynchronize(M->ev_rec[i + per - 1]));
        for (int k = 0; k < SR_MLP_NPHASES; ++k) {
            float a = 0.f;
            MHIP(hipEventElapsedTime(&a, M->ev_rec[i + k], M->ev_rec[i + k + 1]));
            ms[k] += a;
        }
        *steps += 1;
    }
    for (hipEvent_t e : M->ev_rec) M->ev_pool.push_back(e);
    M->ev_rec.clear();
    return SR_OK;
}

sr_status sr_mlp_gemm_test(int device, int passes, int M, int N, int K, const float *A, const float *Bm, float *C,
                           void *stream)
{
    g_merr.clear();
    if (passes != 1 && passes != 3 && passes != 6) return mfail(SR_EINVAL, "sr_mlp_gemm_test: passes must be 1, 3 or 6");
    if (M < 1 || N < 1 || K < 1 || M > 65536 || N > 65536 || K > 65536 || !A || !Bm || !C)
        return mfail(SR_EINVAL, "sr_mlp_gemm_test: bad arguments");
    DevGuard g(device);
    if (!g.ok) return mfail(SR_ENODEV, "sr_mlp_gemm_test: cannot select device");
    hipStream_t s = (hipStream_t)stream;
    // a scratch network object carries the split buffer and the pass count
    sr_mlp T;
    T.passes = passes;
    T.W = 32;
    T.Bpm = 32;
    const int64_t Kp = pad_up(K);
    Bf a, b;
    sr_status st = T.alloc(&T.part, (int64_t)T.Bpm * T.W * kMaxSplit) == hipSuccess ? SR_OK : SR_ENOMEM;
    if (st == SR_OK) st = alloc_bf(&T, a, M, Kp, 0, 0, s);
    if (st == SR_OK) st = alloc_bf(&T, b, N, Kp, 0, 0, s);
    if (st == SR_OK) st = convert(A, M, K, K, M, Kp, a, true, false, passes == 6, s);
    if (st == SR_OK) st = convert(Bm, N, K, K, N, Kp, b, true, false, passes == 6, s);
    if (st == SR_OK) st = gemm(&T, rows_of(a), rows_of(b), M, N, Kp, C, N, nullptr, 0, 1, s);
    (void)hipStreamSynchronize(s);
    for (void *p : T.allocs) (void)hipFree(p);
    return st;
}

const char *sr_mlp_last_error(void) { return g_merr.c_str(); }

}  // extern "C"

// Gather the caller's quadrature and densities into the library's cell-sorted source records:
// rec.x = x_o, rec.fw = f_o w_o, rec.nw = n_o w_o, rec.q = q_o with o = perm[i] (the caller's index of
// sorted record i); the single-precision records are the round-to-nearest images of the double ones,
// with the coordinates taken relative to the origin org.
// pos64 / pos32 (optional) repeat the coordinates in compact 32/16-byte form for the near-pair test.
#include "sr_internal.h"

namespace sr {
namespace {

__global__ __launch_bounds__(kBlock) void pack_kernel(const double *__restrict__ x, const double *__restrict__ nrm,
                                                      const double *__restrict__ w, const double *__restrict__ f,
                                                      const double *__restrict__ q,
                                                      const int64_t *__restrict__ perm, int64_t n, double ox,
                                                      double oy, double oz, SrcRec<double> *__restrict__ rec64,
                                                      SrcRec<float> *__restrict__ rec32,
                                                      Pos4<double> *__restrict__ pos64,
                                                      Pos4<float> *__restrict__ pos32)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    SrcRec<double> r;
    const double ww = w[o];
    r.x = x[3 * o];
    r.y = x[3 * o + 1];
    r.z = x[3 * o + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.nw[k] = nrm[3 * o + k] * ww;
        r.fw[k] = f ? f[3 * o + k] * ww : 0.0;
        r.q[k] = q ? q[3 * o + k] : 0.0;
    }
    rec64[i] = r;
    SrcRec<float> h;
    h.x = (float)(r.x - ox);
    h.y = (float)(r.y - oy);
    h.z = (float)(r.z - oz);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        h.fw[k] = (float)r.fw[k];
        h.nw[k] = (float)r.nw[k];
        h.q[k] = (float)r.q[k];
    }
    rec32[i] = h;
    if (pos64) pos64[i] = Pos4<double>{r.x, r.y, r.z, 0.0};
    if (pos32) pos32[i] = Pos4<float>{h.x, h.y, h.z, 0.0f};
}

}  // namespace

hipError_t launch_pack(const double *x, const double *nrm, const double *w, const double *f, const double *q,
                       const int64_t *perm, int64_t n, const double org[3], SrcRec<double> *rec64, SrcRec<float> *rec32,
                       Pos4<double> *pos64, Pos4<float> *pos32, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, x, nrm, w, f, q, perm, n, org[0], org[1],
                       org[2], rec64, rec32, pos64, pos32);
    return hipGetLastError();
}

}  // namespace sr

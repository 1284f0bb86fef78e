// Internal declarations of libstokesreg: device data layout, the shared pair classification, and
// the kernel launchers.  HIP for gfx950 (wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "stokesreg.h"

namespace sr {

// Source splits of the direct far field.  Workgroups are dispatched round-robin over the 8 XCDs,
// so split = blockIdx.x % 16 puts splits x and x + 8 on XCD x: each XCD's L2 holds one eighth of the
// sources.  16 rather than 8 splits: twice the wavefronts (about 7.6 per SIMD at 62k targets instead
// of 3.8) hide more of the VALU dependency latency (far kernel 2.47 -> 2.25 ms alone).
constexpr int kFarSplits = 16;
constexpr int kBlock = 256;       // threads per workgroup (4 waves of 64)
constexpr int kWave = 64;

// One quadrature point with its density channels, array-of-records so that a wavefront-uniform
// index loads a whole record through the scalar cache:
//   x      point
//   fw     f(x) w        (single layer; zero until an SL density is set)
//   nw     n(x) w        (both layers: the subtraction term of eq. (Stokes_SL1) and the n_k w of
//                         eq. (Stokes_DL1))
//   q      q(x)          (double layer; zero until a DL density is set)
template <typename T>
struct alignas(16) SrcRec {
    T x, y, z;
    T fw[3];
    T nw[3];
    T q[3];
};
static_assert(sizeof(SrcRec<float>) == 48, "record layout");
static_assert(sizeof(SrcRec<double>) == 96, "record layout");

// Candidate positions for the near-pair test, 16/32-byte aligned so a lane fetches one in one or two
// vector loads (w unused).
template <typename T>
struct alignas(4 * sizeof(T)) Pos4 {
    T x, y, z, w;
};

// Squared distance used to classify a pair as near (r^2 <= rc2) or far.  The far-field and the
// near-field kernels call this same function on the same rounded operands, so every pair is
// assigned to exactly one of the two sums.  Explicit fma keeps the instruction sequence fixed.
__device__ __forceinline__ float pair_r2(float yx, float yy, float yz, float xx, float xy, float xz)
{
    const float dx = yx - xx, dy = yy - xy, dz = yz - xz;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}
__device__ __forceinline__ double pair_r2(double yx, double yy, double yz, double xx, double xy, double xz)
{
    const double dx = yx - xx, dy = yy - xy, dz = yz - xz;
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

// Uniform cell grid over the sources: cells in x-major, z-fastest order; sources are stored sorted by
// cell, cell c owning records [cell_start[c], cell_start[c+1]).  The side is a third of the near
// radius plus its rounding margin (the reach), so the near pairs of a target lie in the cells within
// the reach of it: about 7 x 7 columns of 7 cells, of which the near-field kernel skips the columns
// whose box lies beyond the reach.
constexpr int kCellsPerReach = 3;
struct CellGrid {
    double lo[3];
    double side, inv_side;
    int g[3];
};

// Consistency report of a context's targets, written by the kernels and read by sr_check: bits
// kFlagFarTarget (a target of sr_eval_far with a source inside the near radius) and kFlagFarRule (a
// target of sr_eval whose |b| selects the far-field rule w = (1, 0, 0) with a source closer than
// cutoff * max_j delta_j); `first` is the smallest offending target index.
constexpr unsigned kFlagFarTarget = 1u, kFlagFarRule = 2u;
struct NearFlag {
    unsigned int bits;
    unsigned int pad;
    unsigned long long first;
};

// Largest number of targets of one evaluation: 3 * m stays below 2^31, so the kernels' 32-bit
// target indices (3 t + component) cannot overflow.
constexpr int64_t kMaxTargets = int64_t(1) << 28;
// An evaluation runs in chunks of at most this many targets (its far-field partial sums, 768 bytes per
// target, and its target order are sized for one chunk); chunk i reports to NearFlag slot i.
constexpr int64_t kTargetChunk = int64_t(1) << 20;
constexpr int kFlagSlots = (int)(kMaxTargets / kTargetChunk);

struct EvalArgs {
    int layers;          // SR_SL | SR_DL bits
    int64_t m;
    const double *y, *x0, *n0, *b, *f0, *q0;
    double *u, *v, *u_delta, *v_delta;
    // Origin of the single-precision coordinates: the FP32 records hold x - org and the kernels
    // round y - org, so their rounding error scales with the source set's extent, not with its
    // distance from (0,0,0).  Zero for the FP64 path.
    double org[3];
};

// The three smoothing lengths in ascending order (the extrapolation is symmetric under reordering
// them): rho[o], inv_delta[o] for sorted position o; ord[o] is the caller's index of that delta.
struct DevParams {
    double h;
    double rho[3];
    double inv_delta[3];
    int ord[3];
    double cutoff;       // in t = r / delta
    double rnear;        // cutoff * max_j delta_j (and the modified-smoothing delta if larger)
    double rflag;        // a target with |b| >= cutoff * max_j delta_j and a source closer than this is
                         // reported (kFlagFarRule): cutoff * max_j delta_j less a rounding margin
    double reach;        // rnear plus the rounding margin of the pair test: every pair that test calls
                         // near is truly closer than this
    double reach_sharp;  // the same for the near radius rsharp of the surface targets (modified smoothing)
    int precision;
    int pow234;          // the sorted deltas are in the ratio 2 : 3 : 4 (exp(-t_j^2) by powers of one exp)
    int sharp;           // targets on the surface (b == 0) use the modified smoothing at one delta
    double inv_dsharp;   // 1 / that delta
    double rsharp;       // cutoff * that delta: the near radius of those targets (rnear otherwise)
    // Smoothing table of the targets on the surface (b == 0) in the combined mode, or nullptr: see
    // NearTable.  u = r * tab_scale in [0, kTabIntervals] indexes it; ih = 1 / h, ih3 = ih^3, ih5 = ih^5.
    const double *tab;
    double tab_scale, ih, ih3, ih5;
    // Order in which the near-field wavefronts take the targets, or nullptr for the caller's order:
    // the targets on the surface first, then the others, each part in Morton order, so that a
    // workgroup's four targets are neighbours and belong to the same launch (the smoothing-table
    // launch takes the first part, the closed-form launch the second), and the workgroups resident
    // at one time cover a compact piece of the surface, whose source records stay in the L2s.
    const int *order;
};

// Targets on the surface (b = 0) share one set of extrapolation weights (lambda_j = 0), so their
// combined smoothing factors S_k(r) = sum_j w_j s_k(r / delta_j) are fixed functions of x = r / h.  The
// table holds, on kTabIntervals equal intervals of x in [0, X] (X: the near radius over h, slightly
// widened), the degree-kTabDegree interpolants in the local variable s in [-1/2, 1/2] of
//   g1 = S1 / x,  g2 = S2 / x^3,  g3 = S3 / x^5
// (finite and smooth at x = 0; (S2 - S3) / x^3 = g2 - x^2 g3).  Layout: coefficients 2j and 2j + 1 of
// function f on interval i side by side at tab[((f * kTabCoef / 2 + j) * kTabIntervals + i) * 2], so
// that a lane reads a function's coefficients with kTabCoef / 2 16-byte LDS reads and the lanes of a
// wavefront, which read the same pair of different intervals, hit different LDS banks.  S1/r = g1/h
// and so on.
constexpr int kTabIntervals = 160, kTabDegree = 7, kTabCoef = kTabDegree + 1, kTabFuncs = 3;
constexpr int kTabDoubles = kTabIntervals * kTabFuncs * kTabCoef;
// Builds the table for the sorted smoothing ratios rho[3], the cut-off and the range X; returns false
// (and leaves tab empty) if its interpolation error, checked against long-double evaluations, exceeds
// 5e-14 of each function's largest value (6.5e-16 for rho = 2 : 3 : 4).  *maxerr: that error.
bool build_near_table(const double rho[3], double cutoff, double X, std::vector<double> &tab, double *maxerr);

// ---- kernel launchers (return hipSuccess or the launch error) ----
hipError_t launch_pack(const double *x, const double *nrm, const double *w, const double *f, const double *q,
                       const int64_t *perm, int64_t n, const double org[3], SrcRec<double> *rec64, SrcRec<float> *rec32,
                       Pos4<double> *pos64, Pos4<float> *pos32, hipStream_t s);

// rnear: near radius of every target; with sharp, targets with b == 0 use rsharp (<= rnear) instead
hipError_t launch_far_direct(int precision, int layers, const SrcRec<double> *rec64, const SrcRec<float> *rec32,
                             int64_t n, const EvalArgs &a, double rnear, double rsharp, int sharp, double *part,
                             hipStream_t s);
// Plain sums at targets with no closest point (sr_eval_far): the original kernels applied to f w and
// q n w with no subtraction, over every source farther than rnear; a target with a source inside rnear
// is reported in *flag (kFlagFarTarget).  Writes the same partial sums as launch_far_direct.
hipError_t launch_far_plain(int precision, int layers, const SrcRec<double> *rec64, const SrcRec<float> *rec32,
                            int64_t n, const EvalArgs &a, double rnear, NearFlag *flag, double *part, hipStream_t s);

hipError_t launch_near_finalize(int precision, int layers, const SrcRec<double> *rec64,
                                const Pos4<double> *pos64, const Pos4<float> *pos32, const int *cell_start,
                                const CellGrid &grid, const EvalArgs &a, const DevParams &p, const double *part,
                                int nparts, NearFlag *flag, hipStream_t s);
// u += far / (8 pi), v += -6 far / (8 pi) for outputs written by launch_near_finalize with nparts = 0;
// with store, u = far / (8 pi), v = -6 far / (8 pi) (the plain sums of sr_eval_far)
hipError_t launch_far_add(int layers, const double *part, int nparts, const EvalArgs &a, bool store, hipStream_t s);
// flag[0 .. n) = no report (bits 0, first = all ones)
hipError_t launch_flag_clear(NearFlag *flag, int n, hipStream_t s);

// ---- the evaluation shared by the C entry points (sr_api.hip) ----
// Checks layers (SR_SL, SR_DL or both), 0 <= m <= max_m, then the context's state; sets the thread's
// error message.
sr_status eval_check(const char *fn, sr_ctx *c, int layers, int64_t m, int64_t max_m);
// The evaluation of sr_eval on device arrays.  ext_part == nullptr: the far-field partial sums go to a
// context-owned buffer (grown as needed).  Otherwise they go to ext_part (room for kFarSplits * 6 * m
// doubles) and nothing is allocated: SR_ESTATE if the context's cell list or records would have to be
// built, SR_EINVAL for the treecode far field; profiling is then ignored.
sr_status eval_on_device(const char *fn, sr_ctx *c, int layers, int64_t m, const double *y, const double *x0,
                         const double *n0, const double *b, const double *f0, const double *q0, double *u, double *v,
                         double *u_delta, double *v_delta, hipStream_t s, double *ext_part);
// Sets the thread's error message (sr_last_error) and returns st.
sr_status set_error(sr_status st, const char *msg);
// Clears the thread's error message (every entry point starts with it).
void clear_error();
// Makes `dev` the current device and restores the caller's on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
// Resolves the address of the current device's copy of the static scratch array of the
// allocation-free evaluation (sr_noalloc.hip); called once per device by sr_create with that device
// current.  Returns the error of hipGetSymbolAddress.
hipError_t noalloc_setup(int device);
// Device ordinal of a context.
int ctx_device(const sr_ctx *c);

}  // namespace sr

// The evaluation without device allocation (sr_eval_noalloc in include/stokesreg.h).
//
// sr_eval keeps the far-field partial sums part[split][channel][target] in a context buffer that grows
// with the number of targets (hipMalloc on the first call at a larger m).  This variant writes them to
// a file-scope device array of fixed size instead, so that a call allocates nothing: it can be made
// under HIP graph capture or in a loop that must not allocate.  Every GPU the library runs on holds
// its own copy of the array (kScratchBytes) for the life of the process.  sr_create resolves the
// address of the current device's copy once (hipGetSymbolAddress) and the calls pass that address to
// the kernels; the array's name is never used as a device address in host code.
//
// The far kernel writes every partial sum that the far-sum addition reads, so the array needs no
// clearing between calls.  All calls on one GPU share its array: two such calls that overlap in time
// on one GPU (different streams or host threads, any contexts) race on it.
#include <mutex>

#include "sr_internal.h"

namespace sr {
namespace {

constexpr size_t kScratchDoubles = (size_t)kFarSplits * 6 * (size_t)SR_NOALLOC_MAX_TARGETS;
static_assert(kScratchDoubles * sizeof(double) == (size_t)SR_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};  // per device ordinal: the device address of that GPU's copy

}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<double *>(p);
    return hipSuccess;
}

}  // namespace sr

using namespace sr;

extern "C" sr_status sr_eval_noalloc(sr_ctx *c, int layers, int64_t m, const double *y, const double *x0,
                                     const double *n0, const double *b, const double *f0, const double *q0,
                                     double *u, double *v, void *stream)
{
    clear_error();
    sr_status st = eval_check("sr_eval_noalloc", c, layers, m, SR_NOALLOC_MAX_TARGETS);
    if (st != SR_OK) return st;
    if (m == 0) return SR_OK;
    if (!y || !x0 || !n0 || !b) return set_error(SR_EINVAL, "sr_eval_noalloc: NULL target array");
    if ((layers & SR_SL) && (!f0 || !u)) return set_error(SR_EINVAL, "sr_eval_noalloc: SR_SL needs f0 and u");
    if ((layers & SR_DL) && (!q0 || !v)) return set_error(SR_EINVAL, "sr_eval_noalloc: SR_DL needs q0 and v");
    const int dev = ctx_device(c);
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (dev >= 0 && dev < kMaxDevices) part = g_scratch[dev];
    }
    if (!part) return set_error(SR_ESTATE, "sr_eval_noalloc: the scratch array of this device was not resolved");
    DeviceGuard g(dev);
    if (!g.ok) return set_error(SR_ENODEV, "sr_eval_noalloc: cannot select the context's device");
    return eval_on_device("sr_eval_noalloc", c, layers, m, y, x0, n0, b, f0, q0, u, v, nullptr, nullptr,
                          (hipStream_t)stream, part);
}

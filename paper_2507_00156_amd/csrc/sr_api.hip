// C-ABI entry points of libstokesreg (declared and documented in include/stokesreg.h).
//
// Host responsibilities: argument validation, ownership of device buffers, the spatial index of the
// sources (a uniform cell grid whose side is at least the near radius cutoff * max_j delta_j, built
// by a counting sort on the host when the surface or the radius changes), and kernel launches on the
// caller's stream.  All arithmetic of the method runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sr_internal.h"
#include "sr_tree.h"

using namespace sr;

namespace {

thread_local std::string g_err;

sr_status fail(sr_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define SR_HIP(call)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(e_ == hipErrorOutOfMemory ? SR_ENOMEM : SR_EHIP, "%s failed: %s", #call,     \
                        hipGetErrorString(e_));                                                      \
    } while (0)

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;  // elements
    hipError_t reserve(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
        if (e == hipSuccess) cap = n;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

bool is_pos_finite(double v) { return std::isfinite(v) && v > 0.0; }

// Host smoothing tables by parameter set (rho, cutoff, range), shared by the contexts of the process:
// building and checking one takes tens of milliseconds on the host, and the rigid-sphere solve makes
// new contexts with the same parameters for every new geometry.  Failed checks are kept as well.
struct NearTableEntry {
    double key[5];
    bool ok;
    std::vector<double> tab;
};
std::mutex g_tab_mu;
std::vector<NearTableEntry> g_tab_cache;
constexpr size_t kTabCacheMax = 32;

bool near_table_cached(const double key[5], const double rho[3], double cutoff, double X, std::vector<double> &out)
{
    std::lock_guard<std::mutex> lock(g_tab_mu);
    for (const NearTableEntry &e : g_tab_cache)
        if (std::equal(key, key + 5, e.key)) {
            out = e.tab;
            return e.ok;
        }
    NearTableEntry e;
    std::copy(key, key + 5, e.key);
    double err = 0.0;
    e.ok = build_near_table(rho, cutoff, X, e.tab, &err);
    out = e.tab;
    const bool ok = e.ok;
    if (g_tab_cache.size() >= kTabCacheMax) g_tab_cache.erase(g_tab_cache.begin());
    g_tab_cache.push_back(std::move(e));
    return ok;
}

}  // namespace

struct sr_ctx {
    int device = 0;
    sr_params prm{};
    bool have_params = false;

    int64_t n = 0;
    bool have_surface = false, have_sl = false, have_dl = false;
    std::vector<double> hx;  // host copy of the points (caller order), for the spatial index

    DevBuf<double> x, nrm, w, f, q;  // caller order
    DevBuf<int64_t> perm;            // sorted record i <- caller index perm[i]
    DevBuf<int> cell_start;
    DevBuf<SrcRec<double>> rec64;
    DevBuf<SrcRec<float>> rec32;
    DevBuf<Pos4<double>> pos64;
    DevBuf<Pos4<float>> pos32;
    DevBuf<double> part;  // far-field partial sums
    DevBuf<FrontierRec> t_front;
    DevBuf<double> stage;  // device copies of the caller's host arrays (SR_HOST)
    // smoothing table of the targets on the surface (NearTable), built for tab_key = (sorted rho,
    // cutoff, range); tab_ok false when its check failed (the kernels then use the closed forms)
    DevBuf<double> near_tab;
    std::vector<double> near_tab_host;
    double tab_key[5] = {-1.0, -1.0, -1.0, -1.0, -1.0};
    bool tab_ok = false;
    NearFlag *flag = nullptr;     // target-consistency report (sr_check), device memory
    double extent = 0.0;          // max over the points of max_d |x_d - org_d|

    CellGrid grid{};
    double grid_rnear = -1.0;
    int grid_precision = -1;  // the precision the grid's margin was sized for
    double org[3] = {0.0, 0.0, 0.0};  // centre of the points' bounding box: origin of the FP32 coordinates
    bool layout_dirty = true, pack_dirty = true;

    // treecode far field
    TreeHost tree;
    bool tree_dirty = true, tree_weights_dirty = true;
    int tree_p = -1;
    int64_t tree_leaf = -1;
    DevBuf<TreeNode> t_nodes;
    DevBuf<int> t_item_node, t_item_begin, t_item_end, t_node_item0, t_idx_in, t_order;
    DevBuf<int64_t> t_perm;
    DevBuf<SrcRec<double>> t_rec64;
    DevBuf<SrcRec<float>> t_rec32;
    DevBuf<ProxRec<double>> t_prox64;
    DevBuf<ProxRec<float>> t_prox32;
    DevBuf<double> t_partial;
    DevBuf<uint32_t> t_key_in, t_key_out;
    DevBuf<int> t_order_near;  // the near field's target order when the treecode has its own
    DevBuf<char> t_sort_tmp;
    TreeDev tdev;

    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;     // created events, reused
    std::vector<hipEvent_t> ev_recorded; // 3 per profiled evaluation: start, far done, near done

    // concurrent evaluation: the near-field kernel runs on this stream (default priority,
    // non-blocking) while the far field runs on the caller's; fork and join events order the two.
    // Created by sr_create.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    ~sr_ctx()
    {
        x.release();
        nrm.release();
        w.release();
        f.release();
        q.release();
        perm.release();
        cell_start.release();
        rec64.release();
        rec32.release();
        pos64.release();
        pos32.release();
        part.release();
        t_front.release();
        stage.release();
        if (flag) (void)hipFree(flag);
        t_nodes.release();
        t_item_node.release();
        t_item_begin.release();
        t_item_end.release();
        t_node_item0.release();
        t_idx_in.release();
        t_order.release();
        t_perm.release();
        t_rec64.release();
        t_rec32.release();
        t_prox64.release();
        t_prox32.release();
        t_partial.release();
        t_key_in.release();
        t_key_out.release();
        t_sort_tmp.release();
        t_order_near.release();
        near_tab.release();
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_recorded) (void)hipEventDestroy(e);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace {

double near_radius(const sr_params &p)
{
    double r = std::max(p.rho[0], std::max(p.rho[1], p.rho[2]));
    if (p.surface_sharp) r = std::max(r, p.sharp_rho);
    return p.cutoff * r * p.h;
}

// The reach of a near radius: every pair that the near test calls near is truly closer than it.  The
// single-precision test rounds each coordinate relative to org (error <= 2^-24 |x - org| per
// coordinate, and as much again in the difference and the sum of squares), so the margin grows with
// the extent E of the points: 4 * 2^-24 * (2 E + rnear) on the mixed path, plus a relative 1e-5.
double reach_of(const sr_ctx *c, double radius, double rnear)
{
    double r = radius * (1.0 + 1e-5);
    if (c->prm.precision == SR_MIXED) r += 4.0 * std::ldexp(1.0, -24) * (2.0 * c->extent + rnear);
    return r;
}

// The radius the treecode's MAC requires a cluster to lie beyond (launch_tree_far)
double tree_mac_radius(const sr_ctx *c, double rnear)
{
    return c->prm.precision == SR_MIXED ? reach_of(c, rnear, rnear) : rnear;
}

// Uniform grid of cells of side reach / kCellsPerReach (larger only when the grid would exceed
// kMaxCells cells); sources sorted by cell with a stable counting sort.
sr_status build_layout(sr_ctx *c, hipStream_t s)
{
    const double rnear = near_radius(c->prm);
    const int64_t n = c->n;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], c->hx[3 * i + d]);
            hi[d] = std::max(hi[d], c->hx[3 * i + d]);
        }
    double side = reach_of(c, rnear, rnear) / kCellsPerReach;
    const int64_t kMaxCells = int64_t(1) << 22;
    int g[3];
    for (;;) {
        int64_t tot = 1;
        for (int d = 0; d < 3; ++d) {
            g[d] = (int)std::max<double>(1.0, std::floor((hi[d] - lo[d]) / side) + 1.0);
            tot *= g[d];
        }
        if (tot <= kMaxCells) break;
        side *= 1.25;
    }
    const double inv_side = 1.0 / side;
    const int64_t ncell = (int64_t)g[0] * g[1] * g[2];
    std::vector<int> key(n);
    std::vector<int> start(ncell + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        int ic[3];
        for (int d = 0; d < 3; ++d) {
            double u = std::floor((c->hx[3 * i + d] - lo[d]) * inv_side);
            ic[d] = (int)std::min<double>(std::max(u, 0.0), g[d] - 1);
        }
        key[i] = (ic[0] * g[1] + ic[1]) * g[2] + ic[2];
        start[key[i] + 1]++;
    }
    for (int64_t k = 0; k < ncell; ++k) start[k + 1] += start[k];
    std::vector<int64_t> perm(n);
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i) perm[fill[key[i]]++] = i;
    }
    SR_HIP(c->perm.reserve(n));
    SR_HIP(c->cell_start.reserve(ncell + 1));
    SR_HIP(hipMemcpyAsync(c->perm.p, perm.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    SR_HIP(hipMemcpyAsync(c->cell_start.p, start.data(), (ncell + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    // the host vectors die at return: wait for the copies
    SR_HIP(hipStreamSynchronize(s));
    for (int d = 0; d < 3; ++d) {
        c->grid.lo[d] = lo[d];
        c->grid.g[d] = g[d];
    }
    c->grid.side = side;
    c->grid.inv_side = inv_side;
    c->grid_rnear = rnear;
    c->grid_precision = c->prm.precision;
    c->layout_dirty = false;
    c->pack_dirty = true;
    return SR_OK;
}

sr_status ensure_packed(sr_ctx *c, hipStream_t s)
{
    if (c->layout_dirty || c->grid_rnear != near_radius(c->prm) || c->grid_precision != c->prm.precision) {
        sr_status st = build_layout(c, s);
        if (st != SR_OK) return st;
    }
    if (c->pack_dirty) {
        SR_HIP(c->rec64.reserve(c->n));
        SR_HIP(c->rec32.reserve(c->n));
        SR_HIP(c->pos64.reserve(c->n));
        SR_HIP(c->pos32.reserve(c->n));
        SR_HIP(launch_pack(c->x.p, c->nrm.p, c->w.p, c->have_sl ? c->f.p : nullptr, c->have_dl ? c->q.p : nullptr,
                           c->perm.p, c->n, c->org, c->rec64.p, c->rec32.p, c->pos64.p, c->pos32.p, s));
        c->pack_dirty = false;
    }
    return SR_OK;
}

// Octree, proxy points and tree-ordered records for the treecode far field; modified weights when a
// density changed.
sr_status ensure_tree(sr_ctx *c, hipStream_t s)
{
    const int p = c->prm.tree_degree;
    const int64_t leaf = c->prm.tree_leaf;
    if (c->tree_dirty || c->tree_p != p || c->tree_leaf != leaf) {
        TreeHost &T = c->tree;
        build_tree(c->hx.data(), c->n, leaf, p, T);
        const int nn = (int)T.nodes.size(), np1 = p + 1, nprox = np1 * np1 * np1, ni = (int)T.item_node.size();
        SR_HIP(c->t_nodes.reserve(nn));
        SR_HIP(c->t_item_node.reserve(ni));
        SR_HIP(c->t_item_begin.reserve(ni));
        SR_HIP(c->t_item_end.reserve(ni));
        SR_HIP(c->t_node_item0.reserve(nn + 1));
        SR_HIP(c->t_perm.reserve(c->n));
        SR_HIP(c->t_rec64.reserve(c->n));
        SR_HIP(c->t_rec32.reserve(c->n));
        SR_HIP(c->t_prox64.reserve((size_t)nn * nprox));
        SR_HIP(c->t_prox32.reserve((size_t)nn * nprox));
        SR_HIP(c->t_partial.reserve((size_t)ni * nprox * 16));
        std::vector<ProxRec<double>> p64((size_t)nn * nprox);
        std::vector<ProxRec<float>> p32((size_t)nn * nprox);
        for (size_t k = 0; k < p64.size(); ++k) {
            p64[k] = ProxRec<double>{};
            p32[k] = ProxRec<float>{};
            p64[k].x = T.proxy_xyz[3 * k];
            p64[k].y = T.proxy_xyz[3 * k + 1];
            p64[k].z = T.proxy_xyz[3 * k + 2];
            p32[k].x = (float)(p64[k].x - c->org[0]);
            p32[k].y = (float)(p64[k].y - c->org[1]);
            p32[k].z = (float)(p64[k].z - c->org[2]);
        }
        SR_HIP(hipMemcpyAsync(c->t_nodes.p, T.nodes.data(), nn * sizeof(TreeNode), hipMemcpyHostToDevice, s));
        SR_HIP(hipMemcpyAsync(c->t_item_node.p, T.item_node.data(), ni * sizeof(int), hipMemcpyHostToDevice, s));
        SR_HIP(hipMemcpyAsync(c->t_item_begin.p, T.item_begin.data(), ni * sizeof(int), hipMemcpyHostToDevice, s));
        SR_HIP(hipMemcpyAsync(c->t_item_end.p, T.item_end.data(), ni * sizeof(int), hipMemcpyHostToDevice, s));
        SR_HIP(hipMemcpyAsync(c->t_node_item0.p, T.node_item0.data(), (nn + 1) * sizeof(int), hipMemcpyHostToDevice,
                              s));
        SR_HIP(hipMemcpyAsync(c->t_perm.p, T.order.data(), c->n * sizeof(int64_t), hipMemcpyHostToDevice, s));
        SR_HIP(c->t_front.reserve(T.front.size()));
        SR_HIP(hipMemcpyAsync(c->t_front.p, T.front.data(), T.front.size() * sizeof(FrontierRec),
                              hipMemcpyHostToDevice, s));
        SR_HIP(hipMemcpyAsync(c->t_prox64.p, p64.data(), p64.size() * sizeof(ProxRec<double>), hipMemcpyHostToDevice,
                              s));
        SR_HIP(hipMemcpyAsync(c->t_prox32.p, p32.data(), p32.size() * sizeof(ProxRec<float>), hipMemcpyHostToDevice,
                              s));
        SR_HIP(hipStreamSynchronize(s));  // host staging vectors die at return
        TreeDev &D = c->tdev;
        D.nodes = c->t_nodes.p;
        D.item_node = c->t_item_node.p;
        D.item_begin = c->t_item_begin.p;
        D.item_end = c->t_item_end.p;
        D.node_item0 = c->t_node_item0.p;
        D.trec64 = c->t_rec64.p;
        D.trec32 = c->t_rec32.p;
        D.prox64 = c->t_prox64.p;
        D.prox32 = c->t_prox32.p;
        D.nnodes = nn;
        D.nitems = ni;
        D.nprox = nprox;
        D.p = p;
        D.stack_cap = 7 * T.depth + 2;
        D.front = c->t_front.p;
        D.nfront = (int)T.front.size();
        c->tree_p = p;
        c->tree_leaf = leaf;
        c->tree_dirty = false;
        c->tree_weights_dirty = true;
    }
    if (c->tree_weights_dirty) {
        SR_HIP(launch_pack(c->x.p, c->nrm.p, c->w.p, c->have_sl ? c->f.p : nullptr, c->have_dl ? c->q.p : nullptr,
                           c->t_perm.p, c->n, c->org, c->t_rec64.p, c->t_rec32.p, nullptr, nullptr, s));
        SR_HIP(launch_anterp(c->tdev, c->tree.cosk.data(), c->t_partial.p, s));
        c->tree_weights_dirty = false;
    }
    return SR_OK;
}

sr_status record_event(sr_ctx *c, hipStream_t s)
{
    hipEvent_t e;
    if (!c->ev_pool.empty()) {
        e = c->ev_pool.back();
        c->ev_pool.pop_back();
    } else {
        SR_HIP(hipEventCreate(&e));
    }
    c->ev_recorded.push_back(e);
    SR_HIP(hipEventRecord(e, s));
    return SR_OK;
}

}  // namespace

extern "C" {

void sr_default_params(sr_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->h = 0.0;
    p->rho[0] = 2.0;
    p->rho[1] = 3.0;
    p->rho[2] = 4.0;
    p->cutoff = 6.0;
    p->precision = SR_FP64;
    p->far_method = SR_DIRECT;
    p->tree_degree = 8;
    p->tree_theta = 0.7;
    p->tree_leaf = 2000;
    p->surface_sharp = 0;
    p->sharp_rho = 3.0;
}

const char *sr_last_error(void) { return g_err.c_str(); }

const char *sr_version(void) { return "stokesreg 0.1 (gfx950)"; }

sr_status sr_create(sr_ctx **out, int device)
{
    g_err.clear();
    if (!out) return fail(SR_EINVAL, "sr_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(SR_ENODEV, "sr_create: no HIP device available");
    if (device < 0 || device >= count)
        return fail(SR_ENODEV, "sr_create: device %d does not exist (%d devices)", device, count);
    sr_ctx *c = new (std::nothrow) sr_ctx();
    if (!c) return fail(SR_ENOMEM, "sr_create: out of host memory");
    c->device = device;
    sr_default_params(&c->prm);
    {
        // the near-field stream of the concurrent evaluation and its fork and join events
        DeviceGuard g(device);
        hipError_t e = g.ok ? hipSuccess : hipErrorInvalidDevice;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) {
            delete c;
            return fail(SR_EHIP, "sr_create: stream or event creation failed: %s", hipGetErrorString(e));
        }
        // the address of this device's static scratch array (sr_eval_noalloc), resolved once per device
        e = noalloc_setup(device);
        if (e != hipSuccess) {
            delete c;
            return fail(SR_EHIP, "sr_create: cannot resolve the static scratch array: %s", hipGetErrorString(e));
        }
        // the target-consistency report, cleared
        e = hipMalloc((void **)&c->flag, kFlagSlots * sizeof(NearFlag));
        if (e == hipSuccess) e = launch_flag_clear(c->flag, kFlagSlots, c->side);
        if (e == hipSuccess) e = hipStreamSynchronize(c->side);
        if (e != hipSuccess) {
            delete c;
            return fail(e == hipErrorOutOfMemory ? SR_ENOMEM : SR_EHIP, "sr_create: %s", hipGetErrorString(e));
        }
    }
    *out = c;
    return SR_OK;
}

sr_status sr_destroy(sr_ctx *c)
{
    g_err.clear();
    if (!c) return SR_OK;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        delete c;
    }
    return SR_OK;
}

sr_status sr_set_params(sr_ctx *c, const sr_params *p)
{
    g_err.clear();
    if (!c || !p) return fail(SR_EINVAL, "sr_set_params: NULL argument");
    if (!is_pos_finite(p->h)) return fail(SR_EINVAL, "sr_set_params: h must be positive and finite");
    for (int j = 0; j < 3; ++j)
        if (!is_pos_finite(p->rho[j])) return fail(SR_EINVAL, "sr_set_params: rho[%d] must be positive", j);
    if (p->rho[0] == p->rho[1] || p->rho[0] == p->rho[2] || p->rho[1] == p->rho[2])
        return fail(SR_EINVAL, "sr_set_params: the three rho must be distinct");
    if (!is_pos_finite(p->cutoff)) return fail(SR_EINVAL, "sr_set_params: cutoff must be positive");
    if (p->precision != SR_FP64 && p->precision != SR_MIXED)
        return fail(SR_EINVAL, "sr_set_params: precision must be SR_FP64 or SR_MIXED");
    if (p->far_method != SR_DIRECT && p->far_method != SR_TREE)
        return fail(SR_EINVAL, "sr_set_params: far_method must be SR_DIRECT or SR_TREE");
    if (p->far_method == SR_TREE) {
        if (p->tree_degree < 1 || p->tree_degree > 16)
            return fail(SR_EINVAL, "sr_set_params: tree_degree must be in 1..16");
        if (!(p->tree_theta >= 0.0 && p->tree_theta < 1.0))
            return fail(SR_EINVAL, "sr_set_params: tree_theta must be in [0, 1)");
        if (p->tree_leaf < 1) return fail(SR_EINVAL, "sr_set_params: tree_leaf must be >= 1");
    }
    if (p->surface_sharp != 0 && p->surface_sharp != 1)
        return fail(SR_EINVAL, "sr_set_params: surface_sharp must be 0 or 1");
    if (p->surface_sharp && !is_pos_finite(p->sharp_rho))
        return fail(SR_EINVAL, "sr_set_params: sharp_rho must be positive");
    c->prm = *p;
    c->have_params = true;
    return SR_OK;
}

sr_status sr_set_surface(sr_ctx *c, int64_t n, const double *x, const double *nrm, const double *w, void *stream)
{
    g_err.clear();
    if (!c) return fail(SR_EINVAL, "sr_set_surface: ctx is NULL");
    if (n < 1 || n > kMaxTargets)
        return fail(SR_EINVAL, "sr_set_surface: n = %lld out of range (1..%lld)", (long long)n, (long long)kMaxTargets);
    if (!x || !nrm || !w) return fail(SR_EINVAL, "sr_set_surface: NULL array");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(SR_ENODEV, "sr_set_surface: cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> hx(3 * n), hn(3 * n), hw(n);
    SR_HIP(hipMemcpyAsync(hx.data(), x, 3 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    SR_HIP(hipMemcpyAsync(hn.data(), nrm, 3 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    SR_HIP(hipMemcpyAsync(hw.data(), w, n * sizeof(double), hipMemcpyDeviceToHost, s));
    SR_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(hw[i]) || hw[i] < 0.0)
            return fail(SR_EINVAL, "sr_set_surface: weight %lld is negative or not finite", (long long)i);
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(hx[3 * i + d]) || !std::isfinite(hn[3 * i + d]))
                return fail(SR_EINVAL, "sr_set_surface: point or normal %lld not finite", (long long)i);
    }
    SR_HIP(c->x.reserve(3 * n));
    SR_HIP(c->nrm.reserve(3 * n));
    SR_HIP(c->w.reserve(n));
    SR_HIP(hipMemcpyAsync(c->x.p, x, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    SR_HIP(hipMemcpyAsync(c->nrm.p, nrm, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    SR_HIP(hipMemcpyAsync(c->w.p, w, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    c->n = n;
    c->extent = 0.0;
    for (int d = 0; d < 3; ++d) {
        double lo = hx[d], hi = hx[d];
        for (int64_t i = 1; i < n; ++i) {
            lo = std::min(lo, hx[3 * i + d]);
            hi = std::max(hi, hx[3 * i + d]);
        }
        c->org[d] = 0.5 * (lo + hi);
        c->extent = std::max(c->extent, 0.5 * (hi - lo));
    }
    c->hx.swap(hx);
    c->have_surface = true;
    c->have_sl = c->have_dl = false;
    c->layout_dirty = true;
    c->pack_dirty = true;
    c->tree_dirty = true;
    return SR_OK;
}

sr_status sr_set_density(sr_ctx *c, int layer, const double *dens, void *stream)
{
    g_err.clear();
    if (!c || !dens) return fail(SR_EINVAL, "sr_set_density: NULL argument");
    if (layer != SR_SL && layer != SR_DL) return fail(SR_EINVAL, "sr_set_density: layer must be SR_SL or SR_DL");
    if (!c->have_surface) return fail(SR_ESTATE, "sr_set_density: set the surface first");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(SR_ENODEV, "sr_set_density: cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    DevBuf<double> &dst = layer == SR_SL ? c->f : c->q;
    SR_HIP(dst.reserve(3 * c->n));
    SR_HIP(hipMemcpyAsync(dst.p, dens, 3 * c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (layer == SR_SL)
        c->have_sl = true;
    else
        c->have_dl = true;
    c->pack_dirty = true;
    c->tree_weights_dirty = true;
    return SR_OK;
}

}  // extern "C"

namespace {

// One chunk of at most kTargetChunk targets of eval_on_device; its consistency reports go to *flag.
sr_status eval_chunk(const char *fn, sr_ctx *c, int layers, int64_t m, const double *y, const double *x0,
                     const double *n0, const double *b, const double *f0, const double *q0, double *u, double *v,
                     double *u_delta, double *v_delta, hipStream_t s, double *ext_part, NearFlag *flag)
{
    sr_status st;
    const bool noalloc = ext_part != nullptr;
    if (noalloc) {
        if (c->prm.far_method == SR_TREE) return fail(SR_EINVAL, "%s: the treecode far field is not supported", fn);
        if (c->layout_dirty || c->grid_rnear != near_radius(c->prm) || c->grid_precision != c->prm.precision ||
            c->rec64.cap < (size_t)c->n)
            return fail(SR_ESTATE, "%s: the context's cell list and records are not built for the current surface "
                                   "and parameters (one sr_eval call builds them)", fn);
        if (c->pack_dirty) {
            // densities changed: repack into the existing records (no allocation)
            SR_HIP(launch_pack(c->x.p, c->nrm.p, c->w.p, c->have_sl ? c->f.p : nullptr,
                               c->have_dl ? c->q.p : nullptr, c->perm.p, c->n, c->org, c->rec64.p, c->rec32.p,
                               c->pos64.p, c->pos32.p, s));
            c->pack_dirty = false;
        }
    } else if ((st = ensure_packed(c, s)) != SR_OK) {
        return st;
    }

    EvalArgs a{};
    a.layers = layers;
    a.m = m;
    a.y = y;
    a.x0 = x0;
    a.n0 = n0;
    a.b = b;
    a.f0 = f0;
    a.q0 = q0;
    a.u = u;
    a.v = v;
    for (int d = 0; d < 3; ++d) a.org[d] = c->prm.precision == SR_MIXED ? c->org[d] : 0.0;
    a.u_delta = u_delta;
    a.v_delta = v_delta;

    DevParams dp{};
    dp.h = c->prm.h;
    int ord[3] = {0, 1, 2};
    std::sort(ord, ord + 3, [&](int i, int j) { return c->prm.rho[i] < c->prm.rho[j]; });
    for (int o = 0; o < 3; ++o) {
        dp.ord[o] = ord[o];
        dp.rho[o] = c->prm.rho[ord[o]];
        dp.inv_delta[o] = 1.0 / (dp.rho[o] * c->prm.h);
    }
    dp.cutoff = c->prm.cutoff;
    dp.rnear = c->grid_rnear;
    // a far-rule target (|b| >= cutoff * max delta) with a source closer than cutoff * max delta, less
    // the near test's rounding (relative 1e-4 on the mixed path's single-precision squared distance,
    // 1e-9 in double precision), is reported
    dp.rflag = c->prm.cutoff * dp.rho[2] * c->prm.h * (c->prm.precision == SR_MIXED ? 1.0 - 1e-4 : 1.0 - 1e-9);
    dp.precision = c->prm.precision;
    dp.pow234 = (2.0 * dp.rho[1] == 3.0 * dp.rho[0] && dp.rho[2] == 2.0 * dp.rho[0]) ? 1 : 0;
    dp.sharp = c->prm.surface_sharp ? 1 : 0;
    dp.inv_dsharp = 1.0 / (c->prm.sharp_rho * c->prm.h);
    dp.rsharp = dp.sharp ? std::min(dp.rnear, c->prm.cutoff * c->prm.sharp_rho * c->prm.h) : dp.rnear;
    dp.reach = reach_of(c, dp.rnear, dp.rnear);
    dp.reach_sharp = reach_of(c, dp.rsharp, dp.rnear);
    dp.ih = 1.0 / c->prm.h;
    dp.ih3 = dp.ih * dp.ih * dp.ih;
    dp.ih5 = dp.ih3 * dp.ih * dp.ih;
    dp.tab = nullptr;
    if (!u_delta && !v_delta && !dp.sharp) {
        // the table covers r / h up to the near radius (and a little beyond, for the rounding of the
        // pair test); built on the first evaluation with these parameters (not by the allocation-free
        // call, which then uses the closed forms)
        const double X = dp.rnear / c->prm.h * (1.0 + 1e-5);
        const double key[5] = {dp.rho[0], dp.rho[1], dp.rho[2], dp.cutoff, X};
        const bool same = std::equal(key, key + 5, c->tab_key);
        if (!same && !noalloc) {
            c->tab_ok = near_table_cached(key, dp.rho, dp.cutoff, X, c->near_tab_host);
            std::copy(key, key + 5, c->tab_key);
            if (c->tab_ok) {
                // synchronized: the host copy may be rebuilt by the next call with other parameters
                SR_HIP(c->near_tab.reserve(kTabDoubles));
                SR_HIP(hipMemcpyAsync(c->near_tab.p, c->near_tab_host.data(), kTabDoubles * sizeof(double),
                                      hipMemcpyHostToDevice, s));
                SR_HIP(hipStreamSynchronize(s));
            }
        }
        if (std::equal(key, key + 5, c->tab_key) && c->tab_ok) {
            dp.tab = c->near_tab.p;
            dp.tab_scale = kTabIntervals / (X * c->prm.h);
        }
    }

    const bool tree = c->prm.far_method == SR_TREE;
    int nparts = kFarSplits;
    if (tree && (st = ensure_tree(c, s)) != SR_OK) return st;
    // A Morton order of the targets, those on the surface first (DevParams::order): the treecode walks
    // in it and the near-field kernel takes the targets in it.  Not made by the allocation-free call
    // (the caller's order).
    const bool order = tree || !noalloc;
    dp.order = nullptr;
    if (order) {
        TreeDev &D = c->tdev;
        SR_HIP(c->t_key_in.reserve(m));
        SR_HIP(c->t_key_out.reserve(m));
        SR_HIP(c->t_idx_in.reserve(m));
        SR_HIP(c->t_order.reserve(m));
        const size_t tb = target_sort_tmp_bytes((int)m);
        SR_HIP(c->t_sort_tmp.reserve(tb));
        D.key_in = c->t_key_in.p;
        D.key_out = c->t_key_out.p;
        D.idx_in = c->t_idx_in.p;
        D.order = c->t_order.p;
        D.sort_tmp = c->t_sort_tmp.p;
        D.sort_tmp_bytes = c->t_sort_tmp.cap;
        dp.order = D.order;
        if (tree) {
            SR_HIP(c->t_order_near.reserve(m));
            dp.order = c->t_order_near.p;
        }
    }
    if (tree) nparts = c->tdev.nfront;
    // Morton box: the treecode's root box, or the cell grid's, widened by the near radius
    double mlo[3], mext = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (tree) {
            const TreeNode &root = c->tree.nodes[0];
            mlo[d] = root.lo[d] - dp.rnear;
            mext = std::max(mext, root.hi[d] - root.lo[d] + 2.0 * dp.rnear);
        } else {
            mlo[d] = c->grid.lo[d] - dp.rnear;
            mext = std::max(mext, c->grid.g[d] * c->grid.side + 2.0 * dp.rnear);
        }
    }
    double *part;
    if (noalloc) {
        part = ext_part;
    } else {
        SR_HIP(c->part.reserve((size_t)nparts * 6 * (size_t)m));
        part = c->part.p;
    }
    // Without per-delta outputs and without profiling, the near-field kernel (near sums,
    // extrapolation, jump term) runs on the side stream concurrently with the far field, and
    // launch_far_add then adds the far sum on the caller's stream.  Both kernels are bound by vector
    // ALU issue but stall differently, and the near kernel's short one-target wavefronts fill the
    // issue cycles and the wave slots the far kernel leaves (8.5% less time at the 42k-source
    // ellipsoid).  With profiling on, the phases run one after the other so that each has its own
    // time (the no-alloc variant records no events: it runs the phases concurrently).
    const bool profile = c->profiling && !noalloc;
    const bool concurrent = !profile && !u_delta && !v_delta;
    // the target order (1024 steps per axis) before both phases, which read it; the treecode walks in
    // plain Morton order (its workgroups map XCD-aware onto contiguous shares of it: 14.1 against
    // 18.5 ms at the h = 1/128 ellipsoid with the surface targets first), the near field takes the
    // surface targets first
    if (order) {
        if (tree) {
            SR_HIP(launch_target_order(y, nullptr, (int)m, mlo, 1024.0 / mext, c->tdev, s));
            TreeDev Dn = c->tdev;
            Dn.order = c->t_order_near.p;
            SR_HIP(launch_target_order(y, b, (int)m, mlo, 1024.0 / mext, Dn, s));
        } else {
            SR_HIP(launch_target_order(y, b, (int)m, mlo, 1024.0 / mext, c->tdev, s));
        }
    }
    if (concurrent) SR_HIP(hipEventRecord(c->ev_fork, s));
    if (profile && (st = record_event(c, s)) != SR_OK) return st;
    if (tree) {
        SR_HIP(launch_tree_far(c->prm.precision, layers, c->tdev, a, c->prm.tree_theta, dp.rnear,
                               tree_mac_radius(c, dp.rnear), dp.rsharp, dp.sharp,
                               part, s));
    } else {
        SR_HIP(launch_far_direct(c->prm.precision, layers, c->rec64.p, c->rec32.p, c->n, a, dp.rnear, dp.rsharp,
                                 dp.sharp, part, s));
    }
    if (concurrent) {
        // the side stream starts after everything the caller enqueued before this call (fork) and
        // the caller's stream continues after the near kernel (join), whatever the launches return
        hipError_t e0 = hipStreamWaitEvent(c->side, c->ev_fork, 0);
        hipError_t e1 = e0 == hipSuccess
                            ? launch_near_finalize(c->prm.precision, layers, c->rec64.p, c->pos64.p, c->pos32.p,
                                                   c->cell_start.p, c->grid, a, dp, nullptr, 0, flag, c->side)
                            : e0;
        hipError_t e2 = hipEventRecord(c->ev_join, c->side);
        hipError_t e3 = hipStreamWaitEvent(s, c->ev_join, 0);
        for (hipError_t e : {e0, e1, e2, e3})
            if (e != hipSuccess) return fail(SR_EHIP, "%s: %s", fn, hipGetErrorString(e));
        SR_HIP(launch_far_add(layers, part, nparts, a, false, s));
        return SR_OK;
    }
    if (profile && (st = record_event(c, s)) != SR_OK) return st;
    SR_HIP(launch_near_finalize(c->prm.precision, layers, c->rec64.p, c->pos64.p, c->pos32.p, c->cell_start.p,
                                c->grid, a, dp, part, nparts, flag, s));
    if (profile && (st = record_event(c, s)) != SR_OK) return st;
    return SR_OK;
}

}  // namespace

// The evaluation on device arrays (sr::eval_on_device in sr_internal.h): chunks of at most kTargetChunk
// targets one after the other, so that the far-field partial sums (768 bytes per target) and the target
// order stay bounded whatever m is; chunk i reports to the context's flag slot i.
sr_status sr::eval_on_device(const char *fn, sr_ctx *c, int layers, int64_t m, const double *y, const double *x0,
                             const double *n0, const double *b, const double *f0, const double *q0, double *u,
                             double *v, double *u_delta, double *v_delta, hipStream_t s, double *ext_part)
{
    auto at = [](auto *p, int64_t k) { return p ? p + k : p; };
    for (int64_t c0 = 0, i = 0; c0 < m; c0 += kTargetChunk, ++i) {
        const int64_t mc = std::min<int64_t>(kTargetChunk, m - c0);
        const sr_status st =
            eval_chunk(fn, c, layers, mc, at(y, 3 * c0), at(x0, 3 * c0), at(n0, 3 * c0), at(b, c0), at(f0, 3 * c0),
                       at(q0, 3 * c0), at(u, 3 * c0), at(v, 3 * c0), at(u_delta, 9 * c0), at(v_delta, 9 * c0), s,
                       ext_part, c->flag + i);
        if (st != SR_OK) return st;
    }
    return SR_OK;
}

// Validation shared by the evaluation entry points: argument checks first (so that they can be tested
// without a context), then the context's state.
sr_status sr::eval_check(const char *fn, sr_ctx *c, int layers, int64_t m, int64_t max_m)
{
    if (layers != SR_SL && layers != SR_DL && layers != (SR_SL | SR_DL))
        return fail(SR_EINVAL, "%s: layers must be SR_SL, SR_DL or both (with SR_HOST where accepted)", fn);
    if (m < 0 || m > max_m)
        return fail(SR_EINVAL, "%s: m = %lld out of range (0..%lld)", fn, (long long)m, (long long)max_m);
    if (!c) return fail(SR_EINVAL, "%s: ctx is NULL", fn);
    if (!c->have_params) return fail(SR_ESTATE, "%s: parameters not set", fn);
    if (!c->have_surface) return fail(SR_ESTATE, "%s: surface not set", fn);
    if ((layers & SR_SL) && !c->have_sl) return fail(SR_ESTATE, "%s: single-layer density not set", fn);
    if ((layers & SR_DL) && !c->have_dl) return fail(SR_ESTATE, "%s: double-layer density not set", fn);
    return SR_OK;
}

sr_status sr::set_error(sr_status st, const char *msg)
{
    return fail(st, "%s", msg);
}

void sr::clear_error() { g_err.clear(); }

int sr::ctx_device(const sr_ctx *c) { return c->device; }

extern "C" {

// Host arrays of an SR_HOST call: device copies in the context's staging buffer, in the order given;
// outputs are copied back by stage_out.
struct Staged {
    const double *src;
    double **dst;
    size_t count;
    bool in;
};

static sr_status stage_in(const char *fn, sr_ctx *c, std::vector<Staged> &arr, hipStream_t s)
{
    size_t tot = 0;
    for (const Staged &a : arr)
        if (a.src) tot += a.count;
    SR_HIP(c->stage.reserve(tot));
    size_t off = 0;
    for (Staged &a : arr) {
        if (!a.src) {
            *a.dst = nullptr;
            continue;
        }
        *a.dst = c->stage.p + off;
        if (a.in) SR_HIP(hipMemcpyAsync(*a.dst, a.src, a.count * sizeof(double), hipMemcpyHostToDevice, s));
        off += a.count;
    }
    (void)fn;
    return SR_OK;
}

static sr_status stage_out(sr_ctx *c, const std::vector<Staged> &arr, hipStream_t s)
{
    (void)c;
    for (const Staged &a : arr)
        if (a.src && !a.in)
            SR_HIP(hipMemcpyAsync((void *)a.src, *a.dst, a.count * sizeof(double), hipMemcpyDeviceToHost, s));
    SR_HIP(hipStreamSynchronize(s));
    return SR_OK;
}

sr_status sr_eval(sr_ctx *c, int layers, int64_t m, const double *y, const double *x0, const double *n0,
                  const double *b, const double *f0, const double *q0, double *u, double *v, double *u_delta,
                  double *v_delta, void *stream)
{
    g_err.clear();
    const bool host = (layers & SR_HOST) != 0;
    layers &= ~SR_HOST;
    sr_status st = eval_check("sr_eval", c, layers, m, kMaxTargets);
    if (st != SR_OK) return st;
    if (m == 0) return SR_OK;
    if (!y || !x0 || !n0 || !b) return fail(SR_EINVAL, "sr_eval: NULL target array");
    if ((layers & SR_SL) && (!f0 || !u)) return fail(SR_EINVAL, "sr_eval: SR_SL needs f0 and u");
    if ((layers & SR_DL) && (!q0 || !v)) return fail(SR_EINVAL, "sr_eval: SR_DL needs q0 and v");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(SR_ENODEV, "sr_eval: cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    if (!host) return eval_on_device("sr_eval", c, layers, m, y, x0, n0, b, f0, q0, u, v, u_delta, v_delta, s, nullptr);

    const size_t m3 = 3 * (size_t)m;
    const double *dy, *dx0, *dn0, *db, *df0, *dq0;
    double *du, *dv, *dud, *dvd;
    std::vector<Staged> arr = {
        {y, (double **)&dy, m3, true},
        {x0, (double **)&dx0, m3, true},
        {n0, (double **)&dn0, m3, true},
        {b, (double **)&db, (size_t)m, true},
        {(layers & SR_SL) ? f0 : nullptr, (double **)&df0, m3, true},
        {(layers & SR_DL) ? q0 : nullptr, (double **)&dq0, m3, true},
        {(layers & SR_SL) ? u : nullptr, &du, m3, false},
        {(layers & SR_DL) ? v : nullptr, &dv, m3, false},
        {(layers & SR_SL) ? u_delta : nullptr, &dud, 3 * m3, false},
        {(layers & SR_DL) ? v_delta : nullptr, &dvd, 3 * m3, false},
    };
    if ((st = stage_in("sr_eval", c, arr, s)) != SR_OK) return st;
    if ((st = eval_on_device("sr_eval", c, layers, m, dy, dx0, dn0, db, df0, dq0, du, dv, dud, dvd, s, nullptr)) !=
        SR_OK)
        return st;
    return stage_out(c, arr, s);
}

sr_status sr_eval_far(sr_ctx *c, int layers, int64_t m, const double *y, double *u, double *v, void *stream)
{
    g_err.clear();
    const bool host = (layers & SR_HOST) != 0;
    layers &= ~SR_HOST;
    sr_status st = eval_check("sr_eval_far", c, layers, m, kMaxTargets);
    if (st != SR_OK) return st;
    if (m == 0) return SR_OK;
    if (!y) return fail(SR_EINVAL, "sr_eval_far: y is NULL");
    if ((layers & SR_SL) && !u) return fail(SR_EINVAL, "sr_eval_far: SR_SL needs u");
    if ((layers & SR_DL) && !v) return fail(SR_EINVAL, "sr_eval_far: SR_DL needs v");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(SR_ENODEV, "sr_eval_far: cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    if ((st = ensure_packed(c, s)) != SR_OK) return st;
    const size_t m3 = 3 * (size_t)m;
    const double *dy = y;
    double *du = u, *dv = v;
    std::vector<Staged> arr = {
        {y, (double **)&dy, m3, true},
        {(layers & SR_SL) ? u : nullptr, &du, m3, false},
        {(layers & SR_DL) ? v : nullptr, &dv, m3, false},
    };
    if (host && (st = stage_in("sr_eval_far", c, arr, s)) != SR_OK) return st;
    // in chunks of at most kTargetChunk targets, as sr_eval
    for (int64_t c0 = 0, i = 0; c0 < m; c0 += kTargetChunk, ++i) {
        const int64_t mc = std::min<int64_t>(kTargetChunk, m - c0);
        EvalArgs a{};
        a.layers = layers;
        a.m = mc;
        a.y = dy + 3 * c0;
        a.u = du ? du + 3 * c0 : nullptr;
        a.v = dv ? dv + 3 * c0 : nullptr;
        for (int d = 0; d < 3; ++d) a.org[d] = c->prm.precision == SR_MIXED ? c->org[d] : 0.0;
        SR_HIP(c->part.reserve((size_t)kFarSplits * 6 * (size_t)mc));
        SR_HIP(launch_far_plain(c->prm.precision, layers, c->rec64.p, c->rec32.p, c->n, a, c->grid_rnear,
                                c->flag + i, c->part.p, s));
        SR_HIP(launch_far_add(layers, c->part.p, kFarSplits, a, true, s));
    }
    return host ? stage_out(c, arr, s) : SR_OK;
}

sr_status sr_check(sr_ctx *c, void *stream)
{
    g_err.clear();
    if (!c) return fail(SR_EINVAL, "sr_check: ctx is NULL");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(SR_ENODEV, "sr_check: cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    SR_HIP(hipStreamSynchronize(s));
    SR_HIP(hipStreamSynchronize(c->side));
    std::vector<NearFlag> slots(kFlagSlots);
    SR_HIP(hipMemcpy(slots.data(), c->flag, kFlagSlots * sizeof(NearFlag), hipMemcpyDeviceToHost));
    // slot i holds the reports of target chunk i: its first index is relative to the chunk
    NearFlag hf{0u, 0u, ~0ull};
    for (int i = 0; i < kFlagSlots; ++i)
        if (slots[i].bits != 0u) {
            hf.bits |= slots[i].bits;
            hf.first = std::min<unsigned long long>(hf.first, (unsigned long long)i * kTargetChunk + slots[i].first);
        }
    if (hf.bits == 0) return SR_OK;
    SR_HIP(launch_flag_clear(c->flag, kFlagSlots, s));
    SR_HIP(hipStreamSynchronize(s));
    if (hf.bits & kFlagFarTarget)
        return fail(SR_ENEAR, "sr_check: target %llu of sr_eval_far lies within the near radius of a source: it needs "
                              "its closest point and sr_eval", hf.first);
    return fail(SR_ENEAR, "sr_check: target %llu of sr_eval has |b| >= cutoff * max delta (far rule, no "
                          "extrapolation) but a source closer than that: b or x0 is wrong", hf.first);
}

int64_t sr_max_targets(void) { return kMaxTargets; }

static_assert(SR_NEAR_TABLE_INTERVALS == kTabIntervals && SR_NEAR_TABLE_DEGREE == kTabDegree &&
                  SR_NEAR_TABLE_DOUBLES == kTabDoubles,
              "the table layout of the header and of the near-field kernel differ");

sr_status sr_near_table(const double rho[3], double cutoff, double xmax, double *tab, int64_t n, double *maxerr)
{
    g_err.clear();
    if (!rho || !tab || n < kTabDoubles)
        return fail(SR_EINVAL, "sr_near_table: NULL argument or n < %d", kTabDoubles);
    for (int j = 0; j < 3; ++j)
        if (!(rho[j] > 0.0) || !std::isfinite(rho[j]))
            return fail(SR_EINVAL, "sr_near_table: rho[%d] must be positive and finite", j);
    if (rho[0] == rho[1] || rho[0] == rho[2] || rho[1] == rho[2])
        return fail(SR_EINVAL, "sr_near_table: the three rho must be distinct");
    if (!(cutoff > 0.0) || !std::isfinite(cutoff) || !(xmax > 0.0) || !std::isfinite(xmax))
        return fail(SR_EINVAL, "sr_near_table: cutoff and xmax must be positive and finite");
    std::vector<double> t;
    double err = 0.0;
    const bool ok = build_near_table(rho, cutoff, xmax, t, &err);
    if (maxerr) *maxerr = err;
    if (!ok) return fail(SR_ENOCONV, "sr_near_table: interpolation error %.3g exceeds 5e-14", err);
    std::copy(t.begin(), t.end(), tab);
    return SR_OK;
}

sr_status sr_tree_work(sr_ctx *c, int64_t m, const double *y, int64_t *proxy_pairs, int64_t *leaf_pairs,
                       int64_t *cluster_points)
{
#pragma clang fp contract(off)
    g_err.clear();
    if (!c || !proxy_pairs || !leaf_pairs || (m > 0 && !y) || m < 0)
        return fail(SR_EINVAL, "sr_tree_work: NULL argument or m < 0");
    if (c->prm.far_method != SR_TREE || c->n == 0 || c->layout_dirty || c->tree_dirty ||
        c->tree_p != c->prm.tree_degree || c->tree_leaf != c->prm.tree_leaf)
        return fail(SR_ESTATE, "sr_tree_work: needs far_method SR_TREE and a tree built by a previous sr_eval");
    const std::vector<TreeNode> &nodes = c->tree.nodes;
    const int64_t nprox = (int64_t)(c->tree_p + 1) * (c->tree_p + 1) * (c->tree_p + 1);
    const double theta2 = c->prm.tree_theta * c->prm.tree_theta, mac_r = tree_mac_radius(c, c->grid_rnear),
                 rnear2 = mac_r * mac_r;
    int64_t np = 0, nl = 0, nc = 0;
    std::vector<int> stack;
    for (int64_t t = 0; t < m; ++t) {
        const double *yt = y + 3 * t;
        stack.assign(1, 0);
        while (!stack.empty()) {
            const TreeNode &nd = nodes[stack.back()];
            stack.pop_back();
            // the kernels' acceptance test, same operations and order
            double R2 = 0.0, g2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double dc = yt[d] - 0.5 * (nd.lo[d] + nd.hi[d]);
                R2 += dc * dc;
                const double gap =
                    nd.lo[d] - yt[d] > 0.0 ? nd.lo[d] - yt[d] : (yt[d] - nd.hi[d] > 0.0 ? yt[d] - nd.hi[d] : 0.0);
                g2 += gap * gap;
            }
            if (nd.rc2 <= theta2 * R2 && g2 > rnear2) {
                np += nprox;
                nc += nd.end - nd.begin;
            } else if (nd.nchild == 0)
                nl += nd.end - nd.begin;
            else
                for (int k = 0; k < nd.nchild; ++k) stack.push_back(nd.first_child + k);
        }
    }
    *proxy_pairs = np;
    *leaf_pairs = nl;
    if (cluster_points) *cluster_points = nc;
    return SR_OK;
}

sr_status sr_set_profiling(sr_ctx *c, int on)
{
    g_err.clear();
    if (!c) return fail(SR_EINVAL, "sr_set_profiling: ctx is NULL");
    c->profiling = on != 0;
    return SR_OK;
}

sr_status sr_get_profile(sr_ctx *c, double *ms, int64_t *evals)
{
    g_err.clear();
    if (!c || !ms || !evals) return fail(SR_EINVAL, "sr_get_profile: NULL argument");
    DeviceGuard g(c->device);
    for (int k = 0; k < SR_NPHASES; ++k) ms[k] = 0.0;
    const size_t ne = c->ev_recorded.size() / 3;
    for (size_t i = 0; i < ne; ++i) {
        hipEvent_t *e = &c->ev_recorded[3 * i];
        SR_HIP(hipEventSynchronize(e[2]));
        float a = 0.f, b = 0.f;
        SR_HIP(hipEventElapsedTime(&a, e[0], e[1]));
        SR_HIP(hipEventElapsedTime(&b, e[1], e[2]));
        ms[SR_PHASE_FAR] += a;
        ms[SR_PHASE_NEAR] += b;
    }
    *evals = (int64_t)ne;
    for (hipEvent_t e : c->ev_recorded) c->ev_pool.push_back(e);
    c->ev_recorded.clear();
    return SR_OK;
}

}  // extern "C"

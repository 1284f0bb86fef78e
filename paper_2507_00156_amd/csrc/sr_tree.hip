// Barycentric-Lagrange treecode for the far field (paper section 3.4, eqs. (MAC),
// (particle-cluster-KITC), (mod_weights)).
//
// Tree (host, at set-up): octree over the sources; a cluster with more than N0 points is split at the
// midpoint of its box into 8 octants (upper half when x >= mid), empty octants dropped, every box the
// bounding box of its points, children stored contiguously in octant order.  A split that cannot
// separate the points (all in one octant) stops there.
//
// Proxies: per cluster the (p+1)^3 tensor Chebyshev points of the second kind
// s = c + (h/2) cos(k pi / p) per axis (an axis of zero extent: s = lo), and 15 modified-weight
// channels (eq. (mod_weights)): F = sum L f w (3), N = sum L n w (3), Q = sum L q_j n_k w (9), with the
// barycentric Lagrange basis L (weights (-1)^k, halved at both ends; exact-node and zero-extent rules
// as in the oracle).
//
// Anterpolation (per density): the modified weights of a cluster are the contraction
// G_hat[proxy][ch] = sum_points Phi[point][proxy] G[point][ch], a dense GEMM evaluated with FP64
// matrix cores (v_mfma_f64_16x16x4f64: 16 proxies x 16 channels per wave tile, 4 points per step).
// Large clusters are split into chunks whose partial products are summed in a fixed order.
//
// Evaluation (per target set): targets are sorted by a Morton key so that a wavefront's 64 lanes hold
// nearby targets.  Each wavefront walks the tree depth-first with an LDS stack of (cluster, lane mask)
// entries; per lane the MAC r_c^2 <= theta^2 R^2 with the box farther than the near radius (computed in
// FP64 without contraction, the same arithmetic as the oracle) decides between the proxy sum (original
// kernels) and descending; at a leaf the remaining lanes sum the leaf's points directly, skipping the
// near pairs (same pair_r2 test as the near-field kernel).  The walk is split over the clusters of a
// cut of the tree (the frontier, at most kMaxFrontier clusters; blockIdx.y selects one): a split
// first applies the MAC to the frontier node's ancestors, root first, exactly as the per-target walk
// would, so every target accepts the same clusters as in one walk; the proxy sum of an accepted
// ancestor is added by the first frontier node below it.  Output: per split, one partial sum per
// channel and target (the layout of the direct far field).  The proxies of all clusters (80 B each in
// FP32, 22 MB at 169k sources, p = 8) do not fit one XCD's 4 MB L2, but the clusters accepted by the
// targets of one region do: each XCD takes a contiguous eighth of the Morton-sorted targets.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "sr_internal.h"
#include "sr_tree.h"

namespace sr {

// ------------------------------------------------------------------------------------------ host

namespace {

void node_bbox(const double *hx, const std::vector<int64_t> &order, TreeNode &nd)
{
    for (int d = 0; d < 3; ++d) {
        nd.lo[d] = INFINITY;
        nd.hi[d] = -INFINITY;
    }
    for (int64_t i = nd.begin; i < nd.end; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = hx[3 * order[i] + d];
            nd.lo[d] = std::min(nd.lo[d], v);
            nd.hi[d] = std::max(nd.hi[d], v);
        }
}

}  // namespace

void build_tree(const double *hx, int64_t n, int64_t leaf, int p, TreeHost &T)
{
#pragma clang fp contract(off)
    T.nodes.clear();
    T.order.resize(n);
    for (int64_t i = 0; i < n; ++i) T.order[i] = i;
    T.p = p;
    TreeNode root{};
    root.begin = 0;
    root.end = (int)n;
    root.first_child = -1;
    node_bbox(hx, T.order, root);
    T.nodes.push_back(root);
    // depth-first, children created together (contiguous) before descending, as in the oracle
    std::vector<int> stack{0};
    std::vector<int64_t> tmp;
    int depth_max = 0;
    std::vector<int> depth{0};
    while (!stack.empty()) {
        const int id = stack.back();
        stack.pop_back();
        TreeNode nd = T.nodes[id];
        if (nd.end - nd.begin <= leaf) continue;
        double mid[3];
        for (int d = 0; d < 3; ++d) mid[d] = (nd.lo[d] + nd.hi[d]) * 0.5;
        int64_t cnt[8] = {0};
        auto octant = [&](int64_t o) {
            const double *q = hx + 3 * o;
            return (q[0] >= mid[0] ? 1 : 0) | (q[1] >= mid[1] ? 2 : 0) | (q[2] >= mid[2] ? 4 : 0);
        };
        for (int64_t i = nd.begin; i < nd.end; ++i) cnt[octant(T.order[i])]++;
        int nonempty = 0;
        for (int o = 0; o < 8; ++o) nonempty += cnt[o] > 0;
        if (nonempty < 2) continue;  // cannot separate (coincident points): keep as a leaf
        int64_t start[8], fill[8];
        start[0] = 0;
        for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
        for (int o = 0; o < 8; ++o) fill[o] = start[o];
        tmp.resize(nd.end - nd.begin);
        for (int64_t i = nd.begin; i < nd.end; ++i) {
            const int64_t o = T.order[i];
            tmp[fill[octant(o)]++] = o;
        }
        std::copy(tmp.begin(), tmp.end(), T.order.begin() + nd.begin);
        const int first = (int)T.nodes.size();
        int nch = 0;
        for (int o = 0; o < 8; ++o) {
            if (cnt[o] == 0) continue;
            TreeNode c{};
            c.begin = (int)(nd.begin + start[o]);
            c.end = (int)(nd.begin + start[o] + cnt[o]);
            c.first_child = -1;
            node_bbox(hx, T.order, c);
            T.nodes.push_back(c);
            depth.push_back(depth[id] + 1);
            depth_max = std::max(depth_max, depth[id] + 1);
            ++nch;
        }
        T.nodes[id].first_child = first;
        T.nodes[id].nchild = nch;
        for (int k = nch - 1; k >= 0; --k) stack.push_back(first + k);
    }
    for (TreeNode &nd : T.nodes) {
        double rc2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double e = nd.hi[d] - nd.lo[d];
            rc2 += 0.25 * e * e;
        }
        nd.rc2 = rc2;
        if (nd.first_child < 0) nd.nchild = 0;
    }
    T.depth = depth_max;
    // frontier: the tree cut level by level while it has at most kMaxFrontier nodes
    std::vector<int> parent(T.nodes.size(), -1);
    for (size_t id = 0; id < T.nodes.size(); ++id)
        for (int k = 0; k < T.nodes[id].nchild; ++k) parent[T.nodes[id].first_child + k] = (int)id;
    std::vector<int> F{0};
    // every expanded level adds at least one cluster (a split has >= 2 children), so at most
    // kMaxFrontier - 1 levels: the ancestor chains fit kMaxFrontierDepth
    for (int level = 0; level < kMaxFrontierDepth - 1; ++level) {
        std::vector<int> nxt;
        for (int id : F) {
            if (T.nodes[id].nchild == 0)
                nxt.push_back(id);
            else
                for (int k = 0; k < T.nodes[id].nchild; ++k) nxt.push_back(T.nodes[id].first_child + k);
        }
        if (nxt == F || (int)nxt.size() > kMaxFrontier) break;
        F.swap(nxt);
    }
    T.front.clear();
    std::vector<char> seen(T.nodes.size(), 0);
    for (int f : F) {
        FrontierRec r{};
        r.node = f;
        int chain[kMaxFrontierDepth], nc = 0;
        for (int a = parent[f]; a >= 0; a = parent[a]) chain[nc++] = a;  // frontier depth <= log8(kMaxFrontier)
        r.nanc = nc;
        for (int j = 0; j < nc; ++j) {
            r.anc[j] = chain[nc - 1 - j];  // root first
            if (!seen[r.anc[j]]) {
                seen[r.anc[j]] = 1;
                r.first |= 1 << j;
            }
        }
        T.front.push_back(r);
    }
    // Chebyshev points of each cluster
    const int np1 = p + 1, nprox = np1 * np1 * np1;
    T.cosk.resize(np1);
    for (int k = 0; k <= p; ++k) T.cosk[k] = std::cos(k * 3.14159265358979323846264338327950288 / p);
    T.proxy_xyz.resize((size_t)T.nodes.size() * nprox * 3);
    for (size_t id = 0; id < T.nodes.size(); ++id) {
        const TreeNode &nd = T.nodes[id];
        double s[3][17];
        for (int d = 0; d < 3; ++d)
            for (int k = 0; k <= p; ++k) {
                const double c = 0.5 * (nd.lo[d] + nd.hi[d]), hw = 0.5 * (nd.hi[d] - nd.lo[d]);
                s[d][k] = nd.hi[d] == nd.lo[d] ? nd.lo[d] : c + hw * T.cosk[k];
            }
        for (int k1 = 0; k1 <= p; ++k1)
            for (int k2 = 0; k2 <= p; ++k2)
                for (int k3 = 0; k3 <= p; ++k3) {
                    double *o = &T.proxy_xyz[((size_t)id * nprox + (k1 * np1 + k2) * np1 + k3) * 3];
                    o[0] = s[0][k1];
                    o[1] = s[1][k2];
                    o[2] = s[2][k3];
                }
    }
    // anterpolation work items: clusters in chunks of at most kAnterpChunk points
    T.item_node.clear();
    T.item_begin.clear();
    T.item_end.clear();
    T.node_item0.assign(T.nodes.size() + 1, 0);
    for (size_t id = 0; id < T.nodes.size(); ++id) {
        T.node_item0[id] = (int)T.item_node.size();
        for (int b = T.nodes[id].begin; b < T.nodes[id].end; b += kAnterpChunk) {
            T.item_node.push_back((int)id);
            T.item_begin.push_back(b);
            T.item_end.push_back(std::min(b + kAnterpChunk, T.nodes[id].end));
        }
    }
    T.node_item0[T.nodes.size()] = (int)T.item_node.size();
}

// ---------------------------------------------------------------------------------------- device

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxDeg = 16;
constexpr int kSub = 64;         // points per LDS sub-chunk
constexpr int kTilesPerWave = 6;  // 16-proxy tiles per wavefront and pass: degree 6 (22 tiles) keeps all
                                  // four wavefronts busy in one pass, degree 8 (46 tiles) takes two

// barycentric Lagrange basis at v for the Chebyshev points of [lo, hi] (the oracle's rules)
__device__ void lagrange_1d(double v, double lo, double hi, int p, const double *cosk, double *L)
{
#pragma clang fp contract(off)
    if (hi == lo) {
        for (int k = 0; k <= p; ++k) L[k] = k == 0 ? 1.0 : 0.0;
        return;
    }
    const double c = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
    double den = 0.0;
    int hit = -1;
    for (int k = 0; k <= p; ++k) {
        const double s = c + hw * cosk[k];
        if (v == s) hit = hit < 0 ? k : hit;
        const double wk = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == p) ? 0.5 : 1.0);
        L[k] = wk / (v - s);
        den += L[k];
    }
    if (hit >= 0) {
        for (int k = 0; k <= p; ++k) L[k] = k == hit ? 1.0 : 0.0;
        return;
    }
    const double inv = 1.0 / den;
    for (int k = 0; k <= p; ++k) L[k] *= inv;
}

struct AnterpArgs {
    const TreeNode *nodes;
    const int *item_node, *item_begin, *item_end;
    const SrcRec<double> *trec;
    double *partial;  // [item][nprox][16]
    int p, nprox;
    double cosk[kMaxDeg + 1];
};

__global__ __launch_bounds__(kBlock) void anterp_kernel(AnterpArgs a)
{
    __shared__ double basis[kSub][3][kMaxDeg + 1];
    __shared__ double G[kSub][16];
    const int item = blockIdx.x;
    const int pass = blockIdx.y;  // group of 4 * kTilesPerWave proxy tiles
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int lane = (int)threadIdx.x % kWave;
    const TreeNode nd = a.nodes[a.item_node[item]];
    const int b0 = a.item_begin[item], b1 = a.item_end[item];
    const int p = a.p, np1 = p + 1, nprox = a.nprox;

    d4 acc[kTilesPerWave];
    int k1[kTilesPerWave], k2[kTilesPerWave], k3[kTilesPerWave];
    bool live[kTilesPerWave], row[kTilesPerWave];
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) {
        acc[i] = d4{0.0, 0.0, 0.0, 0.0};
        const int tile = (pass * 4 + wave) * kTilesPerWave + i;
        const int P = tile * 16 + lane % 16;
        live[i] = tile * 16 < nprox;
        const int Pc = P < nprox ? P : 0;
        k1[i] = Pc / (np1 * np1);
        k2[i] = (Pc / np1) % np1;
        k3[i] = Pc % np1;
        row[i] = P < nprox;  // padding rows of the last tile: A = 0
    }

    for (int sub = b0; sub < b1; sub += kSub) {
        const int t = (int)threadIdx.x;
        if (t < 3 * kSub) {
            // the basis goes straight to its LDS row (a local array indexed by the run-time degree
            // would live in scratch memory)
            const int pt = t / 3, ax = t % 3;
            const int gi = sub + pt;
            double *L = basis[pt][ax];
            if (gi < b1) {
                const SrcRec<double> &s = a.trec[gi];
                const double v = ax == 0 ? s.x : (ax == 1 ? s.y : s.z);
                lagrange_1d(v, nd.lo[ax], nd.hi[ax], p, a.cosk, L);
            } else {
                for (int k = 0; k <= p; ++k) L[k] = 0.0;
            }
        } else {
            const int pt = t - 3 * kSub;
            const int gi = sub + pt;
            double ch[16];
            if (gi < b1) {
                const SrcRec<double> &s = a.trec[gi];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    ch[j] = s.fw[j];
                    ch[3 + j] = s.nw[j];
                }
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int k = 0; k < 3; ++k) ch[6 + 3 * j + k] = s.q[j] * s.nw[k];
                ch[15] = 0.0;
            } else {
#pragma unroll
                for (int c = 0; c < 16; ++c) ch[c] = 0.0;
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) G[pt][c] = ch[c];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kTilesPerWave; ++i) {
            if (!live[i]) continue;  // wavefront-uniform
#pragma unroll 4
            for (int kq = 0; kq < kSub / 4; ++kq) {
                const int pt = kq * 4 + lane / 16;
                const double prod = basis[pt][0][k1[i]] * basis[pt][1][k2[i]] * basis[pt][2][k3[i]];
                const double av = row[i] ? prod : 0.0;
                const double bv = G[pt][lane % 16];
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[i], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[4v + lane/16][lane%16] sits in element v of the lane
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) {
        if (!live[i]) continue;
        const int tile = (pass * 4 + wave) * kTilesPerWave + i;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int P = tile * 16 + 4 * v + lane / 16;
            if (P < nprox) a.partial[((size_t)item * nprox + P) * 16 + lane % 16] = acc[i][v];
        }
    }
}

// sum the partial products of each cluster's items (in item order) into its proxy records; one lane
// per (cluster, proxy, channel), so that a cluster with many items (the root) is not one thread's
// serial loop, with 8 items' loads in flight; the additions keep the item order
__global__ __launch_bounds__(kBlock) void anterp_reduce_kernel(const int *node_item0, const double *partial,
                                                                int nnodes, int nprox, ProxRec<double> *prox64,
                                                                ProxRec<float> *prox32)
{
    constexpr int kInFlight = 8;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t total = (int64_t)nnodes * nprox * 16;
    if (gid >= total) return;
    const int c = (int)(gid % 16);
    if (c == 15) return;  // padding channel of the partial products
    const int64_t np = gid / 16;  // node * nprox + P
    const int node = (int)(np / nprox);
    const int P = (int)(np % nprox);
    const int i1 = node_item0[node + 1];
    double s = 0.0;
    int it = node_item0[node];
    for (; it + kInFlight <= i1; it += kInFlight) {
        double v[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) v[u] = partial[((size_t)(it + u) * nprox + P) * 16 + c];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) s += v[u];
    }
    for (; it < i1; ++it) s += partial[((size_t)it * nprox + P) * 16 + c];
    prox64[np].g[c] = s;
    prox32[np].g[c] = (float)s;
}

// ---- target ordering ----

__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

__global__ __launch_bounds__(kBlock) void morton_kernel(const double *y, const double *b, int m, double lox,
                                                        double loy, double loz, double inv, uint32_t *key, int *idx)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= m) return;
    uint32_t q[3];
    const double lo[3] = {lox, loy, loz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = (y[3 * t + d] - lo[d]) * inv;
        u = fmin(fmax(u, 0.0), 1023.0);
        q[d] = (uint32_t)u;
    }
    const uint32_t off = (b != nullptr && b[t] != 0.0) ? (1u << 30) : 0u;
    key[t] = off | spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    idx[t] = t;
}

// ---- evaluation ----

__device__ __forceinline__ bool mac_accept(const TreeNode &nd, double yx, double yy, double yz, double theta2,
                                           double rnear2)
{
#pragma clang fp contract(off)
    const double y[3] = {yx, yy, yz};
    double R2 = 0.0, g2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double dc = y[d] - 0.5 * (nd.lo[d] + nd.hi[d]);
        R2 += dc * dc;
        const double gap = nd.lo[d] - y[d] > 0.0 ? nd.lo[d] - y[d] : (y[d] - nd.hi[d] > 0.0 ? y[d] - nd.hi[d] : 0.0);
        g2 += gap * gap;
    }
    return nd.rc2 <= theta2 * R2 && g2 > rnear2;
}

__device__ __forceinline__ float rsqrt_t(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double rsqrt_t(double v) { return rsqrt(v); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
struct Lane {
    T y[3], c, q0[3];
    T rc2;  // the target's near radius squared (smaller for surface targets under the modified smoothing)
};

constexpr int kPromote = 32;  // terms summed in T before promotion to FP64

template <typename T, bool SL, bool DL>
__device__ __forceinline__ void proxy_sum(const ProxRec<T> *__restrict__ pr, int nprox, const Lane<T> &L,
                                          double acc[6])
{
    // the record of the next proxy is loaded while the current one is evaluated (the index is
    // wavefront-uniform: scalar loads, whose latency a plain loop would expose every iteration)
    ProxRec<T> nxt = pr[0];
    for (int k0 = 0; k0 < nprox; k0 += kPromote) {
        T a[6] = {0, 0, 0, 0, 0, 0};
        const int k1 = min(k0 + kPromote, nprox);
        for (int k = k0; k < k1; ++k) {
            const ProxRec<T> s = nxt;
            nxt = pr[min(k + 1, nprox - 1)];
            const T dx = L.y[0] - s.x, dy = L.y[1] - s.y, dz = L.y[2] - s.z;
            const T r2 = fma_t(dz, dz, fma_t(dy, dy, dx * dx));
            const T ir = rsqrt_t(r2);
            const T ir2 = ir * ir, ir3 = ir2 * ir;
            if (SL) {
                const T gx = fma_t(-L.c, s.g[3], s.g[0]);
                const T gy = fma_t(-L.c, s.g[4], s.g[1]);
                const T gz = fma_t(-L.c, s.g[5], s.g[2]);
                const T sc = (dx * gx + dy * gy + dz * gz) * ir3;
                a[0] = fma_t(dx, sc, fma_t(gx, ir, a[0]));
                a[1] = fma_t(dy, sc, fma_t(gy, ir, a[1]));
                a[2] = fma_t(dz, sc, fma_t(gz, ir, a[2]));
            }
            if (DL) {
                // d^T (Q - q0 N^T) d with Q[j][k] = sum L q_j n_k w, N = sum L n w
                const T Qd0 = s.g[6] * dx + s.g[7] * dy + s.g[8] * dz;
                const T Qd1 = s.g[9] * dx + s.g[10] * dy + s.g[11] * dz;
                const T Qd2 = s.g[12] * dx + s.g[13] * dy + s.g[14] * dz;
                const T dQd = dx * Qd0 + dy * Qd1 + dz * Qd2;
                const T dq = dx * L.q0[0] + dy * L.q0[1] + dz * L.q0[2];
                const T dn = dx * s.g[3] + dy * s.g[4] + dz * s.g[5];
                const T co = fma_t(-dq, dn, dQd) * (ir3 * ir2);
                a[3] = fma_t(dx, co, a[3]);
                a[4] = fma_t(dy, co, a[4]);
                a[5] = fma_t(dz, co, a[5]);
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += (double)a[c];
    }
}

template <typename T, bool SL, bool DL>
__device__ __forceinline__ void leaf_sum(const SrcRec<T> *__restrict__ src, int b0, int b1, const Lane<T> &L,
                                         double acc[6])
{
    SrcRec<T> nxt = src[b0];
    for (int k0 = b0; k0 < b1; k0 += kPromote) {
        T a[6] = {0, 0, 0, 0, 0, 0};
        const int k1 = min(k0 + kPromote, b1);
        for (int k = k0; k < k1; ++k) {
            const SrcRec<T> s = nxt;
            nxt = src[min(k + 1, b1 - 1)];
            const T dx = L.y[0] - s.x, dy = L.y[1] - s.y, dz = L.y[2] - s.z;
            const T r2 = pair_r2(L.y[0], L.y[1], L.y[2], s.x, s.y, s.z);
            const T ir = r2 > L.rc2 ? rsqrt_t(r2) : (T)0;  // near pairs belong to the near-field kernel
            const T ir2 = ir * ir, ir3 = ir2 * ir;
            if (SL) {
                const T gx = fma_t(-L.c, s.nw[0], s.fw[0]);
                const T gy = fma_t(-L.c, s.nw[1], s.fw[1]);
                const T gz = fma_t(-L.c, s.nw[2], s.fw[2]);
                const T sc = (dx * gx + dy * gy + dz * gz) * ir3;
                a[0] = fma_t(dx, sc, fma_t(gx, ir, a[0]));
                a[1] = fma_t(dy, sc, fma_t(gy, ir, a[1]));
                a[2] = fma_t(dz, sc, fma_t(gz, ir, a[2]));
            }
            if (DL) {
                const T ax = s.q[0] - L.q0[0], ay = s.q[1] - L.q0[1], az = s.q[2] - L.q0[2];
                const T da = dx * ax + dy * ay + dz * az;
                const T dm = dx * s.nw[0] + dy * s.nw[1] + dz * s.nw[2];
                const T co = da * dm * (ir3 * ir2);
                a[3] = fma_t(dx, co, a[3]);
                a[4] = fma_t(dy, co, a[4]);
                a[5] = fma_t(dz, co, a[5]);
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += (double)a[c];
    }
}

template <typename T, bool SL, bool DL>
__global__ __launch_bounds__(kBlock) void tree_far_kernel(const TreeNode *__restrict__ nodes,
                                                          const ProxRec<T> *__restrict__ prox, int nprox,
                                                          const SrcRec<T> *__restrict__ trec,
                                                          const int *__restrict__ order,
                                                          const FrontierRec *__restrict__ front, EvalArgs a,
                                                          double theta2, double rnear2, T rc2, T rc2s, int sharp,
                                                          int stack_cap, double *__restrict__ part)
{
    extern __shared__ int smem[];
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int lane = (int)threadIdx.x % kWave;
    int *stk_node = smem + wave * stack_cap * 3;
    uint32_t *stk_mask = (uint32_t *)(stk_node + stack_cap);  // 2 words per entry
    const int m = (int)a.m;
    // workgroups are dispatched round-robin over the 8 XCDs (gridDim.x is a multiple of 8, so the XCD
    // is blockIdx.x % 8 for every split): XCD x takes the x-th contiguous eighth of the Morton-sorted
    // targets, a compact region whose accepted clusters' proxies fit its L2
    const int per_xcd = (int)gridDim.x / 8;
    const int bx = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    const int si = (bx * (kBlock / kWave) + wave) * kWave + lane;
    const bool valid = si < m;
    const int t = order[valid ? si : m - 1];

    double yd[3];
    Lane<T> L;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        yd[i] = a.y[3 * t + i];
        L.y[i] = (T)(yd[i] - a.org[i]);
        L.q0[i] = DL ? (T)a.q0[3 * t + i] : (T)0;
    }
    L.c = SL ? (T)(a.f0[3 * t] * a.n0[3 * t] + a.f0[3 * t + 1] * a.n0[3 * t + 1] + a.f0[3 * t + 2] * a.n0[3 * t + 2])
             : (T)0;
    // the MAC keeps the full near radius (conservative); the leaf sums skip the target's own near pairs
    L.rc2 = (sharp && a.b[t] == 0.0) ? rc2s : rc2;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    // this split's frontier node: first its ancestors (root first), as the per-target walk would
    // visit them; a lane that accepts one is done in this split, and the accepted ancestor's proxy
    // sum is added by the first frontier node below it only
    const FrontierRec &fr = front[blockIdx.y];
    uint64_t live = __ballot(valid);
    for (int j = 0; j < fr.nanc; ++j) {
        const int aid = fr.anc[j];
        const TreeNode an = nodes[aid];
        const bool acc_here = ((live >> lane) & 1) && mac_accept(an, yd[0], yd[1], yd[2], theta2, rnear2);
        const uint64_t am = __ballot(acc_here);
        if (am && ((fr.first >> j) & 1) && acc_here) proxy_sum<T, SL, DL>(prox + (size_t)aid * nprox, nprox, L, acc);
        live &= ~am;
    }
    int sp = 0;
    if (lane == 0) {
        stk_node[0] = fr.node;
        stk_mask[0] = (uint32_t)live;
        stk_mask[1] = (uint32_t)(live >> 32);
    }
    sp = live ? 1 : 0;
    while (sp > 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        --sp;
        const int id = __builtin_amdgcn_readfirstlane(stk_node[sp]);
        const uint64_t mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(stk_mask[2 * sp + 1]) << 32) |
                              (uint32_t)__builtin_amdgcn_readfirstlane(stk_mask[2 * sp]);
        const TreeNode nd = nodes[id];
        const bool mine = (mask >> lane) & 1;
        const bool acc_here = mine && mac_accept(nd, yd[0], yd[1], yd[2], theta2, rnear2);
        const uint64_t am = __ballot(acc_here);
        const uint64_t rm = mask & ~am;
        if (am) {
            if (acc_here) proxy_sum<T, SL, DL>(prox + (size_t)id * nprox, nprox, L, acc);
        }
        if (rm) {
            if (nd.nchild == 0) {
                if ((rm >> lane) & 1) leaf_sum<T, SL, DL>(trec, nd.begin, nd.end, L, acc);
            } else {
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    for (int k = nd.nchild - 1; k >= 0; --k) {
                        const int e = sp + (nd.nchild - 1 - k);
                        stk_node[e] = nd.first_child + k;
                        stk_mask[2 * e] = (uint32_t)rm;
                        stk_mask[2 * e + 1] = (uint32_t)(rm >> 32);
                    }
                }
                sp += nd.nchild;
            }
        }
    }
    if (valid) {
        double *ps = part + (size_t)blockIdx.y * 6 * (size_t)m;
        if (SL)
#pragma unroll
            for (int c = 0; c < 3; ++c) ps[(size_t)c * m + t] = acc[c];
        if (DL)
#pragma unroll
            for (int c = 3; c < 6; ++c) ps[(size_t)c * m + t] = acc[c];
    }
}

template <typename T, bool SL, bool DL>
hipError_t launch_far_t(const TreeDev &D, const ProxRec<T> *prox, const SrcRec<T> *trec, const EvalArgs &a,
                        double theta2, double rnear2, T rc2, T rc2s, int sharp, double *part, hipStream_t s)
{
    const int m = (int)a.m;
    const int blocks = ((m + kBlock - 1) / kBlock + 7) / 8 * 8;
    const size_t shmem = (size_t)(kBlock / kWave) * D.stack_cap * 3 * sizeof(int);
    hipLaunchKernelGGL((tree_far_kernel<T, SL, DL>), dim3(blocks, D.nfront), dim3(kBlock), shmem, s, D.nodes, prox,
                       D.nprox, trec, D.order, D.front, a, theta2, rnear2, rc2, rc2s, sharp, D.stack_cap, part);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_anterp(const TreeDev &D, const double *cosk, double *partial, hipStream_t s)
{
    AnterpArgs a{};
    a.nodes = D.nodes;
    a.item_node = D.item_node;
    a.item_begin = D.item_begin;
    a.item_end = D.item_end;
    a.trec = D.trec64;
    a.partial = partial;
    a.p = D.p;
    a.nprox = D.nprox;
    for (int k = 0; k <= D.p; ++k) a.cosk[k] = cosk[k];
    const int tiles = (D.nprox + 15) / 16;
    const int passes = (tiles + 4 * kTilesPerWave - 1) / (4 * kTilesPerWave);
    hipLaunchKernelGGL(anterp_kernel, dim3(D.nitems, passes), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)D.nnodes * D.nprox * 16;
    hipLaunchKernelGGL(anterp_reduce_kernel, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       D.node_item0, partial, D.nnodes, D.nprox, D.prox64, D.prox32);
    return hipGetLastError();
}

hipError_t launch_target_order(const double *y, const double *b, int m, const double lo[3], double inv, TreeDev &D,
                               hipStream_t s)
{
    hipLaunchKernelGGL(morton_kernel, dim3((m + kBlock - 1) / kBlock), dim3(kBlock), 0, s, y, b, m, lo[0], lo[1],
                       lo[2], inv, D.key_in, D.idx_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = D.sort_tmp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(D.sort_tmp, bytes, D.key_in, D.key_out, D.idx_in, D.order, m, 0, 31, s);
}

size_t target_sort_tmp_bytes(int m)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs((void *)nullptr, bytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                       (int *)nullptr, (int *)nullptr, m, 0, 31);
    return bytes;
}

hipError_t launch_tree_far(int precision, int layers, const TreeDev &D, const EvalArgs &a, double theta,
                           double rnear, double mac_rnear, double rsharp, int sharp, double *part, hipStream_t s)
{
#pragma clang fp contract(off)
    const double theta2 = theta * theta, rnear2 = rnear * rnear, rs2 = rsharp * rsharp;
    if (precision == SR_MIXED) {
        const float rc2 = (float)rnear2, rc2s = (float)rs2;
        const double mac2 = mac_rnear * mac_rnear;
        if (layers == (SR_SL | SR_DL))
            return launch_far_t<float, true, true>(D, D.prox32, D.trec32, a, theta2, mac2, rc2, rc2s, sharp, part, s);
        if (layers == SR_SL)
            return launch_far_t<float, true, false>(D, D.prox32, D.trec32, a, theta2, mac2, rc2, rc2s, sharp, part, s);
        return launch_far_t<float, false, true>(D, D.prox32, D.trec32, a, theta2, mac2, rc2, rc2s, sharp, part, s);
    }
    if (layers == (SR_SL | SR_DL))
        return launch_far_t<double, true, true>(D, D.prox64, D.trec64, a, theta2, rnear2, rnear2, rs2, sharp, part, s);
    if (layers == SR_SL)
        return launch_far_t<double, true, false>(D, D.prox64, D.trec64, a, theta2, rnear2, rnear2, rs2, sharp, part, s);
    return launch_far_t<double, false, true>(D, D.prox64, D.trec64, a, theta2, rnear2, rnear2, rs2, sharp, part, s);
}

}  // namespace sr

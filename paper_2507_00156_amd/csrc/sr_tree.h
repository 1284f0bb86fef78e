// Treecode data structures shared by the host set-up (sr_api.hip) and the kernels (sr_tree.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sr_internal.h"

namespace sr {

// Points per anterpolation work item: small enough that the two-sphere problem (68k points per
// sphere, three tree levels) gives about 900 workgroups for the 256 CUs (2048 gave about 140).
constexpr int kAnterpChunk = 256;

// One cluster: bounding box, squared radius r_c^2 = (1/4) |hi - lo|^2, points [begin, end) of the
// tree-ordered sources, children [first_child, first_child + nchild) (nchild = 0 for a leaf).
struct TreeNode {
    double lo[3], hi[3];
    double rc2;
    int begin, end, first_child, nchild;
};

// Chebyshev proxy point of a cluster with its modified weights:
// g[0..2] = F (f w), g[3..5] = N (n w), g[6 + 3 j + k] = Q_jk (q_j n_k w).
template <typename T>
struct alignas(16) ProxRec {
    T x, y, z, pad;
    T g[15];
    T pad2;
};

// One cluster of the frontier (a cut of the tree that splits the walk): its ancestors, root first, and
// bit j of `first` set when it is the first frontier cluster below anc[j].
constexpr int kMaxFrontier = 8;
constexpr int kMaxFrontierDepth = 8;
struct FrontierRec {
    int node, nanc, first;
    int anc[kMaxFrontierDepth];
};

struct TreeHost {
    std::vector<TreeNode> nodes;
    std::vector<int64_t> order;      // tree order -> caller index
    std::vector<double> cosk;        // cos(k pi / p)
    std::vector<double> proxy_xyz;   // [node][proxy][3]
    std::vector<int> item_node, item_begin, item_end, node_item0;
    std::vector<FrontierRec> front;
    int p = 0, depth = 0;
};

struct TreeDev {
    TreeNode *nodes = nullptr;
    int *item_node = nullptr, *item_begin = nullptr, *item_end = nullptr, *node_item0 = nullptr;
    SrcRec<double> *trec64 = nullptr;
    SrcRec<float> *trec32 = nullptr;
    ProxRec<double> *prox64 = nullptr;
    ProxRec<float> *prox32 = nullptr;
    // target ordering
    uint32_t *key_in = nullptr, *key_out = nullptr;
    int *idx_in = nullptr, *order = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    FrontierRec *front = nullptr;
    int nnodes = 0, nitems = 0, nprox = 0, p = 0, stack_cap = 0, nfront = 1;
};

// Build the octree (host), its proxy points and anterpolation items.  hx: (n,3) caller order.
void build_tree(const double *hx, int64_t n, int64_t leaf, int p, TreeHost &T);

// Modified weights of every cluster from the tree-ordered records (FP64 matrix cores), into
// D.prox64 / D.prox32 (channels only; positions are set at upload).  partial: nitems*nprox*16 doubles.
hipError_t launch_anterp(const TreeDev &D, const double *cosk, double *partial, hipStream_t s);

// Sort targets by a 30-bit Morton key of their position quantized in [lo, lo + 1024/inv); D.order
// receives the sorted target indices.
// b (nullable): the targets' signed distances; those with b != 0 then follow those with b == 0 (each
// part in Morton order).
hipError_t launch_target_order(const double *y, const double *b, int m, const double lo[3], double inv, TreeDev &D,
                               hipStream_t s);
size_t target_sort_tmp_bytes(int m);

// Far field by the treecode into part[split][channel][target], D.nfront splits.
// rnear / rsharp / sharp: as for launch_far_direct (the leaf sums' pair test).  mac_rnear: the radius
// the MAC requires a cluster's box to lie beyond: rnear on the FP64 path, whose pair test is exact to
// the MAC's; on the mixed path the cell grid's reach (rnear widened by the FP32 rounding of the pair
// test), so that no source of an accepted cluster is also a near pair of the FP32 test.
hipError_t launch_tree_far(int precision, int layers, const TreeDev &D, const EvalArgs &a, double theta,
                           double rnear, double mac_rnear, double rsharp, int sharp, double *part, hipStream_t s);

}  // namespace sr

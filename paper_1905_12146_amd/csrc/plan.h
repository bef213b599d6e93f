// Host-side planning of the traversal kernels: tree levels, the top levels
// and depth-first clade lists the post- and pre-order kernels walk, the
// pre-order top region kept in LDS, and the dirty-path schedule of a partial
// re-evaluation.  Plain C++ with no HIP dependency, so the planners can be
// built and checked on a host alone (with sanitizers); the library uploads
// what they produce.
//
// Node numbering (Section 2.1, 0-based): tips 0..N-1, internal nodes
// N..2N-2, root 2N-2; branch b joins node b to its parent.
#pragma once

#include <cstddef>
#include <vector>

namespace pg {

// Patterns per tile: one tile is TP consecutive patterns of one rate
// category.  A node's data for one tile, M states x TP patterns, is one
// contiguous run (512 B for FP64 and M = 4).
constexpr int TP = 16;

// Clade walks (small M, FP64 and FP32): the maximal subtrees below the root
// with at most a cap of internal nodes (chosen per tree, at most CLADE_CAP)
// are walked depth first, each by one node slot, with a per-slot LDS stack;
// the other internal nodes (the top) keep the level-synchronous walk.
// Entry flags of a clade walk:
#ifndef PG_CLADE_CAP
#define PG_CLADE_CAP 64
#endif
constexpr int CLADE_CAP = PG_CLADE_CAP;
constexpr int CL_STACK = 1;  // post: push the node's message; pre: pop its q
constexpr int CL_ROOT = 2;   // clade root: pre reads its q from memory
// LDS budget of the clade stacks of one workgroup, and of a traversal
// workgroup's dynamic LDS in all (the schedule is left in memory beyond it).
#ifndef PG_CLADE_STACK_MAX
#define PG_CLADE_STACK_MAX 32768
#endif
constexpr int CLADE_STACK_MAX = PG_CLADE_STACK_MAX;
constexpr int LDS_BLOCK_MAX = 61440;
// The schedule is staged in LDS when it fits this budget (bytes).
constexpr int SCHED_LDS_MAX = 32768;
// LDS budget for the pre-order top region's q vectors, and the largest
// level it admits (one node per node slot).
constexpr int TOP_LDS_MAX = 32768;
constexpr int TOP_LEVEL_MAX_NODES = 16;
// Top nodes per node slot of the top-level launches next to the clade
// launches (node i of the top goes to slot i % slots).
constexpr int TOP_J = 4;

// A schedule entry; the same layout as the device's int4.
struct Ent {
    int x, y, z, w;
};
// The two children of an internal node (x first, y second).
struct Kids {
    int x, y;
};

// Internal nodes grouped by height (tips have height 0); nodes of one level
// have no ancestor relation, so a level is processed in parallel and the
// levels in increasing order form a post-order (decreasing: a pre-order).
struct TreeLevels {
    std::vector<int> level_off;    // [H + 1]; level h (height h + 1) is level_nodes[off[h], off[h+1])
    std::vector<int> level_nodes;  // [N - 1]
    std::vector<int> height;       // [2N - 1]
};
void build_levels(int n_tips, const Kids* children, TreeLevels& out);

// What the traversal kernels need from the host.
struct PlanParams {
    int n_states = 4;
    int elem_bytes = 8;     // bytes per partial-vector entry (8 FP64, 4 FP32)
    bool clades = false;    // depth-first clade walks (row-distributed small M)
    bool top_region = true; // pre-order top region in LDS
    int ns_post = 16;       // node slots of the post-order kernel
    int ns_pre = 16;        // node slots of the pre-order kernel
};

struct TraversalPlan {
    // sched = [top entries, by level][post clade list][pre clade list unless
    // one_list]; a top entry is {node, child 0, child 1, region slots} with
    // 1-based top-region slots packed in w (bits 0-7 node, 8-15 child 0,
    // 16-23 child 1, 0 = outside); a clade entry is {node, first child,
    // second child, CL_* flags}, in post order within its clade (the child
    // with more internal nodes first), clades grouped by node slot.
    std::vector<Ent> sched;
    std::vector<int> level_off;  // [H + 1] offsets of the top levels into sched
    std::vector<int> cl_off;     // [ns_post + 1] post slot ranges, then [ns_pre + 1] pre ranges
    int n_top = 0;               // top entries
    int n_cl = 0;                // entries per clade list (0: no clades)
    int depth = 0;               // stack blocks (M x TP) per node slot
    int cap = 0;                 // clade cap chosen (0: none)
    int ns_post = 0, ns_pre = 0;
    bool one_list = true;        // both kernels walk the same clade list
    int top_level = 0;           // first level of the pre-order top region (H: none)
    int top_nodes = 0;           // nodes in the top region
    int n_levels() const { return (int)level_off.size() - 1; }
};

// Plans the traversal of the tree (parent[2N-1], children[2N-1] with the
// internal nodes' entries set, lv from build_levels).  With p.clades the
// clade cap is chosen among 64, 48, 32, 24 and 16 (not above CLADE_CAP) by a
// cost estimate: the busiest pre-order slot's clade entries plus twice the
// top's level iterations; caps whose stacks exceed CLADE_STACK_MAX are
// skipped.
void plan_traversal(int n_tips, const int* parent, const Kids* children, const TreeLevels& lv,
                    const PlanParams& p, TraversalPlan& out);

// Dirty-path schedule of a partial re-evaluation after changing the lengths
// of branches[0..n): each changed internal node (its message changes with
// its transition matrix) and every ancestor of a changed branch, by level of
// the whole tree.  list: the distinct changed branches (transition matrices
// to recompute); sched: {node, child 0, child 1, 0} of the dirty nodes in
// increasing height; level_off[H + 1] into sched.
struct UpdatePlan {
    std::vector<int> list;
    std::vector<Ent> sched;
    std::vector<int> level_off;
};
void plan_update(int n_tips, const int* parent, const Kids* children, const TreeLevels& lv, int n,
                 const int* branches, UpdatePlan& out);

}  // namespace pg

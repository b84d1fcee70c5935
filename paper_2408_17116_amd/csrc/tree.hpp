// Cluster tree and block cluster tree (Sec. III, eq. 21), built on the host.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

namespace cbie {

struct Cluster {
    int p0 = 0, p1 = 0;          // patch range in tree order
    int node0 = 0, nodes = 0;    // node range in tree order
    int obj = 0;
    int level = 0;
    int child[2] = {-1, -1};
    int upn = 2;                 // unknowns per node
    double bmin[3], bmax[3];     // bounding box of the cluster's nodes
    // unknown range set explicitly (component-wise ordering); -1: the
    // node range times all components of a node, interleaved
    int64_t u0 = -1, nu = -1;
    bool leaf() const { return child[0] < 0; }
    int64_t unk0() const { return u0 >= 0 ? u0 : upn * (int64_t)node0; }
    int64_t nunk() const { return nu >= 0 ? nu : upn * (int64_t)nodes; }
};

enum BlockType { BLK_DENSE = 0, BLK_LR = 1, BLK_HIER = 2 };

struct Block {
    int t = -1, s = -1;          // row / column cluster
    int type = BLK_DENSE;
    int child[4] = {-1, -1, -1, -1};   // (t1,s1), (t1,s2), (t2,s1), (t2,s2)
    int leaf_index = -1;         // index into the dense or low-rank list
};

struct TreeInput {
    int n_patches;
    std::vector<int> patch_obj;             // per original patch
    std::vector<int> patch_nodes;           // nodes per patch (q^2)
    std::vector<std::array<double, 3>> centroid;   // per patch: mean of its nodes
    std::vector<std::array<double, 6>> pbox;       // per patch: node bounding box
    // near sets per patch: original patch indices near to some node of the patch
    std::vector<std::vector<int>> near_patches;
    int n_objs;
    int upn = 2;                            // unknowns per node
};

struct Tree {
    std::vector<Cluster> clusters;
    std::vector<int> roots;                  // one root cluster per object
    std::vector<int> patch_order;            // tree position -> original patch
    std::vector<int> patch_pos;              // original patch -> tree position
    std::vector<int> patch_node0;            // tree position -> first tree node
    std::vector<Block> blocks;
    std::vector<int> block_roots;            // per object: root block (root, root)
    std::vector<int> dense_blocks, lr_blocks;   // block ids
    int n_leaves = 0;
};

// Patch-atomic recursive bisection: a cluster is split along the longest
// axis of its node bounding box at the median patch centroid (stable order,
// ties by original index) until it holds <= leaf_unknowns unknowns or one
// patch.  Block tree: (t, s) is a low-rank leaf when
// min(diam_t, diam_s) <= eta dist(t, s) (diam: box diagonal, dist: box gap)
// and no near pair connects t to s; otherwise a dense leaf when t or s is a
// leaf cluster, otherwise split into the four child pairs.
Tree build_tree(const TreeInput& in, int leaf_unknowns, double eta);

// Component-wise block structure (Sec. III-A, eqs. 22-23) derived from a
// node tree T with upn components per node.  Per object the unknowns are
// ordered component by component: component a of tree node i of an object
// whose nodes are [n0, n0 + n) in tree order sits at upn n0 + a n + (i - n0).
// Each component has its own copy of the object's cluster tree (upn = 1);
// the object's root splits the components in halves down to single ones
// (MFIE: u | v; N-Mueller: (Ju Jv) | (Mu Mv), then each pair), and the root
// block splits the same way into the upn^2 component interaction blocks,
// each the node block tree of the object with the same admissibility.
// dense_src / lr_src give, per leaf of the result, the leaf of T it is
// taken from and its row and column components.
struct ComponentTree {
    Tree tree;
    std::vector<std::array<int, 3>> dense_src, lr_src;
};
ComponentTree component_tree(const Tree& T, int upn);

}  // namespace cbie

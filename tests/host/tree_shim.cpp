// Test shim: flat-array access to the library's host tree builder, built
// with the host compiler by the CPU tests (no device code involved).
#include <array>
#include <vector>

#include "tree.hpp"

extern "C" int tree_leaves(int n_patches, int n_objs, int upn, const int* patch_obj, const int* patch_nodes,
                           const double* centroid, const double* pbox, const int* near_ptr, const int* near_idx,
                           int leaf_unknowns, double eta, int* patch_order, int* blocks, int cap) {
    cbie::TreeInput in;
    in.n_patches = n_patches;
    in.n_objs = n_objs;
    in.upn = upn;
    in.patch_obj.assign(patch_obj, patch_obj + n_patches);
    in.patch_nodes.assign(patch_nodes, patch_nodes + n_patches);
    in.centroid.resize(n_patches);
    in.pbox.resize(n_patches);
    in.near_patches.resize(n_patches);
    for (int p = 0; p < n_patches; ++p) {
        for (int d = 0; d < 3; ++d) in.centroid[p][d] = centroid[3 * p + d];
        for (int d = 0; d < 6; ++d) in.pbox[p][d] = pbox[6 * p + d];
        in.near_patches[p].assign(near_idx + near_ptr[p], near_idx + near_ptr[p + 1]);
    }
    const cbie::Tree T = cbie::build_tree(in, leaf_unknowns, eta);
    for (int i = 0; i < n_patches; ++i) patch_order[i] = T.patch_order[i];
    // leaf blocks, depth first: (kind 1 = low-rank / 0 = dense, t.p0, t.p1, s.p0, s.p1)
    int n = 0;
    std::vector<int> stack;
    for (int o = (int)T.block_roots.size() - 1; o >= 0; --o) stack.push_back(T.block_roots[o]);
    while (!stack.empty()) {
        const cbie::Block& b = T.blocks[stack.back()];
        stack.pop_back();
        if (b.type == cbie::BLK_HIER) {
            for (int k = 3; k >= 0; --k) stack.push_back(b.child[k]);
            continue;
        }
        if (n >= cap) return -1;
        const cbie::Cluster& t = T.clusters[b.t];
        const cbie::Cluster& s = T.clusters[b.s];
        int* o = blocks + 5 * n++;
        o[0] = b.type == cbie::BLK_LR ? 1 : 0;
        o[1] = t.p0;
        o[2] = t.p1;
        o[3] = s.p0;
        o[4] = s.p1;
    }
    return n;
}

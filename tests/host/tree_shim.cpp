// Test shim: flat-array access to the library's host tree builder, built
// with the host compiler by the CPU tests (no device code involved).
#include <array>
#include <vector>

#include "tree.hpp"

static cbie::TreeInput make_input(int n_patches, int n_objs, int upn, const int* patch_obj, const int* patch_nodes,
                                  const double* centroid, const double* pbox, const int* near_ptr,
                                  const int* near_idx) {
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
    return in;
}

// Component-wise structure of the tree: its leaf blocks, depth first, as
// (kind, row unknown 0, rows, column unknown 0, columns, source leaf kind,
// source row node 0, source row nodes, source column node 0, source column
// nodes, row component, column component, diagonal).  Returns -2 when a
// hierarchical block's children do not match its clusters' children or a
// cluster's children do not split its unknown range in two.
extern "C" int component_leaves(int n_patches, int n_objs, int upn, const int* patch_obj, const int* patch_nodes,
                                const double* centroid, const double* pbox, const int* near_ptr, const int* near_idx,
                                int leaf_unknowns, double eta, int* out, int cap) {
    const cbie::Tree T = cbie::build_tree(
        make_input(n_patches, n_objs, upn, patch_obj, patch_nodes, centroid, pbox, near_ptr, near_idx), leaf_unknowns,
        eta);
    const cbie::ComponentTree CT = cbie::component_tree(T, upn);
    const cbie::Tree& C = CT.tree;
    for (const auto& k : C.clusters) {
        if (k.leaf()) continue;
        const auto &a = C.clusters[k.child[0]], &b = C.clusters[k.child[1]];
        if (a.unk0() != k.unk0() || b.unk0() != a.unk0() + a.nunk() || a.nunk() + b.nunk() != k.nunk()) return -2;
    }
    for (const auto& b : C.blocks) {
        if (b.type != cbie::BLK_HIER) continue;
        const auto &t = C.clusters[b.t], &s = C.clusters[b.s];
        for (int q = 0; q < 4; ++q) {
            const auto& ch = C.blocks[b.child[q]];
            if (ch.t != t.child[q / 2] || ch.s != s.child[q % 2]) return -2;
        }
    }
    int n = 0;
    std::vector<int> stack;
    for (int o = (int)C.block_roots.size() - 1; o >= 0; --o) stack.push_back(C.block_roots[o]);
    while (!stack.empty()) {
        const cbie::Block& b = C.blocks[stack.back()];
        stack.pop_back();
        if (b.type == cbie::BLK_HIER) {
            for (int k = 3; k >= 0; --k) stack.push_back(b.child[k]);
            continue;
        }
        if (n >= cap) return -1;
        const cbie::Cluster& t = C.clusters[b.t];
        const cbie::Cluster& s = C.clusters[b.s];
        const bool lr = b.type == cbie::BLK_LR;
        const auto& src = lr ? CT.lr_src[b.leaf_index] : CT.dense_src[b.leaf_index];
        const int sid = lr ? T.lr_blocks[src[0]] : T.dense_blocks[src[0]];
        const cbie::Block& sb = T.blocks[sid];
        const cbie::Cluster& st = T.clusters[sb.t];
        const cbie::Cluster& ss = T.clusters[sb.s];
        int* o = out + 13 * n++;
        o[0] = lr ? 1 : 0;
        o[1] = (int)t.unk0();
        o[2] = (int)t.nunk();
        o[3] = (int)s.unk0();
        o[4] = (int)s.nunk();
        o[5] = sb.type == cbie::BLK_LR ? 1 : 0;
        o[6] = st.node0;
        o[7] = st.nodes;
        o[8] = ss.node0;
        o[9] = ss.nodes;
        o[10] = src[1];
        o[11] = src[2];
        o[12] = b.t == b.s ? 1 : 0;
    }
    return n;
}

extern "C" int tree_leaves(int n_patches, int n_objs, int upn, const int* patch_obj, const int* patch_nodes,
                           const double* centroid, const double* pbox, const int* near_ptr, const int* near_idx,
                           int leaf_unknowns, double eta, int* patch_order, int* blocks, int cap) {
    const cbie::Tree T = cbie::build_tree(
        make_input(n_patches, n_objs, upn, patch_obj, patch_nodes, centroid, pbox, near_ptr, near_idx), leaf_unknowns,
        eta);
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

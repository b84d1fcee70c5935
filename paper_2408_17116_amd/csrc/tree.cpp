// Host construction of the cluster tree and the block cluster tree.
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>

namespace cbie {

namespace {

double box_diam(const Cluster& c) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) s += (c.bmax[d] - c.bmin[d]) * (c.bmax[d] - c.bmin[d]);
    return std::sqrt(s);
}

double box_dist(const Cluster& a, const Cluster& b) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double g = std::max(0.0, std::max(a.bmin[d] - b.bmax[d], b.bmin[d] - a.bmax[d]));
        s += g * g;
    }
    return std::sqrt(s);
}

}  // namespace

Tree build_tree(const TreeInput& in, int leaf_unknowns, double eta) {
    Tree T;
    T.patch_order.reserve(in.n_patches);
    std::vector<std::vector<int>> obj_patches(in.n_objs);
    for (int p = 0; p < in.n_patches; ++p) obj_patches[in.patch_obj[p]].push_back(p);

    // recursive bisection; emits leaves in order, so patch order = DFS order
    std::function<int(std::vector<int>&, int, int)> rec = [&](std::vector<int>& ps, int obj, int level) -> int {
        Cluster c;
        c.obj = obj;
        c.level = level;
        c.upn = in.upn;
        int nodes = 0;
        for (int d = 0; d < 3; ++d) { c.bmin[d] = 1e300; c.bmax[d] = -1e300; }
        for (int p : ps) {
            nodes += in.patch_nodes[p];
            for (int d = 0; d < 3; ++d) {
                c.bmin[d] = std::min(c.bmin[d], in.pbox[p][d]);
                c.bmax[d] = std::max(c.bmax[d], in.pbox[p][3 + d]);
            }
        }
        c.nodes = nodes;
        const int id = (int)T.clusters.size();
        T.clusters.push_back(c);
        if ((int64_t)in.upn * nodes <= leaf_unknowns || ps.size() == 1) {
            Cluster& cc = T.clusters[id];
            cc.p0 = (int)T.patch_order.size();
            for (int p : ps) T.patch_order.push_back(p);
            cc.p1 = (int)T.patch_order.size();
            T.n_leaves++;
            return id;
        }
        int ax = 0;
        double ext = -1.0;
        for (int d = 0; d < 3; ++d) {
            double e = c.bmax[d] - c.bmin[d];
            if (e > ext) { ext = e; ax = d; }
        }
        std::stable_sort(ps.begin(), ps.end(), [&](int a, int b) {
            if (in.centroid[a][ax] != in.centroid[b][ax]) return in.centroid[a][ax] < in.centroid[b][ax];
            return a < b;
        });
        std::vector<int> left(ps.begin(), ps.begin() + ps.size() / 2);
        std::vector<int> right(ps.begin() + ps.size() / 2, ps.end());
        const int p0 = (int)T.patch_order.size();
        int c0 = rec(left, obj, level + 1);
        int c1 = rec(right, obj, level + 1);
        Cluster& cc = T.clusters[id];
        cc.child[0] = c0;
        cc.child[1] = c1;
        cc.p0 = p0;
        cc.p1 = (int)T.patch_order.size();
        return id;
    };
    for (int o = 0; o < in.n_objs; ++o) {
        std::vector<int> ps = obj_patches[o];
        T.roots.push_back(rec(ps, o, 0));
    }
    // tree positions and node offsets
    T.patch_pos.assign(in.n_patches, -1);
    T.patch_node0.assign(in.n_patches + 1, 0);
    for (int pos = 0; pos < in.n_patches; ++pos) {
        T.patch_pos[T.patch_order[pos]] = pos;
        T.patch_node0[pos + 1] = T.patch_node0[pos] + in.patch_nodes[T.patch_order[pos]];
    }
    for (auto& c : T.clusters) c.node0 = T.patch_node0[c.p0];

    // patch-level near sets in tree positions, sorted
    std::vector<std::vector<int>> near_pos(in.n_patches);
    for (int p = 0; p < in.n_patches; ++p) {
        auto& v = near_pos[T.patch_pos[p]];
        for (int np : in.near_patches[p]) v.push_back(T.patch_pos[np]);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    auto has_near = [&](const Cluster& t, const Cluster& s) {
        for (int P = t.p0; P < t.p1; ++P) {
            const auto& v = near_pos[P];
            auto it = std::lower_bound(v.begin(), v.end(), s.p0);
            if (it != v.end() && *it < s.p1) return true;
        }
        return false;
    };

    std::function<int(int, int)> brec = [&](int t, int s) -> int {
        const Cluster& ct = T.clusters[t];
        const Cluster& cs = T.clusters[s];
        Block b;
        b.t = t;
        b.s = s;
        const int id = (int)T.blocks.size();
        T.blocks.push_back(b);
        const double dist = box_dist(ct, cs);
        const bool adm = dist > 0.0 && std::min(box_diam(ct), box_diam(cs)) <= eta * dist &&
                         !has_near(ct, cs);
        if (adm) {
            T.blocks[id].type = BLK_LR;
            T.blocks[id].leaf_index = (int)T.lr_blocks.size();
            T.lr_blocks.push_back(id);
        } else if (ct.leaf() || cs.leaf()) {
            T.blocks[id].type = BLK_DENSE;
            T.blocks[id].leaf_index = (int)T.dense_blocks.size();
            T.dense_blocks.push_back(id);
        } else {
            T.blocks[id].type = BLK_HIER;
            int k = 0;
            for (int a = 0; a < 2; ++a)
                for (int c = 0; c < 2; ++c) {
                    int ch = brec(ct.child[a], cs.child[c]);
                    T.blocks[id].child[k++] = ch;
                }
        }
        return id;
    };
    for (int o = 0; o < in.n_objs; ++o) T.block_roots.push_back(brec(T.roots[o], T.roots[o]));
    return T;
}

}  // namespace cbie

// Host construction of the cluster tree and the block cluster tree.
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
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

ComponentTree component_tree(const Tree& T, int upn) {
    ComponentTree out;
    Tree& C = out.tree;
    int depth0 = 0;   // levels of the component split above the node trees
    for (int w = upn; w > 1; w /= 2) ++depth0;
    for (size_t o = 0; o < T.roots.size(); ++o) {
        const Cluster& R = T.clusters[T.roots[o]];
        const int64_t base = upn * (int64_t)R.node0;
        // a copy of the object's cluster tree for each component
        std::vector<std::vector<int>> cid(upn, std::vector<int>(T.clusters.size(), -1));
        std::function<int(int, int, int)> copy = [&](int id, int a, int depth) -> int {
            Cluster k = T.clusters[id];
            k.upn = 1;
            k.level = depth;
            k.u0 = base + (int64_t)a * R.nodes + (k.node0 - R.node0);
            k.nu = k.nodes;
            const int nid = (int)C.clusters.size();
            C.clusters.push_back(k);
            cid[a][id] = nid;
            if (!T.clusters[id].leaf()) {
                const int c0 = copy(T.clusters[id].child[0], a, depth + 1);
                const int c1 = copy(T.clusters[id].child[1], a, depth + 1);
                C.clusters[nid].child[0] = c0;
                C.clusters[nid].child[1] = c1;
            }
            return nid;
        };
        for (int a = 0; a < upn; ++a) copy(T.roots[o], a, depth0);
        // cluster of components [lo, hi): a single component is its copy's
        // root, a range is split in halves
        std::map<std::pair<int, int>, int> gid;
        std::function<int(int, int, int)> group = [&](int lo, int hi, int depth) -> int {
            if (hi - lo == 1) return cid[lo][T.roots[o]];
            Cluster k = R;
            k.upn = hi - lo;
            k.level = depth;
            k.u0 = base + (int64_t)lo * R.nodes;
            k.nu = (int64_t)(hi - lo) * R.nodes;
            const int nid = (int)C.clusters.size();
            C.clusters.push_back(k);
            const int mid = (lo + hi) / 2;
            const int c0 = group(lo, mid, depth + 1);
            const int c1 = group(mid, hi, depth + 1);
            C.clusters[nid].child[0] = c0;
            C.clusters[nid].child[1] = c1;
            gid[{lo, hi}] = nid;
            return nid;
        };
        C.roots.push_back(group(0, upn, 0));
        auto cluster_of = [&](int lo, int hi) { return hi - lo == 1 ? cid[lo][T.roots[o]] : gid.at({lo, hi}); };
        // the object's node block tree for row component a, column component b
        std::function<int(int, int, int)> bcopy = [&](int bid, int a, int b) -> int {
            const Block& src = T.blocks[bid];
            Block k;
            k.t = cid[a][src.t];
            k.s = cid[b][src.s];
            k.type = src.type;
            const int nid = (int)C.blocks.size();
            C.blocks.push_back(k);
            if (src.type == BLK_LR) {
                C.blocks[nid].leaf_index = (int)C.lr_blocks.size();
                C.lr_blocks.push_back(nid);
                out.lr_src.push_back({src.leaf_index, a, b});
            } else if (src.type == BLK_DENSE) {
                C.blocks[nid].leaf_index = (int)C.dense_blocks.size();
                C.dense_blocks.push_back(nid);
                out.dense_src.push_back({src.leaf_index, a, b});
            } else {
                for (int q = 0; q < 4; ++q) {
                    const int ch = bcopy(src.child[q], a, b);
                    C.blocks[nid].child[q] = ch;
                }
            }
            return nid;
        };
        // row components [rl, rh) x column components [cl, ch), halved together
        std::function<int(int, int, int, int)> brec = [&](int rl, int rh, int cl, int ch) -> int {
            if (rh - rl == 1) return bcopy(T.block_roots[o], rl, cl);
            Block k;
            k.t = cluster_of(rl, rh);
            k.s = cluster_of(cl, ch);
            k.type = BLK_HIER;
            const int nid = (int)C.blocks.size();
            C.blocks.push_back(k);
            const int rm = (rl + rh) / 2, cm = (cl + ch) / 2;
            const int q0 = brec(rl, rm, cl, cm), q1 = brec(rl, rm, cm, ch);
            const int q2 = brec(rm, rh, cl, cm), q3 = brec(rm, rh, cm, ch);
            Block& B = C.blocks[nid];
            B.child[0] = q0;
            B.child[1] = q1;
            B.child[2] = q2;
            B.child[3] = q3;
            return nid;
        };
        C.block_roots.push_back(brec(0, upn, 0, upn));
    }
    for (const auto& k : C.clusters)
        if (k.leaf()) ++C.n_leaves;
    return out;
}

}  // namespace cbie

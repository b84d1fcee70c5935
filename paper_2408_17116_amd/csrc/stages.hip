// Host orchestration of geometry, near classification, tree, fill and export.
#include <algorithm>
#include <cmath>
#include <map>

#include "ctx.hpp"
#include "rules.hpp"

namespace cbie {

// Tables of all Fejer rules n = 1..kMaxRule, rule n at offset n(n-1)/2.
static const int kMaxRule = 96;
void make_fejer_tables(Ctx& c) {
    std::vector<double> ax, aw, bx, bw, x, w;
    for (int n = 1; n <= kMaxRule; ++n) {
        fejer_rule(n, x, w);
        for (int l = 0; l < n; ++l) {
            ax.push_back(x[l]);
            aw.push_back(w[l]);
            bx.push_back(0.5 * (x[l] + 1.0));
            bw.push_back(0.5 * w[l]);
        }
    }
    c.d_fej11_x.upload(ax, c.stream);
    c.d_fej11_w.upload(aw, c.stream);
    c.d_fej01_x.upload(bx, c.stream);
    c.d_fej01_w.upload(bw, c.stream);
    // differentiation matrices of the interpolant, q = 1..8
    std::vector<double> dm;
    cheb_diff_matrices(8, dm);
    c.d_dmat.upload(dm, c.stream);
}

void stage_build_tree(Ctx& c, int leaf_size, double eta, double delta) {
    const double t0 = now_s();
    const int n = c.n_nodes;
    const int P = (int)c.patches.size();
    c.d_geom.alloc(12 * (size_t)n);
    double* g = c.d_geom.p;
    c.nd = NodeArrays{g, g + n, g + 2 * n, g + 3 * n, g + 4 * n, g + 5 * n, g + 6 * n, g + 7 * n,
                      g + 8 * n, g + 9 * n, g + 10 * n, g + 11 * n};
    k_nodes<<<ceil_div(n, 256), 256, 0, c.stream>>>(c.d_patches.p, c.d_objs.p, c.d_fej11_x.p,
                                                    c.d_fej11_w.p, c.d_node_patch.p, n, c.nd);
    check_launch("k_nodes");
    c.d_patch_info.alloc(5 * (size_t)P);
    k_patch_info<<<ceil_div(P, 128), 128, 0, c.stream>>>(c.d_patches.p, c.d_objs.p, P, c.d_patch_info.p);
    check_launch("k_patch_info");

    // near classification: count, scan, fill (sorted by target then patch)
    DBuf<int> d_cnt;
    d_cnt.alloc(n);
    k_near<<<ceil_div(n, 128), 128, 0, c.stream>>>(c.d_patches.p, c.d_objs.p, c.d_patch_info.p,
                                                   c.d_node_patch.p, c.d_obj_patch0.p, c.d_obj_npatch.p,
                                                   c.nd, n, delta, d_cnt.p, nullptr, nullptr);
    check_launch("k_near count");
    std::vector<int> cnt(n);
    d_cnt.download(cnt.data(), n, c.stream);
    c.sync();
    std::vector<int64_t> off(n + 1, 0);
    for (int i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[i];
    const int64_t npairs = off[n];
    DBuf<int64_t> d_off;
    d_off.upload(off, c.stream);
    c.d_near.alloc(npairs);
    k_near<<<ceil_div(n, 128), 128, 0, c.stream>>>(c.d_patches.p, c.d_objs.p, c.d_patch_info.p,
                                                   c.d_node_patch.p, c.d_obj_patch0.p, c.d_obj_npatch.p,
                                                   c.nd, n, delta, nullptr, d_off.p, c.d_near.p);
    check_launch("k_near fill");
    c.near.resize(npairs);
    c.d_near.download(c.near.data(), npairs, c.stream);
    c.h_r.resize(3 * (size_t)n);
    CBIE_HIP(hipMemcpyAsync(c.h_r.data(), c.nd.rx, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    CBIE_HIP(hipMemcpyAsync(c.h_r.data() + n, c.nd.ry, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    CBIE_HIP(hipMemcpyAsync(c.h_r.data() + 2 * n, c.nd.rz, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();

    // tree input: per patch centroid, node box, near set
    TreeInput in;
    in.n_patches = P;
    in.n_objs = (int)c.objs.size();
    in.patch_obj.resize(P);
    in.patch_nodes.resize(P);
    in.centroid.resize(P);
    in.pbox.resize(P);
    in.near_patches.resize(P);
    for (int p = 0; p < P; ++p) {
        const PatchDev& pd = c.patches[p];
        in.patch_obj[p] = pd.obj;
        in.patch_nodes[p] = pd.q * pd.q;
        std::array<double, 3> cen = {0, 0, 0};
        std::array<double, 6> box = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
        for (int l = 0; l < pd.q * pd.q; ++l) {
            const int i = pd.node0 + l;
            for (int d = 0; d < 3; ++d) {
                const double x = c.h_r[(size_t)d * n + i];
                cen[d] += x;
                box[d] = std::min(box[d], x);
                box[3 + d] = std::max(box[3 + d], x);
            }
        }
        for (int d = 0; d < 3; ++d) cen[d] /= pd.q * pd.q;
        in.centroid[p] = cen;
        in.pbox[p] = box;
    }
    for (const NearPair& e : c.near) in.near_patches[c.node_patch[e.target]].push_back(e.patch);
    in.upn = c.upn;
    c.tree = build_tree(in, leaf_size, eta);
    c.leaf_size = leaf_size;
    c.eta = eta;
    c.delta = delta;
    const Tree& T = c.tree;

    // tree node -> original node
    c.tree_node.resize(n);
    c.orig_to_tree_node.resize(n);
    for (int pos = 0; pos < P; ++pos) {
        const PatchDev& pd = c.patches[T.patch_order[pos]];
        for (int l = 0; l < pd.q * pd.q; ++l) {
            c.tree_node[T.patch_node0[pos] + l] = pd.node0 + l;
            c.orig_to_tree_node[pd.node0 + l] = T.patch_node0[pos] + l;
        }
    }
    c.d_tree_node.upload(c.tree_node, c.stream);

    // dense and low-rank block geometry
    auto mkblk = [&](const Block& b) {
        const Cluster& ct = T.clusters[b.t];
        const Cluster& cs = T.clusters[b.s];
        DenseBlockDev d{};
        d.ld = c.upn * ct.nodes;
        d.upn = c.upn;
        d.row_node0 = ct.node0;
        d.row_nodes = ct.nodes;
        d.col_node0 = cs.node0;
        d.col_nodes = cs.nodes;
        d.obj = ct.obj;
        return d;
    };
    c.dblk.clear();
    int64_t off_d = 0;
    for (int id : T.dense_blocks) {
        DenseBlockDev d = mkblk(T.blocks[id]);
        d.offset = off_d;
        off_d += (int64_t)d.ld * c.upn * d.col_nodes;
        c.dblk.push_back(d);
    }
    c.lblk.clear();
    for (int id : T.lr_blocks) c.lblk.push_back(mkblk(T.blocks[id]));
    c.d_dblk.upload(c.dblk, c.stream);
    c.d_lblk.upload(c.lblk, c.stream);

    // statistics
    cbie_stats& st = c.stats;
    st.n_unknowns = c.n_unk;
    st.n_nodes = n;
    st.n_patches = P;
    st.n_objects = (int64_t)c.objs.size();
    st.n_clusters = (int64_t)T.clusters.size();
    st.n_leaves = T.n_leaves;
    st.n_dense_blocks = (int64_t)T.dense_blocks.size();
    st.n_lr_blocks = (int64_t)T.lr_blocks.size();
    st.n_near_pairs = npairs;
    st.dense_entries = off_d;
    c.sync();
    st.t_tree = now_s() - t0;
}

// Plain-rule N-Mueller entries of the given blocks (host list and its device
// copy; offsets and leading dimensions into dst): tiles of 32 row nodes
// against one source patch.
void fill_blocks_nm(Ctx& c, const std::vector<DenseBlockDev>& blocks, const DenseBlockDev* d_blocks, zd* dst) {
    std::vector<DenseTile> tiles;
    for (int b = 0; b < (int)blocks.size(); ++b) {
        const DenseBlockDev& d = blocks[b];
        const int q = c.objs[d.obj].q;
        for (int r0 = 0; r0 < d.row_nodes; r0 += 32)
            for (int c0 = 0; c0 < d.col_nodes; c0 += q * q) tiles.push_back(DenseTile{b, r0, c0, q});
    }
    if (tiles.empty()) return;
    DBuf<DenseTile> d_tiles;
    d_tiles.upload(tiles, c.stream);
    k_far_fill_nm<double><<<(unsigned)tiles.size(), 256, 0, c.stream>>>(
        d_tiles.p, (int)tiles.size(), d_blocks, c.d_tree_node.p, c.nd, c.d_objs.p, c.d_dmat.p, dst);
    check_launch("k_far_fill_nm");
    c.sync();   // the tile list is released on return
}

void stage_fill(Ctx& c, int n_ang, int n_rad) {
    const double t0 = now_s();
    const Tree& T = c.tree;
    // singular rule of the change of variables
    // default sizes grow with the order above 8: the integrand carries the
    // interpolation basis, a polynomial of degree q - 1 in each direction
    int qmax_rule = 0;
    for (const auto& p : c.patches) qmax_rule = std::max(qmax_rule, p.q);
    QuadRule rule{};
    rule.n_ang = n_ang > 0 ? n_ang : std::max(40, 6 * qmax_rule - 8);
    rule.n_rad = n_rad > 0 ? n_rad : std::max(32, 5 * qmax_rule - 8);
    rule.n_in = std::max(4, (rule.n_rad * 5) / 8);
    rule.n_out = rule.n_rad;
    CBIE_REQUIRE(rule.n_ang <= kMaxRule && rule.n_rad <= kMaxRule, CBIE_EINVAL, "rule size above 96");
    rule.off_ang = rule.n_ang * (rule.n_ang - 1) / 2;
    rule.off_rad = rule.n_rad * (rule.n_rad - 1) / 2;
    rule.off_in = rule.n_in * (rule.n_in - 1) / 2;
    rule.off_out = rule.n_out * (rule.n_out - 1) / 2;

    // 1) near/self integrals, one work-group per pair, in chunks
    const int64_t np = (int64_t)c.near.size();
    int qmax = 0;
    for (const auto& p : c.patches) qmax = std::max(qmax, p.q);
    bool cheb = false;   // any Chebyshev-interpolated patches
    for (const auto& o : c.objs) cheb = cheb || o.deg > 0;
    const int q2 = qmax * qmax;
    const int64_t stride = (int64_t)c.upn * c.upn * q2;   // entries of one (target, patch) pair
    DBuf<zd> vals;
    vals.alloc((size_t)np * stride);
    hipEvent_t e0, e1;
    CBIE_HIP(hipEventCreate(&e0));
    CBIE_HIP(hipEventCreate(&e1));
    CBIE_HIP(hipEventRecord(e0, c.stream));
    const int64_t chunk = 1 << 20;
    for (int64_t p0 = 0; p0 < np; p0 += chunk) {
        const int64_t cnt = std::min(chunk, np - p0);
        if (c.upn == 4) {
            k_quad_nm<<<(unsigned)cnt, 256, 0, c.stream>>>(c.d_patches.p, c.d_objs.p, c.nd, c.d_near.p + p0, cnt,
                                                           c.d_fej11_x.p, c.d_fej01_x.p, c.d_fej01_w.p, c.d_dmat.p,
                                                           rule, stride, vals.p + p0 * stride);
            check_launch("k_quad_nm");
        } else {
            // orders above 8: two nodes per lane (a separate instance keeps
            // the registers of the common case); the Chebyshev-patch
            // geometry only in the instances of contexts that hold such
            // patches
            auto launch = [&](auto kern) {
                kern<<<(unsigned)cnt, 256, 0, c.stream>>>(c.d_patches.p, c.d_objs.p, c.nd, c.d_near.p + p0, cnt,
                                                          c.d_fej11_x.p, c.d_fej01_x.p, c.d_fej01_w.p, rule, stride,
                                                          vals.p + p0 * stride);
            };
            if (qmax <= 8) {
                if (cheb) launch(k_quad<8, true>);
                else launch(k_quad<8, false>);
            } else {
                if (cheb) launch(k_quad<11, true>);
                else launch(k_quad<11, false>);
            }
            check_launch("k_quad");
        }
    }
    CBIE_HIP(hipEventRecord(e1, c.stream));

    // 2) far entries of every dense block
    c.dense.alloc((size_t)c.stats.dense_entries);
    hipEvent_t e2, e3;
    CBIE_HIP(hipEventCreate(&e2));
    CBIE_HIP(hipEventCreate(&e3));
    CBIE_HIP(hipEventRecord(e2, c.stream));
    if (c.upn == 4) {
        fill_blocks_nm(c, c.dblk, c.d_dblk.p, c.dense.p);
    } else {
        std::vector<DenseTile> tiles;
        for (int b = 0; b < (int)c.dblk.size(); ++b) {
            const DenseBlockDev& d = c.dblk[b];
            for (int r0 = 0; r0 < d.row_nodes; r0 += 64)
                for (int c0 = 0; c0 < d.col_nodes; c0 += 16) tiles.push_back(DenseTile{b, r0, c0, 0});
        }
        DBuf<DenseTile> d_tiles;
        d_tiles.upload(tiles, c.stream);
        if (!tiles.empty()) {
            k_far_fill<double><<<(unsigned)tiles.size(), 256, 0, c.stream>>>(
                d_tiles.p, (int)tiles.size(), c.d_dblk.p, c.d_tree_node.p, c.nd, c.d_objs.p, c.dense.p);
            check_launch("k_far_fill");
        }
    }
    CBIE_HIP(hipEventRecord(e3, c.stream));

    // 3) overwrite near/self entries: destination block of each pair
    // (row leaf cluster of the target, column range holding the patch)
    std::vector<int> node_leaf(c.n_nodes, -1);   // tree node -> leaf cluster
    for (int ci = 0; ci < (int)T.clusters.size(); ++ci) {
        const Cluster& cl = T.clusters[ci];
        if (!cl.leaf()) continue;
        for (int t = 0; t < cl.nodes; ++t) node_leaf[cl.node0 + t] = ci;
    }
    // per leaf row cluster: dense blocks whose row range contains it
    std::vector<std::vector<int>> row_blocks(T.clusters.size());
    for (int b = 0; b < (int)c.dblk.size(); ++b) {
        const DenseBlockDev& d = c.dblk[b];
        for (int ci = 0; ci < (int)T.clusters.size(); ++ci) {
            const Cluster& cl = T.clusters[ci];
            if (cl.leaf() && cl.node0 >= d.row_node0 && cl.node0 < d.row_node0 + d.row_nodes)
                row_blocks[ci].push_back(b);
        }
    }
    std::vector<NearDest> dest(np);
    for (int64_t k = 0; k < np; ++k) {
        const NearPair& e = c.near[k];
        const int tn = c.orig_to_tree_node[e.target];
        const int pn0 = c.orig_to_tree_node[c.patches[e.patch].node0];
        const int leaf = node_leaf[tn];
        int found = -1;
        for (int b : row_blocks[leaf]) {
            const DenseBlockDev& d = c.dblk[b];
            if (pn0 >= d.col_node0 && pn0 < d.col_node0 + d.col_nodes) { found = b; break; }
        }
        CBIE_REQUIRE(found >= 0, CBIE_EINTERNAL, "near pair outside every dense block");
        const DenseBlockDev& d = c.dblk[found];
        const int pq = c.patches[e.patch].q;
        dest[k] = NearDest{found, tn - d.row_node0, pn0 - d.col_node0, pq * pq};
    }
    DBuf<NearDest> d_dest;
    d_dest.upload(dest, c.stream);
    if (np > 0) {
        k_near_scatter<double><<<(unsigned)np, 256, 0, c.stream>>>(d_dest.p, np, stride, vals.p, c.d_dblk.p,
                                                                  c.dense.p);
        check_launch("k_near_scatter");
    }
    c.sync();
    float ms = 0.f;
    CBIE_HIP(hipEventElapsedTime(&ms, e0, e1));
    c.stats.quad_seconds = ms * 1e-3;
    CBIE_HIP(hipEventElapsedTime(&ms, e2, e3));
    c.stats.far_fill_seconds = ms * 1e-3;
    (void)hipEventDestroy(e2);
    (void)hipEventDestroy(e3);
    // work of the near quadrature: points of every pair's rule (two Duffy
    // triangles per non-degenerate rectangle around the singular point) and
    // the flops of the basis contraction, the kernel's dominant FP64 term:
    // per point and source node 8 (MFIE) or 32 (N-Mueller) fused
    // multiply-adds
    {
        double pts = 0.0, fl = 0.0;
        for (const NearPair& e : c.near) {
            int ntri = 0;
            for (int iu = 0; iu < 2; ++iu)
                for (int iv = 0; iv < 2; ++iv)
                    if (std::fabs((iu ? 1.0 : -1.0) - e.us) >= 1e-14 && std::fabs((iv ? 1.0 : -1.0) - e.vs) >= 1e-14)
                        ntri += 2;
            const double np_ = (double)ntri * rule.n_ang * (e.self ? rule.n_rad : rule.n_in + rule.n_out);
            const int pq = c.patches[e.patch].q;
            pts += np_;
            fl += np_ * pq * pq * (c.upn == 4 ? 64.0 : 16.0);
        }
        c.stats.quad_points = pts;
        c.stats.quad_flops = fl;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.stats.t_fill = now_s() - t0;
}

void stage_export_dense(Ctx& c, zd* A, long ld) {
    CBIE_HIP(hipMemsetAsync(A, 0, sizeof(zd) * (size_t)ld * c.n_unk, c.stream));
    if (!c.dblk.empty()) {
        dim3 grid(64, (unsigned)c.dblk.size());
        k_export_dense_block<<<grid, 256, 0, c.stream>>>(c.d_dblk.p, (int)c.dblk.size(), c.d_tree_node.p,
                                                         c.dense.p, A, ld);
        check_launch("k_export_dense_block");
    }
    if (!c.lblk.empty()) {
        if (c.state >= ST_COMPRESSED) {
            void export_lowrank(Ctx & c, zd * A, long ld);
            export_lowrank(c, A, ld);
        } else if (c.upn == 4) {
            // plain-rule entries of each admissible block, through a dense copy
            for (const DenseBlockDev& d0 : c.lblk) {
                DenseBlockDev d = d0;
                d.offset = 0;
                d.ld = c.upn * d.row_nodes;
                DBuf<zd> tmp;
                tmp.alloc((size_t)d.ld * c.upn * d.col_nodes);
                DBuf<DenseBlockDev> d_b;
                std::vector<DenseBlockDev> one{d};
                d_b.upload(one, c.stream);
                fill_blocks_nm(c, one, d_b.p, tmp.p);
                k_export_dense_block<<<dim3(64, 1), 256, 0, c.stream>>>(d_b.p, 1, c.d_tree_node.p, tmp.p, A, ld);
                check_launch("k_export_dense_block");
                c.sync();
            }
        } else {
            dim3 grid(64, (unsigned)c.lblk.size());
            k_export_far<<<grid, 256, 0, c.stream>>>(c.d_lblk.p, (int)c.lblk.size(), c.d_tree_node.p, c.nd,
                                                     c.d_objs.p, A, ld);
            check_launch("k_export_far");
        }
    }
    c.sync();
}

}  // namespace cbie

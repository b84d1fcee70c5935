// C-ABI entry points: argument checks, state machine, error capture.
#include <cmath>
#include <cstring>

#include "ctx.hpp"
#include "mlp.hpp"
#include "ops.hpp"

struct cbie_ctx {
    cbie::Ctx c;
};

namespace cbie {
void make_fejer_tables(Ctx& c);
}

using namespace cbie;

template <typename F> static cbie_status guarded(cbie_ctx* ctx, F&& f) {
    if (!ctx) return CBIE_EINVAL;
    try {
        CBIE_HIP(hipSetDevice(ctx->c.device));
        f(ctx->c);
        ctx->c.err.clear();
        return CBIE_OK;
    } catch (const Error& e) {
        ctx->c.err = e.msg;
        // a failed kernel leaves the stream in an error state: report it
        (void)hipStreamSynchronize(ctx->c.stream);
        return (cbie_status)e.code;
    } catch (const std::bad_alloc&) {
        ctx->c.err = "host allocation failed";
        return CBIE_ENOMEM;
    } catch (const std::exception& e) {
        ctx->c.err = std::string("internal: ") + e.what();
        return CBIE_EINTERNAL;
    }
}

// entry points on a bare stream: no context holds an error message
template <typename F> static cbie_status guarded_stream(F&& f) {
    try {
        f();
        return CBIE_OK;
    } catch (const Error& e) {
        return (cbie_status)e.code;
    } catch (const std::bad_alloc&) {
        return CBIE_ENOMEM;
    } catch (const std::exception&) {
        return CBIE_EINTERNAL;
    }
}

extern "C" {

cbie_status cbie_create(const cbie_object* objs, int n_objs, void* hip_stream, cbie_ctx** out) {
    if (!out || !objs || n_objs <= 0) return CBIE_EINVAL;
    *out = nullptr;
    for (int o = 0; o < n_objs; ++o) {
        const cbie_object& ob = objs[o];
        if (ob.form != CBIE_MFIE_PEC && ob.form != CBIE_NMULLER) return CBIE_EINVAL;
        if (ob.form != objs[0].form) return CBIE_EINVAL;
        if (ob.form == CBIE_NMULLER &&
            !(ob.eps_r > 0 && ob.mu_r > 0 && std::isfinite(ob.eps_r) && std::isfinite(ob.mu_r)))
            return CBIE_EINVAL;
        if (!(ob.k0 > 0) || ob.q < 2 || ob.q > 11 || ob.n_patches <= 0) return CBIE_EINVAL;
        if (ob.form == CBIE_NMULLER && ob.q > 8) return CBIE_EINVAL;
        if (ob.patch_degree != 0) {
            if (ob.patch_degree < 1 || ob.patch_degree > kChebMaxDeg || !ob.patch_coeffs) return CBIE_EINVAL;
            const int64_t nc = (int64_t)ob.n_patches * 3 * (ob.patch_degree + 1) * (ob.patch_degree + 1);
            for (int64_t e = 0; e < nc; ++e)
                if (!std::isfinite(ob.patch_coeffs[e])) return CBIE_EINVAL;
            continue;
        }
        if (!ob.patches) return CBIE_EINVAL;
        for (int d = 0; d < 3; ++d)
            if (!(ob.axes[d] > 0)) return CBIE_EINVAL;
        for (int p = 0; p < ob.n_patches; ++p) {
            const cbie_patch& pt = ob.patches[p];
            if (pt.face < 0 || pt.face > 5 || pt.split < 1 || pt.i < 0 || pt.j < 0 || pt.i >= pt.split ||
                pt.j >= pt.split)
                return CBIE_EINVAL;
        }
    }
    cbie_ctx* ctx = nullptr;
    try {
        ctx = new cbie_ctx();
    } catch (...) {
        return CBIE_ENOMEM;
    }
    // the context lives on the caller's current device
    if (hipGetDevice(&ctx->c.device) != hipSuccess) {
        delete ctx;
        return CBIE_EHIP;
    }
    cbie_status st = guarded(ctx, [&](Ctx& c) {
        c.stream = (hipStream_t)hip_stream;
        int node = 0;
        std::vector<int64_t> coef_off(n_objs, -1);
        std::vector<double> coef;
        for (int o = 0; o < n_objs; ++o) {
            const cbie_object& ob = objs[o];
            const bool cheb = ob.patch_degree > 0;
            ObjDev od{};
            for (int d = 0; d < 3; ++d) { od.axes[d] = cheb ? 1.0 : ob.axes[d]; od.center[d] = cheb ? 0.0 : ob.center[d]; }
            od.k0 = ob.k0;
            od.q = ob.q;
            od.form = ob.form;
            od.eps_r = ob.form == CBIE_NMULLER ? ob.eps_r : 1.0;
            od.mu_r = ob.form == CBIE_NMULLER ? ob.mu_r : 1.0;
            od.deg = cheb ? ob.patch_degree : 0;
            if (cheb) {
                coef_off[o] = (int64_t)coef.size();
                coef.insert(coef.end(), ob.patch_coeffs,
                            ob.patch_coeffs + (size_t)ob.n_patches * 3 * (ob.patch_degree + 1) * (ob.patch_degree + 1));
            }
            c.objs.push_back(od);
            c.obj_patch0.push_back((int)c.patches.size());
            c.obj_npatch.push_back(ob.n_patches);
            c.obj_node0.push_back(node);
            for (int p = 0; p < ob.n_patches; ++p) {
                PatchDev pd{};
                if (cheb) {
                    pd.face = -1;
                    pd.i = p;
                } else {
                    pd.face = ob.patches[p].face;
                    pd.i = ob.patches[p].i;
                    pd.j = ob.patches[p].j;
                    pd.split = ob.patches[p].split;
                }
                pd.obj = o;
                pd.node0 = node;
                pd.q = ob.q;
                for (int l = 0; l < ob.q * ob.q; ++l) c.node_patch.push_back((int)c.patches.size());
                node += ob.q * ob.q;
                c.patches.push_back(pd);
            }
            c.obj_nodes.push_back(node - c.obj_node0.back());
        }
        CBIE_REQUIRE(node < (1 << 30), CBIE_EINVAL, "too many nodes");
        c.n_nodes = node;
        c.upn = objs[0].form == CBIE_NMULLER ? 4 : 2;
        c.n_unk = c.upn * (int64_t)node;
        if (!coef.empty()) {
            c.d_coef.upload(coef, c.stream);
            for (int o = 0; o < n_objs; ++o)
                if (coef_off[o] >= 0) c.objs[o].coef = c.d_coef.p + coef_off[o];
        }
        c.d_patches.upload(c.patches, c.stream);
        c.d_objs.upload(c.objs, c.stream);
        c.d_node_patch.upload(c.node_patch, c.stream);
        c.d_obj_patch0.upload(c.obj_patch0, c.stream);
        c.d_obj_npatch.upload(c.obj_npatch, c.stream);
        make_fejer_tables(c);
        resolve_scratch(c.device);
        c.sync();
        c.state = ST_CREATED;
    });
    if (st != CBIE_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return CBIE_OK;
}

cbie_status cbie_build_tree(cbie_ctx* ctx, int leaf_size, double eta, double near_delta) {
    return guarded(ctx, [&](Ctx& c) {
        int qmax = 0;
        for (const auto& o : c.objs) qmax = std::max(qmax, o.q);
        CBIE_REQUIRE(leaf_size >= c.upn * qmax * qmax && leaf_size <= 256 && eta > 0 && near_delta > 0,
                     CBIE_EINVAL, "leaf_size outside [unknowns of one patch, 256], eta <= 0 or near_delta <= 0");
        c.hm.reset();
        c.state = ST_CREATED;   // a stage that fails part-way must be redone
        stage_build_tree(c, leaf_size, eta, near_delta);
        c.state = ST_TREE;
    });
}

cbie_status cbie_fill(cbie_ctx* ctx, int n_ang, int n_rad) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_TREE, CBIE_ESTATE, "fill before build_tree");
        CBIE_REQUIRE(n_ang >= 0 && n_rad >= 0, CBIE_EINVAL, "negative rule size");
        c.hm.reset();
        c.state = ST_TREE;
        stage_fill(c, n_ang, n_rad);
        c.state = ST_FILLED;
    });
}

cbie_status cbie_compress(cbie_ctx* ctx, double aca_tol, cbie_rank_mode mode) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_FILLED, CBIE_ESTATE, "compress before fill");
        CBIE_REQUIRE(aca_tol > 0 && aca_tol < 1, CBIE_EINVAL, "aca_tol outside (0, 1)");
        CBIE_REQUIRE(mode == CBIE_RANK_ADAPTIVE || mode == CBIE_RANK_PREDICTED, CBIE_EINVAL, "rank mode");
        c.hm.reset();
        c.state = ST_FILLED;
        stage_compress(c, aca_tol, (int)mode);
        c.state = ST_COMPRESSED;
    });
}

cbie_status cbie_factor(cbie_ctx* ctx, cbie_precision prec) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_COMPRESSED, CBIE_ESTATE, "factor before compress");
        CBIE_REQUIRE(prec == CBIE_PREC_C128 || prec == CBIE_PREC_C64_IR, CBIE_EINVAL, "precision");
        c.state = ST_COMPRESSED;
        stage_factor(c, (int)prec);
        c.state = ST_FACTORED;
    });
}

cbie_status cbie_set_factor_tolerance(cbie_ctx* ctx, double tol) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(tol >= 0 && tol < 1, CBIE_EINVAL, "factor tolerance outside [0, 1)");
        c.factor_tol = tol;
    });
}

cbie_status cbie_set_factor_ordering(cbie_ctx* ctx, cbie_ordering ordering) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(ordering == CBIE_ORDER_ENTIRE || ordering == CBIE_ORDER_COMPONENT, CBIE_EINVAL, "ordering");
        c.factor_ordering = (int)ordering;
    });
}

cbie_status cbie_solve(cbie_ctx* ctx, int nrhs, const void* b_dev, void* x_dev, long ld, double ir_tol,
                       int ir_maxit, int* ir_iters_out) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_FACTORED, CBIE_ESTATE, "solve before factor");
        CBIE_REQUIRE(nrhs > 0 && b_dev && x_dev && ld >= c.n_unk && b_dev != x_dev && ir_maxit >= 0,
                     CBIE_EINVAL, "solve arguments");
        stage_solve(c, nrhs, (const zd*)b_dev, (zd*)x_dev, ld, ir_tol, ir_maxit, ir_iters_out);
    });
}

cbie_status cbie_solve_gmres(cbie_ctx* ctx, int nrhs, const void* b_dev, void* x_dev, long ld, double tol,
                             int restart, int maxit, int* iters_out) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_FACTORED, CBIE_ESTATE, "solve before factor");
        CBIE_REQUIRE(nrhs > 0 && b_dev && x_dev && ld >= c.n_unk && b_dev != x_dev && restart > 0 && maxit >= 0 &&
                         tol > 0,
                     CBIE_EINVAL, "solve_gmres arguments");
        stage_solve_gmres(c, nrhs, (const zd*)b_dev, (zd*)x_dev, ld, tol, restart, maxit, iters_out);
    });
}

cbie_status cbie_matvec(cbie_ctx* ctx, int nrhs, const void* x_dev, void* y_dev, long ld) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_COMPRESSED, CBIE_ESTATE, "matvec before compress");
        CBIE_REQUIRE(nrhs > 0 && x_dev && y_dev && ld >= c.n_unk && x_dev != y_dev, CBIE_EINVAL,
                     "matvec arguments");
        stage_matvec(c, nrhs, (const zd*)x_dev, (zd*)y_dev, ld);
    });
}

cbie_status cbie_matvec_noalloc(cbie_ctx* ctx, int nrhs, const void* x_dev, void* y_dev, long ld) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_COMPRESSED, CBIE_ESTATE, "matvec before compress");
        CBIE_REQUIRE(nrhs > 0 && x_dev && y_dev && ld >= c.n_unk && x_dev != y_dev, CBIE_EINVAL,
                     "matvec arguments");
        stage_matvec_noalloc(c, nrhs, (const zd*)x_dev, (zd*)y_dev, ld);
    });
}

cbie_status cbie_rhs_planewave(cbie_ctx* ctx, int nw, const double* khat, const double* pol, void* b_dev,
                               long ld) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_TREE, CBIE_ESTATE, "rhs before build_tree");
        CBIE_REQUIRE(nw > 0 && khat && pol && b_dev && ld >= c.n_unk, CBIE_EINVAL, "rhs arguments");
        stage_rhs(c, nw, khat, pol, (zd*)b_dev, ld);
    });
}

cbie_status cbie_rhs_dipole(cbie_ctx* ctx, int n_dipoles, const double* pos, const double* moment, void* b_dev,
                            long ld) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_TREE, CBIE_ESTATE, "rhs before build_tree");
        CBIE_REQUIRE(n_dipoles > 0 && pos && moment && b_dev && ld >= c.n_unk, CBIE_EINVAL, "dipole rhs arguments");
        stage_rhs_dipole(c, n_dipoles, pos, moment, (zd*)b_dev, ld);
    });
}

cbie_status cbie_farfield(cbie_ctx* ctx, int nrhs, const void* x_dev, long ld, int ndir, const double* rhat,
                          void* E_out) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_TREE, CBIE_ESTATE, "farfield before build_tree");
        CBIE_REQUIRE(nrhs > 0 && x_dev && ld >= c.n_unk && ndir > 0 && rhat && E_out, CBIE_EINVAL,
                     "farfield arguments");
        stage_farfield(c, nrhs, (const zd*)x_dev, ld, ndir, rhat, (zd*)E_out);
    });
}

cbie_status cbie_get_stats(cbie_ctx* ctx, void* stats_out, size_t bytes) {
    if (!ctx || !stats_out) return CBIE_EINVAL;
    std::memcpy(stats_out, &ctx->c.stats, std::min(bytes, sizeof(cbie_stats)));
    return CBIE_OK;
}

cbie_status cbie_set_profiling(cbie_ctx* ctx, int on) {
    return guarded(ctx, [&](Ctx& c) { c.gemm_timer.on = c.leaf_timer.on = on != 0; });
}

cbie_status cbie_get_near_pairs(cbie_ctx* ctx, int64_t cap, int32_t* targets, int32_t* patches,
                                int64_t* count_out) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_TREE, CBIE_ESTATE, "near pairs before build_tree");
        CBIE_REQUIRE(count_out && cap >= 0 && (cap == 0 || (targets && patches)), CBIE_EINVAL, "near arguments");
        *count_out = (int64_t)c.near.size();
        const int64_t m = std::min<int64_t>(cap, (int64_t)c.near.size());
        for (int64_t k = 0; k < m; ++k) {
            targets[k] = c.near[k].target;
            patches[k] = c.near[k].patch;
        }
    });
}

cbie_status cbie_export_dense(cbie_ctx* ctx, void* a_dev, long ld) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_FILLED, CBIE_ESTATE, "export before fill");
        CBIE_REQUIRE(a_dev && ld >= c.n_unk, CBIE_EINVAL, "export arguments");
        stage_export_dense(c, (zd*)a_dev, ld);
    });
}

cbie_status cbie_get_block_features(cbie_ctx* ctx, double aca_tol, int64_t cap, float* feat, int32_t* ranks,
                                    int64_t* count_out) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(c.state >= ST_TREE, CBIE_ESTATE, "features before build_tree");
        CBIE_REQUIRE(count_out && cap >= 0 && aca_tol > 0 && aca_tol < 1, CBIE_EINVAL, "feature arguments");
        const int64_t nb = (int64_t)c.lblk.size();
        *count_out = nb;
        const int64_t m = std::min(cap, nb);
        if (feat && m > 0) {
            std::vector<float> f;
            block_features(c, aca_tol, f);
            std::memcpy(feat, f.data(), (size_t)m * kMlpIn * sizeof(float));
        }
        if (ranks)
            for (int64_t b = 0; b < m; ++b)
                ranks[b] = (c.state >= ST_COMPRESSED && (int64_t)c.lr.rank.size() == nb) ? c.lr.rank[b] : -1;
    });
}

cbie_status cbie_set_rank_model(cbie_ctx* ctx, const float* params, const float* mean, const float* sdev,
                                float margin) {
    return guarded(ctx, [&](Ctx& c) {
        CBIE_REQUIRE(params && mean && sdev && margin >= 0 && margin < 100, CBIE_EINVAL, "rank model arguments");
        for (int k = 0; k < kMlpIn; ++k)
            CBIE_REQUIRE(sdev[k] > 0 && std::isfinite(mean[k]), CBIE_EINVAL, "feature scaling");
        for (int e = 0; e < kMlpParams; ++e) CBIE_REQUIRE(std::isfinite(params[e]), CBIE_EINVAL, "parameters");
        auto& M = c.rank_model;
        M.params.assign(params, params + kMlpParams);
        M.mean.assign(mean, mean + kMlpIn);
        M.sdev.assign(sdev, sdev + kMlpIn);
        M.margin = margin;
        M.set = true;
    });
}

cbie_status cbie_mlp_forward(void* hip_stream, const float* params, const float* mean, const float* sdev,
                             const float* X, int64_t n, float* y) {
    if (n < 0 || (n > 0 && (!params || !mean || !sdev || !X || !y))) return CBIE_EINVAL;
    return guarded_stream([&] { mlp_forward((hipStream_t)hip_stream, params, mean, sdev, X, n, y); });
}

cbie_status cbie_mlp_grad(void* hip_stream, const float* params, const float* mean, const float* sdev,
                          const float* X, const float* t, int64_t n, float* grad, float* loss) {
    if (n <= 0 || !params || !mean || !sdev || !X || !t || !grad || !loss) return CBIE_EINVAL;
    return guarded_stream([&] { mlp_grad((hipStream_t)hip_stream, params, mean, sdev, X, t, n, grad, loss); });
}

cbie_status cbie_mlp_train(void* hip_stream, float* params, const float* mean, const float* sdev, const float* X,
                           const float* t, const int32_t* order, int64_t nsteps, int batch, float lr,
                           float* losses) {
    if (nsteps < 0 || batch <= 0 || !(lr > 0) || !params || !mean || !sdev || !X || !t || !order ||
        (nsteps > 0 && !losses))
        return CBIE_EINVAL;
    if (nsteps == 0) return CBIE_OK;
    return guarded_stream(
        [&] { mlp_train((hipStream_t)hip_stream, params, mean, sdev, X, t, order, nsteps, batch, lr, losses); });
}

const char* cbie_last_error(const cbie_ctx* ctx) {
    if (!ctx) return "null context";
    return ctx->c.err.c_str();
}

void cbie_destroy(cbie_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;
}

}  // extern "C"

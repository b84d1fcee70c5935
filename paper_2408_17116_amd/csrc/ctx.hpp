// Library context: everything a cbie_ctx owns.
#pragma once
#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cbie.h"
#include "fill.hpp"
#include "tree.hpp"

namespace cbie {

enum State { ST_CREATED = 0, ST_TREE = 1, ST_FILLED = 2, ST_COMPRESSED = 3, ST_FACTORED = 4 };

// Storage of a low-rank block A ~ U V^T (U: m x rank, V: n x rank, both
// column-major with leading dimensions m and n).
template <typename T> struct LRStore {
    std::vector<int64_t> u_off, v_off;   // element offsets
    std::vector<int> rank, cap;          // current rank, capacity (columns)
    DBuf<cplx<T>> mem;
    DBuf<int64_t> d_u_off, d_v_off;
    DBuf<int> d_rank;
};

struct HMat;   // factorization state (hmat.hpp)

struct Ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int state = ST_CREATED;
    std::string err;

    // problem
    std::vector<ObjDev> objs;
    std::vector<PatchDev> patches;          // original order
    std::vector<int> obj_patch0, obj_npatch, obj_node0, obj_nodes;
    std::vector<int> node_patch;            // original node -> original patch
    int n_nodes = 0;
    int64_t n_unk = 0;
    int upn = 2;                            // unknowns per node: 2 (MFIE) or 4 (N-Mueller)

    // device problem tables
    DBuf<PatchDev> d_patches;
    DBuf<double> d_coef;                    // Chebyshev-interpolated patch coefficients (all objects)
    DBuf<ObjDev> d_objs;
    DBuf<int> d_node_patch, d_obj_patch0, d_obj_npatch;
    DBuf<double> d_fej11_x, d_fej11_w, d_fej01_x, d_fej01_w;
    DBuf<double> d_dmat;                    // Chebyshev differentiation matrices, q = 1..8

    // geometry (original node order)
    DBuf<double> d_geom;                    // 12 arrays of n_nodes
    NodeArrays nd{};
    DBuf<double> d_patch_info;
    std::vector<double> h_r;                // host copy of positions (3 n)

    // near pairs (sorted by target, patch; original numbering)
    std::vector<NearPair> near;
    DBuf<NearPair> d_near;

    // tree
    Tree tree;
    double eta = 1.0, delta = 1.0;
    int leaf_size = 256;
    std::vector<int> tree_node;             // tree node -> original node
    DBuf<int> d_tree_node;
    std::vector<int> orig_to_tree_node;

    // operator storage (complex128, tree order)
    std::vector<DenseBlockDev> dblk;        // per dense block
    DBuf<DenseBlockDev> d_dblk;
    DBuf<zd> dense;                         // all dense blocks
    LRStore<double> lr;                     // all low-rank blocks
    std::vector<DenseBlockDev> lblk;        // geometry of low-rank blocks (same layout)
    DBuf<DenseBlockDev> d_lblk;
    double aca_tol = 1e-6;
    double factor_tol = 0.0;                // truncation of formatted sums (0: aca_tol)
    int factor_ordering = CBIE_ORDER_ENTIRE;   // unknown ordering of the factorization

    // exclusive prefix sums of the low-rank ranks (nl + 1 entries, set by
    // compress): block b's V^T x occupies rows prefix[b] * nrhs .. of the
    // matvec scratch
    std::vector<int64_t> lr_prefix;
    DBuf<int64_t> d_lr_prefix;
    DBuf<zd> mv_tmp;                        // matvec scratch of the allocating path

    // factorization
    std::shared_ptr<HMat> hm;   // type-erased deleter: HMat stays incomplete here

    // rank predictor for compress(CBIE_RANK_PREDICTED): parameters, feature
    // mean and standard deviation, allocation margin
    struct RankModel {
        bool set = false;
        std::vector<float> params, mean, sdev;
        float margin = 0.25f;
    } rank_model;

    // statistics
    cbie_stats stats{};

    // Event pairs around timed launches.  When the pool is full, the pairs
    // that have completed are read without waiting (they complete in stream
    // order) and their events reused; the pool grows only while none has.
    // harvest() waits for all of them, at the end of a stage.
    struct KernelTimer {
        bool on = false;
        std::vector<hipEvent_t> ev;
        size_t used = 0;
        double seconds = 0.0;
        std::vector<float>* log = nullptr;   // each pair's milliseconds, in order (debug)
        void begin(hipStream_t s);
        void end(hipStream_t s);
        void harvest();
        void harvest_ready();
        ~KernelTimer();
    } gemm_timer, leaf_timer;

    Ctx();
    ~Ctx();
    void sync() { CBIE_HIP(hipStreamSynchronize(stream)); }
};

// stage entry points (implemented across the sources)
void stage_build_tree(Ctx& c, int leaf_size, double eta, double delta);
void stage_fill(Ctx& c, int n_ang, int n_rad);
void stage_compress(Ctx& c, double tol, int mode);
void stage_factor(Ctx& c, int prec);
void stage_solve(Ctx& c, int nrhs, const zd* b, zd* x, long ld, double tol, int maxit, int* iters);
void stage_solve_gmres(Ctx& c, int nrhs, const zd* b, zd* x, long ld, double tol, int restart, int maxit,
                       int* iters);
void stage_matvec(Ctx& c, int nrhs, const zd* x, zd* y, long ld);
void stage_export_dense(Ctx& c, zd* A, long ld);
void stage_rhs(Ctx& c, int nw, const double* khat, const double* pol, zd* b, long ld);
void stage_rhs_dipole(Ctx& c, int ndp, const double* pos, const double* mom, zd* b, long ld);
void stage_farfield(Ctx& c, int nrhs, const zd* x, long ld, int ndir, const double* rhat, zd* E);
// plain-rule N-Mueller entries of blocks (offsets / leading dimensions into dst)
void fill_blocks_nm(Ctx& c, const std::vector<DenseBlockDev>& blocks, const DenseBlockDev* d_blocks, zd* dst);

inline double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace cbie

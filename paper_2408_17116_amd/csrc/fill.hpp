// Device data layouts and kernels of the fill stage.
#pragma once
#include "geom.hpp"

namespace cbie {

// Node geometry, structure of arrays, original node order.
struct NodeArrays {
    double *rx, *ry, *rz;
    double *aux, *auy, *auz;
    double *avx, *avy, *avz;
    double *w, *u, *v;
};

// (target node, source patch) pair that needs the singular rule.
struct NearPair {
    int target;      // original node index
    int patch;       // original patch index
    double us, vs;   // singular point on the patch (node itself when self)
    double dist;     // target-to-patch distance (0 when self)
    int self;
    int pad;
};

// Sizes and offsets (into the Fejer tables) of the singular rule.
struct QuadRule {
    int n_ang, n_rad, n_in, n_out;
    int off_ang, off_rad, off_in, off_out;   // n(n-1)/2 offsets into the [0,1] Fejer tables
};

// A dense block as the fill kernels see it (tree order).
struct DenseBlockDev {
    int64_t offset;      // element offset into the dense store
    int ld;              // leading dimension (= upn row_nodes)
    int row_node0, row_nodes;   // tree-order node range of the rows
    int col_node0, col_nodes;   // tree-order node range of the columns
    int obj;
    int upn;             // unknowns per node: 2 (MFIE) or 4 (N-Mueller)
};

struct DenseTile {
    int block, row0, col0, pad;
};

// Where the 2 x 2 q^2 entries of a near pair go.
struct NearDest {
    int block;       // dense block id
    int row_node;    // target node, local row node in the block
    int col_node0;   // first node of the patch, local column node in the block
    int q2;          // nodes of the patch
};

__global__ void k_nodes(const PatchDev*, const ObjDev*, const double*, const double*, const int*, int,
                        NodeArrays);
__global__ void k_patch_info(const PatchDev*, const ObjDev*, int, double*);
__global__ void k_near(const PatchDev*, const ObjDev*, const double*, const int*, const int*, const int*,
                       NodeArrays, int, double, int*, const int64_t*, NearPair*);
template <int QM, bool CHEB>
__global__ void k_quad(const PatchDev*, const ObjDev*, NodeArrays, const NearPair*, int64_t,
                       const double*, const double*, const double*, QuadRule, int64_t, zd*);
template <typename T>
__global__ void k_far_fill(const DenseTile*, int, const DenseBlockDev*, const int*, NodeArrays,
                           const ObjDev*, cplx<T>*);
__global__ void k_quad_nm(const PatchDev*, const ObjDev*, NodeArrays, const NearPair*, int64_t, const double*,
                          const double*, const double*, const double*, QuadRule, int64_t, zd*);
template <typename T>
__global__ void k_far_fill_nm(const DenseTile*, int, const DenseBlockDev*, const int*, NodeArrays, const ObjDev*,
                              const double*, cplx<T>*);
template <typename T>
__global__ void k_near_scatter(const NearDest*, int64_t, int64_t, const zd*, const DenseBlockDev*, cplx<T>*);

}  // namespace cbie

namespace cbie {
__global__ void k_export_dense_block(const DenseBlockDev*, int, const int*, const zd*, zd*, int64_t);
__global__ void k_export_far(const DenseBlockDev*, int, const int*, NodeArrays, const ObjDev*, zd*, int64_t);
}  // namespace cbie

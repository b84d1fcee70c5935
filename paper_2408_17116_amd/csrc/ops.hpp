// Operator application and permutation helpers.
#pragma once
#include "common.hpp"

namespace cbie {
struct Ctx;
template <typename T>
__global__ void k_to_tree(const int*, int, int64_t, int, const zd*, int64_t, cplx<T>*);
template <typename T>
__global__ void k_from_tree(const int*, int, int64_t, int, const cplx<T>*, zd*, int64_t);
// y_t = A x_t (tree order, FP64, leading dimension n_unk), y_t overwritten
void apply_operator_tree(Ctx& c, int nrhs, const zd* xt, zd* yt);

}  // namespace cbie

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

// Allocation-free matvec: complex128 elements of the per-GPU scratch array
// (2^23, 128 MiB) and what one call needs, 2 n_unk nrhs + sum(ranks) nrhs.
constexpr int64_t kScratchElems = int64_t(1) << 23;
int64_t matvec_scratch_elems(const Ctx& c, int nrhs);
// Resolve the device address of the scratch array on `device` (current);
// once per device, thread-safe.
void resolve_scratch(int device);
void stage_matvec_noalloc(Ctx& c, int nrhs, const zd* x, zd* y, long ld);
}  // namespace cbie

// Dense complex kernels used by the H-LU (column-major, complex64 or
// complex128).  Every routine enqueues work on `s` and returns at once.
#pragma once
#include <vector>
#include "common.hpp"

namespace cbie {

// C = alpha op(A) op(B) + beta C, op in {'N', 'T'} (plain transpose)
template <typename T>
void gemm(hipStream_t s, char ta, char tb, int m, int n, int k, cplx<T> alpha, const cplx<T>* A, int lda,
          const cplx<T>* B, int ldb, cplx<T> beta, cplx<T>* C, int ldc);

// P A = L U in place for an n x n leaf (partial pivoting, LAPACK-style
// ipiv: row j was swapped with row piv[j]).  info[0] > 0 when a pivot is
// exactly zero (first such column + 1); the factorization still completes.
template <typename T>
void getrf(hipStream_t s, int n, cplx<T>* A, int lda, int* piv, int* info);

// B (m x n) := L^{-1} P^T B with the unit-lower factor and pivots of getrf
template <typename T>
void trsm_llnu_piv(hipStream_t s, int m, int n, const cplx<T>* LU, int ld, const int* piv, cplx<T>* B, int ldb);
// B (m x n) := U^{-1} B (upper, non-unit, left)
template <typename T>
void trsm_lunn(hipStream_t s, int m, int n, const cplx<T>* LU, int ld, cplx<T>* B, int ldb);
// B (m x n) := B U^{-1} (upper n x n, non-unit, right)
template <typename T>
void trsm_runn(hipStream_t s, int m, int n, const cplx<T>* LU, int ld, cplx<T>* B, int ldb);

// B (n x m) = A^T (A: m x n)
template <typename T>
void transpose(hipStream_t s, int m, int n, const cplx<T>* A, int lda, cplx<T>* B, int ldb);
// B (m x n) = alpha A (A may be null: B = 0)
template <typename T>
void copy_scale(hipStream_t s, int m, int n, cplx<T> alpha, const cplx<T>* A, int lda, cplx<T>* B, int ldb);
// element-wise precision conversion of a contiguous array
template <typename Tin, typename Tout>
void convert(hipStream_t s, int64_t n, const cplx<Tin>* a, cplx<Tout>* b);
// b_i[0, n_i) = (Tout) a_i[0, n_i) for every descriptor, one launch
template <typename Tin, typename Tout> struct ConvDesc {
    const cplx<Tin>* a;
    cplx<Tout>* b;
    int64_t n;
};
template <typename Tin, typename Tout>
void convert_batched(hipStream_t s, const std::vector<ConvDesc<Tin, Tout>>& v);
// work-group t converts elements [e0, e0 + 4096) of array desc
struct ConvTile {
    int desc, pad;
    int64_t e0;
};
// convert_batched over descriptors and tiles already on the device (no
// allocation, no synchronization)
template <typename Tin, typename Tout>
void convert_batched_dev(hipStream_t s, const ConvDesc<Tin, Tout>* d, const ConvTile* t, int nt);
// b[i + j ldb] = (Tout) a[i rs + j cs] for i < m, j < n, every descriptor,
// one launch (a strided sub-matrix, e.g. every upn-th row of a block)
template <typename Tin, typename Tout> struct SliceDesc {
    const cplx<Tin>* a;
    cplx<Tout>* b;
    int m, n;
    int64_t rs, cs, ldb;
};
template <typename Tin, typename Tout>
void slice_batched(hipStream_t s, const std::vector<SliceDesc<Tin, Tout>>& v);

// ACA of an implicit product M = Uc Vc^T (m x n, inner K <= 2048): writes
// U (m x cap) and V (n x cap), cap <= 1024, with M ~ U V^T to relative
// Frobenius tolerance tol; rank_out[0] gets the rank.  One work-group per
// job.  The copy-back moves U[:, :rank], V[:, :rank] to dstU, dstV.
template <typename T> struct AcaProdJob {
    int m, n, K, cap;
    const cplx<T>* D;        // optional dense addend (m x n, leading dim m): M = D + Uc Vc^T
    const cplx<T>* Uc;
    const cplx<T>* Vc;
    cplx<T>* U;
    cplx<T>* V;
    cplx<T>* dstU;
    cplx<T>* dstV;
    unsigned char* used;
    int* rank_out;
};
template <typename T>
void aca_product_batched(hipStream_t s, int njobs, const AcaProdJob<T>* d_jobs, double tol);
template <typename T>
void aca_copyback_batched(hipStream_t s, int njobs, const AcaProdJob<T>* d_jobs);

// Explicit inverses of the factors of a diagonal leaf after getrf:
// LP = L^{-1} P and UI = U^{-1} (both n x n, leading dimension n).
template <typename T>
void leaf_inverse(hipStream_t s, int n, const cplx<T>* LU, int ld, const int* piv, cplx<T>* LP, cplx<T>* UI);

}  // namespace cbie

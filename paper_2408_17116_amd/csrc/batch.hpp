// Batched kernels executed level by level by the H-LU task scheduler.
#pragma once
#include "common.hpp"

namespace cbie {

// C = alpha op(A) op(B) + beta C; op N, T (transpose) or C (conjugate transpose)
template <typename T> struct GemmDesc {
    int m, n, k;
    int ta, tb;              // 0 = N, 1 = T, 2 = C
    cplx<T> alpha, beta;
    const cplx<T>* A;
    const cplx<T>* B;
    cplx<T>* C;
    int lda, ldb, ldc;
    int pad;
};
// one output tile of a product: the descriptor and the tile's index in it,
// row-major over the product's tile grid (m0 = (lt / tiles per row) * rows,
// n0 = (lt % tiles per row) * columns of the launch's tile shape)
struct GemmTile {
    int desc, lt;
};
// output tile shapes of the batched GEMM (rows x columns of C)
enum { kTile64x64 = 0, kTile256x32 = 1, kTile32x256 = 2, kNumTileShapes = 3 };
inline int tile_rows(int shape) { return shape == kTile64x64 ? 64 : (shape == kTile256x32 ? 256 : 32); }
inline int tile_cols(int shape) { return shape == kTile64x64 ? 64 : (shape == kTile256x32 ? 32 : 256); }

// B = alpha op(A) (A == nullptr: B = 0); op 'N' or 'T'
template <typename T> struct CopyDesc {
    int m, n;                // size of B
    int trans;
    int lda, ldb;
    cplx<T> alpha;
    const cplx<T>* A;
    cplx<T>* B;
};
struct CopyTile {
    int desc, e0;            // element chunk start
};

// Second phase of a split-k product: C = alpha sum_s W_s + beta C, where
// W_s (m x n, leading dimension m, stored one after another) are the
// partial products over consecutive k ranges.  Tiles are CopyTile chunks.
template <typename T> struct ReduceDesc {
    int m, n, nsplit, ldc;
    cplx<T> alpha, beta;
    const cplx<T>* W;
    cplx<T>* C;
};
template <typename T>
void reduce_batched(hipStream_t s, const ReduceDesc<T>* d_desc, const CopyTile* d_tiles, int ntiles);

// LU with partial pivoting of a diagonal leaf followed by the explicit
// inverses LP = L^{-1} P and UI = U^{-1} (n x n each, leading dimension n)
template <typename T> struct LeafDesc {
    int n, lda;
    cplx<T>* A;
    int* piv;
    int* info;
    cplx<T>* LP;
    cplx<T>* UI;
};

// uniform random entries in (-1, 1) + i (-1, 1) from a counter-based hash
template <typename T> struct RandDesc {
    cplx<T>* p;
    int m, n, ld;
    uint32_t seed;
};

// Hermitian eigen-decomposition A = E diag(lam) E^H of a p x p matrix
// (p <= 512) by parallel cyclic Jacobi; eigenvalues descending.  A is
// overwritten.  mode 0: write E;  mode 1 (orthonormalisation of a Gram
// matrix): scale column k of E by lam_k^{-1/2}, or 0 when lam_k <= thr lam_0;
// mode 2 (truncation): rank_out = smallest r with sum_{k>=r} lam_k <=
// tol^2 sum lam_k.
template <typename T> struct EigDesc {
    cplx<T>* A;
    cplx<T>* Ework;
    cplx<T>* E;
    int p, mode;
    double thr;
    int* rank_out;
};

// Pivoted Cholesky of a p x p Hermitian positive semi-definite Gram matrix
// G (p <= 512, overwritten): G[pi, pi] ~ R^H R with pivots by largest
// remaining diagonal, stopped when it falls below thr times the largest
// diagonal; k = number of pivots taken.  Writes S (p x p): S[pi(t), j] =
// (R^{-1})[t, j] for t <= j < k, zero elsewhere, so that Q = Y S has k
// orthonormal columns spanning the range of Y (then zero columns).
template <typename T> struct PcholDesc {
    cplx<T>* G;
    cplx<T>* S;
    int p;
    double thr;
    int* k_out;
};
template <typename T>
void pchol_batched(hipStream_t s, const PcholDesc<T>* d_desc, int n);

template <typename T>
void rand_batched(hipStream_t s, const RandDesc<T>* d_desc, int n);
template <typename T>
void eig_batched(hipStream_t s, const EigDesc<T>* d_desc, int n);

// complex64 products on 64 x 64 tiles by three real products instead of
// four (on unless CBIE_GEMM_3M=0)
bool gemm_three_mult();
template <typename T>
void gemm_batched(hipStream_t s, const GemmDesc<T>* d_desc, const GemmTile* d_tiles, int ntiles, int shape);
template <typename T>
void copy_batched(hipStream_t s, const CopyDesc<T>* d_desc, const CopyTile* d_tiles, int ntiles);
template <typename T>
void leaf_batched(hipStream_t s, const LeafDesc<T>* d_desc, int n);

constexpr int kCopyChunk = 8192;

}  // namespace cbie

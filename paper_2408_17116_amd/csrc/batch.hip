// Batched GEMM / copy / leaf-LU kernels driven by descriptor and tile lists.
#include "batch.hpp"

namespace cbie {

template <typename T> __device__ inline cplx<T> bz() { return cplx<T>{(T)0, (T)0}; }

// ---------------------------------------------------------------- GEMM
// Complex GEMM on the matrix cores.  A complex product is four real
// 16x16x4 MFMAs into separate real and imaginary accumulators:
//   Cr += Ar Br - Ai Bi,   Ci += Ar Bi + Ai Br.
// Operand layout of v_mfma_*_16x16x4 (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; its v-th result (v = 0..3) is D[row(l, v)][l%16] with
// row = 4 (l/16) + v for f32 and row = l/16 + 4 v for f64 (measured).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int g, int v) { return 4 * g + v; }
};
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int g, int v) { return g + 4 * v; }
};

// One work-group (4 waves) per BM x BN output tile; op(A) and op(B) are
// staged through LDS by BK-deep slices with the next slice prefetched into
// registers.  Waves split the tile WGM x (4 / WGM).  A work-group reads
// only the rows of op(A) and columns of op(B) of its own tile and stores
// after its last read, so a tile that spans all rows (or all columns) of
// C may overwrite its own operand: X := M X and X := X M in place.
template <typename T, int BM, int BN, int WGM, int BK>
__global__ __launch_bounds__(256) void k_zgemm(const GemmDesc<T>* __restrict__ descs,
                                               const GemmTile* __restrict__ tiles, int ntiles) {
    constexpr int WGN = 4 / WGM, WM = BM / WGM, WN = BN / WGN, FM = WM / 16, FN = WN / 16;
    constexpr int PAD = sizeof(T) == 4 ? 16 : 2;
    constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
    static_assert(NA >= 1 && NB >= 1 && FM >= 1 && FN >= 1, "tile shape");
    typedef typename Mfma<T>::v4 v4;
    __shared__ cplx<T> As[BK][BM + PAD];
    __shared__ cplx<T> Bs[BK][BN + PAD];
    // consecutive tiles (which share operand panels) go to one XCD: the
    // hardware deals work-groups round-robin over the 8 XCDs
    const int per = (int)gridDim.x >> 3;
    const int t = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (t >= ntiles) return;
    const GemmTile tl = tiles[t];
    const GemmDesc<T> D = descs[tl.desc];
    const int m = D.m, n = D.n, k = D.k;
    const int m0 = tl.m0, n0 = tl.n0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int r = lane & 15, kq = lane >> 4;

    v4 cr[FM][FN], ci[FM][FN];
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j)
            for (int v = 0; v < 4; ++v) { cr[i][j][v] = (T)0; ci[i][j][v] = (T)0; }

    cplx<T> ra[NA], rb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q;
            int i, kk;
            if (D.ta == 0) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
            const int gi = m0 + i, gk = k0 + kk;
            cplx<T> v{(T)0, (T)0};
            if (gi < m && gk < k) {
                v = D.ta == 0 ? D.A[gi + (int64_t)gk * D.lda] : D.A[gk + (int64_t)gi * D.lda];
                if (D.ta == 2) v.im = -v.im;
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q;
            int j, kk;
            if (D.tb == 0) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
            const int gj = n0 + j, gk = k0 + kk;
            cplx<T> v{(T)0, (T)0};
            if (gj < n && gk < k) {
                v = D.tb == 0 ? D.B[gk + (int64_t)gj * D.ldb] : D.B[gj + (int64_t)gk * D.ldb];
                if (D.tb == 2) v.im = -v.im;
            }
            rb[q] = v;
        }
    };
    load(0);
    for (int k0 = 0; k0 < k; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int e = tid + 256 * q;
            if (D.ta == 0) As[e / BM][e % BM] = ra[q]; else As[e % BK][e / BK] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q;
            if (D.tb == 0) Bs[e % BK][e / BK] = rb[q]; else Bs[e / BN][e % BN] = rb[q];
        }
        __syncthreads();
        if (k0 + BK < k) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            cplx<T> a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[kk + kq][wm * WM + 16 * i + r];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = Bs[kk + kq][wn * WN + 16 * j + r];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const T nai = -a[i].im;
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    cr[i][j] = Mfma<T>::op(a[i].re, b[j].re, cr[i][j]);
                    cr[i][j] = Mfma<T>::op(nai, b[j].im, cr[i][j]);
                    ci[i][j] = Mfma<T>::op(a[i].re, b[j].im, ci[i][j]);
                    ci[i][j] = Mfma<T>::op(a[i].im, b[j].re, ci[i][j]);
                }
            }
        }
    }
    const bool zb = (D.beta.re == (T)0 && D.beta.im == (T)0);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn * WN + 16 * j + r;
        if (col >= n) continue;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int row0 = m0 + wm * WM + 16 * i;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + Mfma<T>::row(kq, v);
                if (row >= m) continue;
                cplx<T>* cp = D.C + row + (int64_t)col * D.ldc;
                cplx<T> o = D.alpha * cplx<T>{cr[i][j][v], ci[i][j][v]};
                if (!zb) cfma(o, D.beta, *cp);
                *cp = o;
            }
        }
    }
}

template <typename T>
void gemm_batched(hipStream_t s, const GemmDesc<T>* d_desc, const GemmTile* d_tiles, int ntiles, int shape) {
    if (ntiles <= 0) return;
    const int grid = (ntiles + 7) / 8 * 8;
    constexpr int BKW = sizeof(T) == 4 ? 16 : 8;   // deep slices of the wide tiles fit LDS
    switch (shape) {
        case kTile64x64: k_zgemm<T, 64, 64, 2, 16><<<grid, 256, 0, s>>>(d_desc, d_tiles, ntiles); break;
        case kTile256x32: k_zgemm<T, 256, 32, 4, BKW><<<grid, 256, 0, s>>>(d_desc, d_tiles, ntiles); break;
        case kTile32x256: k_zgemm<T, 32, 256, 1, BKW><<<grid, 256, 0, s>>>(d_desc, d_tiles, ntiles); break;
        default: throw Error{-7, "gemm_batched: unknown tile shape"};
    }
    check_launch("k_zgemm");
}

// ---------------------------------------------------------------- copies
template <typename T>
__global__ __launch_bounds__(256) void k_copy_b(const CopyDesc<T>* __restrict__ descs,
                                                const CopyTile* __restrict__ tiles, int ntiles) {
    if ((int)blockIdx.x >= ntiles) return;
    const CopyTile tl = tiles[blockIdx.x];
    const CopyDesc<T> D = descs[tl.desc];
    const int64_t tot = (int64_t)D.m * D.n;
    const int64_t e1 = min(tot, (int64_t)tl.e0 + kCopyChunk);
    for (int64_t e = tl.e0 + threadIdx.x; e < e1; e += 256) {
        const int i = (int)(e % D.m), j = (int)(e / D.m);
        cplx<T> v = bz<T>();
        if (D.A) v = D.alpha * (D.trans ? D.A[j + (int64_t)i * D.lda] : D.A[i + (int64_t)j * D.lda]);
        D.B[i + (int64_t)j * D.ldb] = v;
    }
}

template <typename T>
void copy_batched(hipStream_t s, const CopyDesc<T>* d_desc, const CopyTile* d_tiles, int ntiles) {
    if (ntiles <= 0) return;
    k_copy_b<T><<<ntiles, 256, 0, s>>>(d_desc, d_tiles, ntiles);
    check_launch("k_copy_b");
}

// ------------------------------------------------------- leaf LU + inverse
struct AMx {
    double v;
    int i;
};
__device__ inline AMx amx_better(AMx a, AMx b) { return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a; }

// One work-group of 256 threads per leaf.  Right-looking LU with partial
// pivoting by panels of 16 columns; the U12 panel row is staged in LDS for
// the trailing update (leaves of at most 256 unknowns).  Then
// LP = L^{-1} P and UI = U^{-1} by one thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_leaf(const LeafDesc<T>* __restrict__ descs, int nd) {
    constexpr int NB = 16, RMAX = 240;
    __shared__ AMx sh[4];
    __shared__ cplx<T> su[NB][RMAX];
    __shared__ int perm[1024];
    if ((int)blockIdx.x >= nd) return;
    const LeafDesc<T> D = descs[blockIdx.x];
    const int n = D.n, lda = D.lda;
    cplx<T>* A = D.A;
    const int tid = threadIdx.x;
    int first_zero = 0;
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        for (int j = j0; j < j0 + jb; ++j) {
            AMx a{-1.0, 0x7fffffff};
            for (int i = j + tid; i < n; i += 256) a = amx_better(a, AMx{(double)abs2(A[i + (int64_t)j * lda]), i});
            for (int off = 32; off > 0; off >>= 1) {
                AMx o{__shfl_xor(a.v, off), __shfl_xor(a.i, off)};
                a = amx_better(a, o);
            }
            __syncthreads();
            if ((tid & 63) == 0) sh[tid >> 6] = a;
            __syncthreads();
            a = sh[0];
            for (int w = 1; w < 4; ++w) a = amx_better(a, sh[w]);
            const int p = a.i;
            if (tid == 0) D.piv[j] = p;
            if (a.v <= 0.0 && first_zero == 0) first_zero = j + 1;
            if (p != j)
                for (int c = j0 + tid; c < j0 + jb; c += 256) {
                    const cplx<T> t = A[j + (int64_t)c * lda];
                    A[j + (int64_t)c * lda] = A[p + (int64_t)c * lda];
                    A[p + (int64_t)c * lda] = t;
                }
            __syncthreads();
            const cplx<T> d = A[j + (int64_t)j * lda];
            if (a.v > 0.0)
                for (int i = j + 1 + tid; i < n; i += 256) A[i + (int64_t)j * lda] = cdiv(A[i + (int64_t)j * lda], d);
            __syncthreads();
            for (int i = j + 1 + tid; i < n; i += 256) {
                const cplx<T> l = A[i + (int64_t)j * lda];
                for (int c = j + 1; c < j0 + jb; ++c) {
                    cplx<T> v = A[i + (int64_t)c * lda];
                    cfma(v, -l, A[j + (int64_t)c * lda]);
                    A[i + (int64_t)c * lda] = v;
                }
            }
            __syncthreads();
        }
        for (int j = j0; j < j0 + jb; ++j) {
            const int p = D.piv[j];
            if (p != j)
                for (int c = tid; c < n; c += 256) {
                    if (c >= j0 && c < j0 + jb) continue;
                    const cplx<T> t = A[j + (int64_t)c * lda];
                    A[j + (int64_t)c * lda] = A[p + (int64_t)c * lda];
                    A[p + (int64_t)c * lda] = t;
                }
            __syncthreads();
        }
        for (int c = j0 + jb + tid; c < n; c += 256) {
            for (int r = j0 + 1; r < j0 + jb; ++r) {
                cplx<T> v = A[r + (int64_t)c * lda];
                for (int t = j0; t < r; ++t) cfma(v, -A[r + (int64_t)t * lda], A[t + (int64_t)c * lda]);
                A[r + (int64_t)c * lda] = v;
            }
        }
        __syncthreads();
        const int r0 = j0 + jb, R = n - r0;
        if (R > 0 && R <= RMAX) {
            for (int e = tid; e < jb * R; e += 256) {
                const int t = e % jb, c = e / jb;
                su[t][c] = A[j0 + t + (int64_t)(r0 + c) * lda];
            }
            __syncthreads();
            for (int64_t e = tid; e < (int64_t)R * R; e += 256) {
                const int i = (int)(e % R), c = (int)(e / R);
                cplx<T> v = A[r0 + i + (int64_t)(r0 + c) * lda];
                for (int t = 0; t < jb; ++t) cfma(v, -A[r0 + i + (int64_t)(j0 + t) * lda], su[t][c]);
                A[r0 + i + (int64_t)(r0 + c) * lda] = v;
            }
        } else {
            for (int64_t e = tid; e < (int64_t)R * R; e += 256) {
                const int i = r0 + (int)(e % R), c = r0 + (int)(e / R);
                cplx<T> v = A[i + (int64_t)c * lda];
                for (int t = j0; t < j0 + jb; ++t) cfma(v, -A[i + (int64_t)t * lda], A[t + (int64_t)c * lda]);
                A[i + (int64_t)c * lda] = v;
            }
        }
        __syncthreads();
    }
    if (tid == 0) D.info[0] = first_zero;
    // inverses
    if (tid == 0) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int j = 0; j < n; ++j) {
            const int p = D.piv[j];
            const int t = perm[j]; perm[j] = perm[p]; perm[p] = t;
        }
    }
    __syncthreads();
    for (int c = tid; c < n; c += 256) {
        int sidx = 0;
        for (int i = 0; i < n; ++i)
            if (perm[i] == c) sidx = i;
        cplx<T>* x = D.LP + (int64_t)c * n;
        for (int i = 0; i < n; ++i) {
            cplx<T> v = cplx<T>{(T)(i == sidx ? 1 : 0), (T)0};
            for (int t = sidx; t < i; ++t) cfma(v, -A[i + (int64_t)t * lda], x[t]);
            x[i] = (i < sidx) ? bz<T>() : v;
        }
        cplx<T>* y = D.UI + (int64_t)c * n;
        for (int i = n - 1; i >= 0; --i) {
            cplx<T> v = cplx<T>{(T)(i == c ? 1 : 0), (T)0};
            for (int t = i + 1; t <= c; ++t) cfma(v, -A[i + (int64_t)t * lda], y[t]);
            y[i] = (i > c) ? bz<T>() : cdiv(v, A[i + (int64_t)i * lda]);
        }
    }
}

template <typename T>
void leaf_batched(hipStream_t s, const LeafDesc<T>* d_desc, int nd) {
    if (nd <= 0) return;
    k_leaf<T><<<nd, 256, 0, s>>>(d_desc, nd);
    check_launch("k_leaf");
}

// --------------------------------------------------------------- random
__device__ inline uint32_t hash32(uint32_t x) {
    // integer finalizer of the 32-bit MurmurHash3
    x ^= x >> 16; x *= 0x85ebca6bu; x ^= x >> 13; x *= 0xc2b2ae35u; x ^= x >> 16;
    return x;
}
template <typename T>
__global__ void k_rand_b(const RandDesc<T>* __restrict__ descs, int nd) {
    const int d = blockIdx.y;
    if (d >= nd) return;
    const RandDesc<T> D = descs[d];
    const int64_t tot = (int64_t)D.m * D.n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % D.m), j = (int)(e / D.m);
        const uint32_t h1 = hash32(D.seed ^ hash32((uint32_t)(2 * e)));
        const uint32_t h2 = hash32(D.seed ^ hash32((uint32_t)(2 * e + 1)));
        D.p[i + (int64_t)j * D.ld] = cplx<T>{(T)(h1 * (2.0 / 4294967296.0) - 1.0), (T)(h2 * (2.0 / 4294967296.0) - 1.0)};
    }
}
template <typename T>
void rand_batched(hipStream_t s, const RandDesc<T>* d_desc, int n) {
    if (n <= 0) return;
    k_rand_b<T><<<dim3(64, n), 256, 0, s>>>(d_desc, n);
    check_launch("k_rand_b");
}

// ------------------------------------------------------ pivoted Cholesky
template <typename T>
__global__ __launch_bounds__(256) void k_pchol_b(const PcholDesc<T>* __restrict__ descs, int nd) {
    if ((int)blockIdx.x >= nd) return;
    const PcholDesc<T> D = descs[blockIdx.x];
    const int p = D.p;
    cplx<T>* G = D.G;
    __shared__ int perm[512];
    __shared__ double dv[4];
    __shared__ int di[4];
    __shared__ double dmax0;
    __shared__ int kk;
    const int tid = threadIdx.x;
    for (int i = tid; i < p; i += 256) perm[i] = i;
    if (tid == 0) {
        double m0 = 0.0;
        for (int i = 0; i < p; ++i) m0 = fmax(m0, (double)G[i + (int64_t)i * p].re);
        dmax0 = m0;
        kk = p;
    }
    __syncthreads();
    for (int j = 0; j < p; ++j) {
        // pivot: largest remaining diagonal
        double bv = -1.0;
        int bi = j;
        for (int t = j + tid; t < p; t += 256) {
            const double v = (double)G[t + (int64_t)t * p].re;
            if (v > bv) { bv = v; bi = t; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        __syncthreads();
        if ((tid & 63) == 0) { dv[tid >> 6] = bv; di[tid >> 6] = bi; }
        __syncthreads();
        bv = dv[0]; bi = di[0];
        for (int w = 1; w < 4; ++w)
            if (dv[w] > bv || (dv[w] == bv && di[w] < bi)) { bv = dv[w]; bi = di[w]; }
        if (!(bv > D.thr * dmax0) || bv <= 0.0) {
            if (tid == 0) kk = j;
            break;
        }
        // symmetric swap of rows/columns j and bi
        if (bi != j) {
            for (int t = tid; t < p; t += 256) {
                const cplx<T> a = G[j + (int64_t)t * p];
                G[j + (int64_t)t * p] = G[bi + (int64_t)t * p];
                G[bi + (int64_t)t * p] = a;
            }
            __syncthreads();
            for (int t = tid; t < p; t += 256) {
                const cplx<T> a = G[t + (int64_t)j * p];
                G[t + (int64_t)j * p] = G[t + (int64_t)bi * p];
                G[t + (int64_t)bi * p] = a;
            }
            if (tid == 0) { const int x = perm[j]; perm[j] = perm[bi]; perm[bi] = x; }
            __syncthreads();
        }
        // row j of R: R[j, j] = sqrt(G[j, j]), R[j, t] = G[j, t] / R[j, j]
        const T rjj = sqrt((T)bv);
        for (int t = j + 1 + tid; t < p; t += 256) G[j + (int64_t)t * p] = (T(1) / rjj) * G[j + (int64_t)t * p];
        __syncthreads();
        if (tid == 0) G[j + (int64_t)j * p] = cplx<T>{rjj, (T)0};
        // trailing downdate G[t, u] -= conj(R[j, t]) R[j, u], t, u > j
        const int R = p - j - 1;
        for (int64_t e = tid; e < (int64_t)R * R; e += 256) {
            const int t = j + 1 + (int)(e % R), u = j + 1 + (int)(e / R);
            cplx<T> v = G[t + (int64_t)u * p];
            cfma(v, -conj(G[j + (int64_t)t * p]), G[j + (int64_t)u * p]);
            G[t + (int64_t)u * p] = v;
        }
        __syncthreads();
    }
    __syncthreads();
    const int k = kk;
    // S = Pi R_kk^{-1}: column j solves R x = e_j by back substitution
    for (int64_t e = tid; e < (int64_t)p * p; e += 256) D.S[e] = bz<T>();
    __syncthreads();
    for (int j = tid; j < k; j += 256) {
        // x[t] for t <= j, kept in S (row perm[t], column j)
        for (int t = j; t >= 0; --t) {
            cplx<T> v = cplx<T>{(T)(t == j ? 1 : 0), (T)0};
            for (int u = t + 1; u <= j; ++u) cfma(v, -G[t + (int64_t)u * p], D.S[perm[u] + (int64_t)j * p]);
            D.S[perm[t] + (int64_t)j * p] = cdiv(v, G[t + (int64_t)t * p]);
        }
    }
    if (tid == 0) D.k_out[0] = k;
}
template <typename T>
void pchol_batched(hipStream_t s, const PcholDesc<T>* d_desc, int n) {
    if (n <= 0) return;
    k_pchol_b<T><<<n, 256, 0, s>>>(d_desc, n);
    check_launch("k_pchol_b");
}

// ------------------------------------------------------ Hermitian Jacobi
// One work-group per matrix.  Each sweep runs the p-1 rounds of a
// round-robin tournament; in a round the p/2 disjoint pairs (i, j) are
// rotated together: rotation parameters from the 2 x 2 principal blocks,
// then all row updates (A := J^H A), then all column updates (A := A J,
// E := E J).  For the pair block [[a, b], [conj(b), d]], b = |b| e^{i phi}:
// J = diag(1, e^{-i phi}) [[c, s], [-s, c]] with the real rotation that
// annihilates [[a, |b|], [|b|, d]]: zeta = (d - a)/(2|b|),
// t = sgn(zeta)/(|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = t c.
template <typename T>
__global__ __launch_bounds__(256) void k_heig_b(const EigDesc<T>* __restrict__ descs, int nd) {
    if ((int)blockIdx.x >= nd) return;
    const EigDesc<T> D = descs[blockIdx.x];
    const int p = D.p;
    const int P = (p + 1) & ~1;           // even number of players (one dummy when p is odd)
    cplx<T>* A = D.A;
    cplx<T>* E = D.Ework;
    __shared__ int pi_[256], pj_[256];    // p <= 512: at most 256 pairs
    __shared__ T pc[256], pr[256];        // c and the signed real s of each pair
    __shared__ cplx<T> ps[256];           // s e^{-i phi}
    __shared__ cplx<T> ph[256];           // e^{-i phi}
    __shared__ double red[4];
    __shared__ int order[512];
    __shared__ double lam[512];
    const int tid = threadIdx.x;
    for (int64_t e = tid; e < (int64_t)p * p; e += 256)
        E[e] = cplx<T>{(T)((e % p) == (e / p) ? 1 : 0), (T)0};
    __syncthreads();
    const double eps = sizeof(T) == 8 ? 1e-15 : 1e-7;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int64_t e = tid; e < (int64_t)p * p; e += 256) {
            const int i = (int)(e % p), j = (int)(e / p);
            const double v = (double)abs2(A[e]);
            if (i == j) dg += v; else off += v;
        }
        for (int o = 32; o > 0; o >>= 1) { off += __shfl_xor(off, o); dg += __shfl_xor(dg, o); }
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = off;
        __syncthreads();
        const double offt = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = dg;
        __syncthreads();
        const double dgt = red[0] + red[1] + red[2] + red[3];
        if (offt <= eps * eps * dgt || dgt == 0.0) break;
        for (int rnd = 0; rnd < P - 1; ++rnd) {
            // pairs of this round
            for (int k = tid; k < P / 2; k += 256) {
                int i, j;
                if (k == 0) { i = P - 1; j = rnd; }
                else { i = (rnd + k) % (P - 1); j = (rnd - k + P - 1) % (P - 1); }
                if (i > j) { const int t = i; i = j; j = t; }
                T c = (T)1, sreal = (T)0;
                cplx<T> se{(T)0, (T)0}, e{(T)1, (T)0};
                if (j < p) {
                    const T a = A[i + (int64_t)i * p].re, d = A[j + (int64_t)j * p].re;
                    const cplx<T> b = A[i + (int64_t)j * p];
                    const T bb = sqrt(abs2(b));
                    if (bb > (T)0 && bb > (T)(sizeof(T) == 8 ? 1e-300 : 1e-30)) {
                        const T zeta = (d - a) / (2 * bb);
                        const T t = (zeta >= 0 ? (T)1 : (T)-1) / (fabs(zeta) + sqrt((T)1 + zeta * zeta));
                        c = (T)1 / sqrt((T)1 + t * t);
                        const T sr = t * c;
                        sreal = sr;
                        e = cplx<T>{b.re / bb, -b.im / bb};            // e^{-i phi}
                        se = cplx<T>{sr * e.re, sr * e.im};
                    }
                }
                pi_[k] = i; pj_[k] = j; pc[k] = c; pr[k] = sreal; ps[k] = se; ph[k] = e;
            }
            __syncthreads();
            // rows: row_i' = c row_i - conj(se) row_j ; row_j' = s row_i + c conj(e) row_j
            for (int64_t e2 = tid; e2 < (int64_t)(P / 2) * p; e2 += 256) {
                const int k = (int)(e2 / p), col = (int)(e2 % p);
                const int i = pi_[k], j = pj_[k];
                if (j >= p) continue;
                const T c = pc[k], s = pr[k];
                const cplx<T> se = ps[k], e = ph[k];
                const cplx<T> ai = A[i + (int64_t)col * p], aj = A[j + (int64_t)col * p];
                cplx<T> ni = c * ai, nj = s * ai;
                cfma(ni, -conj(se), aj);
                cfma(nj, c * conj(e), aj);
                A[i + (int64_t)col * p] = ni;
                A[j + (int64_t)col * p] = nj;
            }
            __syncthreads();
            // columns (and E): col_i' = c col_i - se col_j ; col_j' = s col_i + c e col_j
            for (int64_t e2 = tid; e2 < (int64_t)(P / 2) * p * 2; e2 += 256) {
                const int which = (int)(e2 / ((int64_t)(P / 2) * p));
                const int64_t r2 = e2 % ((int64_t)(P / 2) * p);
                const int k = (int)(r2 / p), row = (int)(r2 % p);
                const int i = pi_[k], j = pj_[k];
                if (j >= p) continue;
                cplx<T>* M = which ? E : A;
                const T c = pc[k], s = pr[k];
                const cplx<T> se = ps[k], e = ph[k];
                const cplx<T> xi = M[row + (int64_t)i * p], xj = M[row + (int64_t)j * p];
                cplx<T> ni = c * xi, nj = s * xi;
                cfma(ni, -se, xj);
                cfma(nj, c * e, xj);
                M[row + (int64_t)i * p] = ni;
                M[row + (int64_t)j * p] = nj;
            }
            __syncthreads();
        }
    }
    // sort eigenvalues descending (thread 0, insertion sort)
    for (int i = tid; i < p; i += 256) lam[i] = (double)A[i + (int64_t)i * p].re;
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < p; ++i) order[i] = i;
        for (int i = 1; i < p; ++i) {
            const int x = order[i];
            int j = i - 1;
            while (j >= 0 && lam[order[j]] < lam[x]) { order[j + 1] = order[j]; --j; }
            order[j + 1] = x;
        }
    }
    __syncthreads();
    const double l0 = fmax(lam[order[0]], 0.0);
    if (D.mode == 2 && tid == 0) {
        double tot = 0.0;
        for (int k = 0; k < p; ++k) tot += fmax(lam[order[k]], 0.0);
        double tail = 0.0;
        int r = p;
        for (int k = p - 1; k >= 0; --k) {
            tail += fmax(lam[order[k]], 0.0);
            if (tail > D.thr * D.thr * tot) break;
            r = k;
        }
        D.rank_out[0] = r;
    }
    for (int64_t e = tid; e < (int64_t)p * p; e += 256) {
        const int row = (int)(e % p), k = (int)(e / p);
        cplx<T> v = E[row + (int64_t)order[k] * p];
        if (D.mode == 1) {
            const double l = lam[order[k]];
            const T sc = (l > D.thr * l0 && l > 0.0) ? (T)(1.0 / sqrt(l)) : (T)0;
            v = sc * v;
        }
        D.E[row + (int64_t)k * p] = v;
    }
}
template <typename T>
void eig_batched(hipStream_t s, const EigDesc<T>* d_desc, int n) {
    if (n <= 0) return;
    k_heig_b<T><<<n, 256, 0, s>>>(d_desc, n);
    check_launch("k_heig_b");
}

#define CBIE_BATCH_INST(T)                                                                    \
    template void gemm_batched<T>(hipStream_t, const GemmDesc<T>*, const GemmTile*, int, int); \
    template void copy_batched<T>(hipStream_t, const CopyDesc<T>*, const CopyTile*, int);      \
    template void leaf_batched<T>(hipStream_t, const LeafDesc<T>*, int);                       \
    template void rand_batched<T>(hipStream_t, const RandDesc<T>*, int);                       \
    template void pchol_batched<T>(hipStream_t, const PcholDesc<T>*, int);                     \
    template void eig_batched<T>(hipStream_t, const EigDesc<T>*, int);
CBIE_BATCH_INST(double)
CBIE_BATCH_INST(float)

}  // namespace cbie

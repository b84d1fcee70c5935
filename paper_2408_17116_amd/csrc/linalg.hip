// Dense complex kernels of the H-LU: GEMM, leaf LU, triangular solves,
// transposes, conversions and ACA recompression of low-rank products.
#include "linalg.hpp"

namespace cbie {

template <typename T> __device__ inline cplx<T> czero() { return cplx<T>{(T)0, (T)0}; }

// ------------------------------------------------------------------ GEMM
// 64 x 64 output tile per work-group, K step 16 staged in LDS; thread
// (tx, ty) owns rows tx + 16 i and columns ty + 16 j (i, j < 4), so a wave
// stores 16 consecutive rows of 4 columns.
template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int m, int n, int k, cplx<T> alpha, const cplx<T>* __restrict__ A,
                                              int lda, const cplx<T>* __restrict__ B, int ldb, cplx<T> beta,
                                              cplx<T>* __restrict__ C, int ldc) {
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ cplx<T> As[BK][BM + 1];
    __shared__ cplx<T> Bs[BK][BN + 1];
    const int bm = blockIdx.x * BM, bn = blockIdx.y * BN;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    cplx<T> acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = czero<T>();
    for (int k0 = 0; k0 < k; k0 += BK) {
        for (int e = tid; e < BM * BK; e += 256) {
            int i, kk;
            if (!TA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
            const int gi = bm + i, gk = k0 + kk;
            cplx<T> v = czero<T>();
            if (gi < m && gk < k) v = TA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda];
            As[kk][i] = v;
        }
        for (int e = tid; e < BK * BN; e += 256) {
            int kk, j;
            if (!TB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
            const int gj = bn + j, gk = k0 + kk;
            cplx<T> v = czero<T>();
            if (gj < n && gk < k) v = TB ? B[gj + (int64_t)gk * ldb] : B[gk + (int64_t)gj * ldb];
            Bs[kk][j] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < BK; ++kk) {
            cplx<T> a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tx + 16 * i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][ty + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) cfma(acc[i][j], a[i], b[j]);
        }
        __syncthreads();
    }
    const bool zb = (beta.re == (T)0 && beta.im == (T)0);
    for (int j = 0; j < 4; ++j) {
        const int col = bn + ty + 16 * j;
        if (col >= n) continue;
        for (int i = 0; i < 4; ++i) {
            const int row = bm + tx + 16 * i;
            if (row >= m) continue;
            cplx<T>* cp = C + row + (int64_t)col * ldc;
            cplx<T> v = alpha * acc[i][j];
            if (!zb) cfma(v, beta, *cp);
            *cp = v;
        }
    }
}

template <typename T>
void gemm(hipStream_t s, char ta, char tb, int m, int n, int k, cplx<T> alpha, const cplx<T>* A, int lda,
          const cplx<T>* B, int ldb, cplx<T> beta, cplx<T>* C, int ldc) {
    if (m <= 0 || n <= 0) return;
    if (k <= 0) {
        copy_scale<T>(s, m, n, beta, C, ldc, C, ldc);
        return;
    }
    dim3 grid(ceil_div(m, 64), ceil_div(n, 64));
    const bool a = (ta == 'T'), b = (tb == 'T');
    if (!a && !b) k_gemm<T, false, false><<<grid, 256, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (!a && b) k_gemm<T, false, true><<<grid, 256, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (a && !b) k_gemm<T, true, false><<<grid, 256, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    else k_gemm<T, true, true><<<grid, 256, 0, s>>>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    check_launch("k_gemm");
}

// ---------------------------------------------------------------- reductions
struct AM {
    double v;
    int i;
};
__device__ inline AM am_better(AM a, AM b) { return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a; }
__device__ inline AM am_block(AM a, AM* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        AM o{__shfl_xor(a.v, off), __shfl_xor(a.i, off)};
        a = am_better(a, o);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    AM r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = am_better(r, sh[w]);
    return r;
}
__device__ inline double sum_block(double x, double* sh) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    return r;
}

// ---------------------------------------------------------------- leaf LU
// Right-looking LU with partial pivoting by panels of 16 columns, one
// work-group of 256 threads per matrix.
template <typename T>
__global__ __launch_bounds__(256) void k_getrf(int n, cplx<T>* __restrict__ A, int lda, int* __restrict__ piv,
                                               int* __restrict__ info) {
    constexpr int NB = 16;
    __shared__ AM sh[4];
    const int tid = threadIdx.x;
    int first_zero = 0;
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        for (int j = j0; j < j0 + jb; ++j) {
            AM a{-1.0, 0x7fffffff};
            for (int i = j + tid; i < n; i += 256) a = am_better(a, AM{(double)abs2(A[i + (int64_t)j * lda]), i});
            a = am_block(a, sh);
            const int p = a.i;
            if (tid == 0) piv[j] = p;
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
        // row swaps of the panel applied to the other columns
        for (int j = j0; j < j0 + jb; ++j) {
            const int p = piv[j];
            if (p != j)
                for (int c = tid; c < n; c += 256) {
                    if (c >= j0 && c < j0 + jb) continue;
                    const cplx<T> t = A[j + (int64_t)c * lda];
                    A[j + (int64_t)c * lda] = A[p + (int64_t)c * lda];
                    A[p + (int64_t)c * lda] = t;
                }
            __syncthreads();
        }
        // U12 = L11^{-1} A12 (thread per column)
        for (int c = j0 + jb + tid; c < n; c += 256) {
            for (int r = j0 + 1; r < j0 + jb; ++r) {
                cplx<T> v = A[r + (int64_t)c * lda];
                for (int t = j0; t < r; ++t) cfma(v, -A[r + (int64_t)t * lda], A[t + (int64_t)c * lda]);
                A[r + (int64_t)c * lda] = v;
            }
        }
        __syncthreads();
        // A22 -= L21 U12
        const int r0 = j0 + jb, R = n - r0;
        for (int64_t e = tid; e < (int64_t)R * R; e += 256) {
            const int i = r0 + (int)(e % R), c = r0 + (int)(e / R);
            cplx<T> v = A[i + (int64_t)c * lda];
            for (int t = j0; t < j0 + jb; ++t) cfma(v, -A[i + (int64_t)t * lda], A[t + (int64_t)c * lda]);
            A[i + (int64_t)c * lda] = v;
        }
        __syncthreads();
    }
    if (tid == 0) info[0] = first_zero;
}

template <typename T>
void getrf(hipStream_t s, int n, cplx<T>* A, int lda, int* piv, int* info) {
    k_getrf<T><<<1, 256, 0, s>>>(n, A, lda, piv, info);
    check_launch("k_getrf");
}

// ------------------------------------------------------ triangular solves
// thread per right-hand-side column
template <typename T>
__global__ void k_trsm_llnu_piv(int m, int n, const cplx<T>* __restrict__ LU, int ld, const int* __restrict__ piv,
                                cplx<T>* __restrict__ B, int ldb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    cplx<T>* b = B + (int64_t)c * ldb;
    for (int j = 0; j < m; ++j) {
        const int p = piv[j];
        if (p != j) { const cplx<T> t = b[j]; b[j] = b[p]; b[p] = t; }
    }
    for (int r = 1; r < m; ++r) {
        cplx<T> v = b[r];
        for (int t = 0; t < r; ++t) cfma(v, -LU[r + (int64_t)t * ld], b[t]);
        b[r] = v;
    }
}

template <typename T>
__global__ void k_trsm_lunn(int m, int n, const cplx<T>* __restrict__ LU, int ld, cplx<T>* __restrict__ B, int ldb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    cplx<T>* b = B + (int64_t)c * ldb;
    for (int r = m - 1; r >= 0; --r) {
        cplx<T> v = b[r];
        for (int t = r + 1; t < m; ++t) cfma(v, -LU[r + (int64_t)t * ld], b[t]);
        b[r] = cdiv(v, LU[r + (int64_t)r * ld]);
    }
}

// thread per row of B: x U = b, x_j = (b_j - sum_{i<j} x_i U_ij) / U_jj
template <typename T>
__global__ void k_trsm_runn(int m, int n, const cplx<T>* __restrict__ LU, int ld, cplx<T>* __restrict__ B, int ldb) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    for (int j = 0; j < n; ++j) {
        cplx<T> v = B[r + (int64_t)j * ldb];
        for (int i = 0; i < j; ++i) cfma(v, -B[r + (int64_t)i * ldb], LU[i + (int64_t)j * ld]);
        B[r + (int64_t)j * ldb] = cdiv(v, LU[j + (int64_t)j * ld]);
    }
}

template <typename T>
void trsm_llnu_piv(hipStream_t s, int m, int n, const cplx<T>* LU, int ld, const int* piv, cplx<T>* B, int ldb) {
    if (m <= 0 || n <= 0) return;
    k_trsm_llnu_piv<T><<<ceil_div(n, 64), 64, 0, s>>>(m, n, LU, ld, piv, B, ldb);
    check_launch("k_trsm_llnu_piv");
}
template <typename T>
void trsm_lunn(hipStream_t s, int m, int n, const cplx<T>* LU, int ld, cplx<T>* B, int ldb) {
    if (m <= 0 || n <= 0) return;
    k_trsm_lunn<T><<<ceil_div(n, 64), 64, 0, s>>>(m, n, LU, ld, B, ldb);
    check_launch("k_trsm_lunn");
}
template <typename T>
void trsm_runn(hipStream_t s, int m, int n, const cplx<T>* LU, int ld, cplx<T>* B, int ldb) {
    if (m <= 0 || n <= 0) return;
    k_trsm_runn<T><<<ceil_div(m, 64), 64, 0, s>>>(m, n, LU, ld, B, ldb);
    check_launch("k_trsm_runn");
}

// ----------------------------------------------------- copies, conversions
template <typename T>
__global__ void k_transpose(int m, int n, const cplx<T>* __restrict__ A, int lda, cplx<T>* __restrict__ B, int ldb) {
    __shared__ cplx<T> t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int i = bx + tx, j = by + k;
        if (i < m && j < n) t[k][tx] = A[i + (int64_t)j * lda];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int j = by + tx, i = bx + k;   // B(j, i) = A(i, j)
        if (i < m && j < n) B[j + (int64_t)i * ldb] = t[tx][k];
    }
}

template <typename T>
void transpose(hipStream_t s, int m, int n, const cplx<T>* A, int lda, cplx<T>* B, int ldb) {
    if (m <= 0 || n <= 0) return;
    k_transpose<T><<<dim3(ceil_div(m, 32), ceil_div(n, 32)), 256, 0, s>>>(m, n, A, lda, B, ldb);
    check_launch("k_transpose");
}

template <typename T>
__global__ void k_copy_scale(int m, int n, cplx<T> alpha, const cplx<T>* __restrict__ A, int lda,
                             cplx<T>* __restrict__ B, int ldb) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    const int i = (int)(e % m), j = (int)(e / m);
    B[i + (int64_t)j * ldb] = A ? alpha * A[i + (int64_t)j * lda] : czero<T>();
}

template <typename T>
void copy_scale(hipStream_t s, int m, int n, cplx<T> alpha, const cplx<T>* A, int lda, cplx<T>* B, int ldb) {
    if (m <= 0 || n <= 0) return;
    k_copy_scale<T><<<ceil_div((int64_t)m * n, 256), 256, 0, s>>>(m, n, alpha, A, lda, B, ldb);
    check_launch("k_copy_scale");
}

template <typename Tin, typename Tout>
__global__ void k_convert(int64_t n, const cplx<Tin>* __restrict__ a, cplx<Tout>* __restrict__ b) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) b[e] = cplx<Tout>{(Tout)a[e].re, (Tout)a[e].im};
}

// many conversions in one launch: work-group t converts elements
// [e0, e0 + 4096) of array desc
template <typename Tin, typename Tout>
__global__ void k_convert_b(const ConvDesc<Tin, Tout>* __restrict__ d, const ConvTile* __restrict__ t, int nt) {
    if ((int)blockIdx.x >= nt) return;
    const ConvTile tl = t[blockIdx.x];
    const ConvDesc<Tin, Tout> D = d[tl.desc];
    const int64_t e1 = min(D.n, tl.e0 + 4096);
    for (int64_t e = tl.e0 + threadIdx.x; e < e1; e += 256) D.b[e] = cplx<Tout>{(Tout)D.a[e].re, (Tout)D.a[e].im};
}
template <typename Tin, typename Tout>
void convert_batched(hipStream_t s, const std::vector<ConvDesc<Tin, Tout>>& v) {
    std::vector<ConvTile> t;
    for (size_t i = 0; i < v.size(); ++i)
        for (int64_t e0 = 0; e0 < v[i].n; e0 += 4096) t.push_back(ConvTile{(int)i, 0, e0});
    if (t.empty()) return;
    DBuf<ConvDesc<Tin, Tout>> dd;
    DBuf<ConvTile> dt;
    dd.upload(v, s);
    dt.upload(t, s);
    k_convert_b<Tin, Tout><<<(unsigned)t.size(), 256, 0, s>>>(dd.p, dt.p, (int)t.size());
    check_launch("k_convert_b");
    CBIE_HIP(hipStreamSynchronize(s));   // the descriptor buffers are released on return
}

// work-group t copies flat elements [e0, e0 + 4096) (column-major over
// m x n) of slice desc; consecutive threads take consecutive rows
template <typename Tin, typename Tout>
__global__ void k_slice_b(const SliceDesc<Tin, Tout>* __restrict__ d, const ConvTile* __restrict__ t, int nt) {
    if ((int)blockIdx.x >= nt) return;
    const ConvTile tl = t[blockIdx.x];
    const SliceDesc<Tin, Tout> D = d[tl.desc];
    const int64_t e1 = min((int64_t)D.m * D.n, tl.e0 + 4096);
    for (int64_t e = tl.e0 + threadIdx.x; e < e1; e += 256) {
        const int64_t i = e % D.m, j = e / D.m;
        const cplx<Tin> x = D.a[i * D.rs + j * D.cs];
        D.b[i + j * D.ldb] = cplx<Tout>{(Tout)x.re, (Tout)x.im};
    }
}
template <typename Tin, typename Tout>
void slice_batched(hipStream_t s, const std::vector<SliceDesc<Tin, Tout>>& v) {
    std::vector<ConvTile> t;
    for (size_t i = 0; i < v.size(); ++i)
        for (int64_t e0 = 0; e0 < (int64_t)v[i].m * v[i].n; e0 += 4096) t.push_back(ConvTile{(int)i, 0, e0});
    if (t.empty()) return;
    DBuf<SliceDesc<Tin, Tout>> dd;
    DBuf<ConvTile> dt;
    dd.upload(v, s);
    dt.upload(t, s);
    k_slice_b<Tin, Tout><<<(unsigned)t.size(), 256, 0, s>>>(dd.p, dt.p, (int)t.size());
    check_launch("k_slice_b");
    CBIE_HIP(hipStreamSynchronize(s));   // the descriptor buffers are released on return
}

// the same launch over descriptors and tiles already on the device
template <typename Tin, typename Tout>
void convert_batched_dev(hipStream_t s, const ConvDesc<Tin, Tout>* d, const ConvTile* t, int nt) {
    if (nt <= 0) return;
    k_convert_b<Tin, Tout><<<(unsigned)nt, 256, 0, s>>>(d, t, nt);
    check_launch("k_convert_b");
}

template <typename Tin, typename Tout>
void convert(hipStream_t s, int64_t n, const cplx<Tin>* a, cplx<Tout>* b) {
    if (n <= 0) return;
    k_convert<Tin, Tout><<<ceil_div(n, 256), 256, 0, s>>>(n, a, b);
    check_launch("k_convert");
}

// --------------------------------------------------- ACA of a product
// M = Ucat Vcat^T given in factored form (inner dimension K); the same
// partial-pivot ACA as for the kernel blocks, entries formed as dot
// products.  One work-group of 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_aca_prod(const AcaProdJob<T>* __restrict__ jobs, int njobs, double tol) {
    if ((int)blockIdx.x >= njobs) return;
    const AcaProdJob<T> J = jobs[blockIdx.x];
    const int m = J.m, n = J.n, K = J.K, cap = J.cap;
    const cplx<T>* __restrict__ Uc = J.Uc;
    const cplx<T>* __restrict__ Vc = J.Vc;
    cplx<T>* __restrict__ U = J.U;
    cplx<T>* __restrict__ V = J.V;
    unsigned char* __restrict__ used = J.used;
    const cplx<T>* __restrict__ Dd = J.D;
    __shared__ AM sh_am[4];
    __shared__ double sh_s[4];
    __shared__ cplx<T> s_row[2048];   // Ucat[i, :] or Vcat[j, :] (K <= 2048)
    __shared__ cplx<T> s_coef[1024];  // U[i, :rank] or V[j, :rank]
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += 256) used[i] = 0;
    // a plain dense input (K = 0): its Frobenius norm is computed exactly once
    // and stands in for the running estimate of the approximation's norm
    double dn2 = -1.0;
    if (K == 0 && Dd) {
        double a2 = 0.0;
        for (int64_t e = tid; e < (int64_t)m * n; e += 256) a2 += (double)abs2(Dd[e]);
        dn2 = sum_block(a2, sh_s);
    }
    __syncthreads();
    int irow = 0, rank = 0;
    double s2 = 0.0;
    while (rank < cap) {
        for (int l = tid; l < K; l += 256) s_row[l] = Uc[irow + (int64_t)l * m];
        for (int l = tid; l < rank; l += 256) s_coef[l] = U[irow + (int64_t)l * m];
        if (tid == 0) used[irow] = 1;
        __syncthreads();
        cplx<T>* vk = V + (int64_t)rank * n;
        AM am{-1.0, 0x7fffffff};
        for (int j = tid; j < n; j += 256) {
            cplx<T> r = Dd ? Dd[irow + (int64_t)j * m] : czero<T>();
            for (int l = 0; l < K; ++l) cfma(r, s_row[l], Vc[j + (int64_t)l * n]);
            for (int l = 0; l < rank; ++l) cfma(r, -s_coef[l], V[j + (int64_t)l * n]);
            vk[j] = r;
            am = am_better(am, AM{(double)abs2(r), j});
        }
        am = am_block(am, sh_am);
        if (am.v <= 0.0) {
            AM nx{-1.0, 0x7fffffff};
            for (int i = tid; i < m; i += 256)
                if (!used[i]) nx = am_better(nx, AM{0.0, i});
            nx = am_block(nx, sh_am);
            if (nx.v < 0.0) break;
            irow = nx.i;
            continue;
        }
        const int jp = am.i;
        const cplx<T> pv = vk[jp];
        __syncthreads();
        for (int j = tid; j < n; j += 256) vk[j] = cdiv(vk[j], pv);
        for (int l = tid; l < K; l += 256) s_row[l] = Vc[jp + (int64_t)l * n];
        for (int l = tid; l < rank; l += 256) s_coef[l] = V[jp + (int64_t)l * n];
        __syncthreads();
        cplx<T>* uk = U + (int64_t)rank * m;
        AM nx{-1.0, 0x7fffffff};
        double nu2 = 0.0;
        for (int i = tid; i < m; i += 256) {
            cplx<T> cc = Dd ? Dd[i + (int64_t)jp * m] : czero<T>();
            for (int l = 0; l < K; ++l) cfma(cc, Uc[i + (int64_t)l * m], s_row[l]);
            for (int l = 0; l < rank; ++l) cfma(cc, -s_coef[l], U[i + (int64_t)l * m]);
            uk[i] = cc;
            nu2 += (double)abs2(cc);
            if (!used[i]) nx = am_better(nx, AM{(double)abs2(cc), i});
        }
        double nv2 = 0.0;
        for (int j = tid; j < n; j += 256) nv2 += (double)abs2(vk[j]);
        nu2 = sum_block(nu2, sh_s);
        nv2 = sum_block(nv2, sh_s);
        nx = am_block(nx, sh_am);
        double cross = 0.0;
        if (dn2 < 0.0) {
            const int w = tid >> 6, lane = tid & 63;
            for (int l = w; l < rank; l += 4) {
                double ur = 0, ui = 0, vr = 0, vi = 0;
                for (int i = lane; i < m; i += 64) {
                    const cplx<T> x = U[i + (int64_t)l * m], y = uk[i];
                    ur += (double)x.re * y.re + (double)x.im * y.im;
                    ui += (double)x.re * y.im - (double)x.im * y.re;
                }
                for (int j = lane; j < n; j += 64) {
                    const cplx<T> x = V[j + (int64_t)l * n], y = vk[j];
                    vr += (double)x.re * y.re + (double)x.im * y.im;
                    vi += (double)x.re * y.im - (double)x.im * y.re;
                }
                for (int off = 32; off > 0; off >>= 1) {
                    ur += __shfl_xor(ur, off); ui += __shfl_xor(ui, off);
                    vr += __shfl_xor(vr, off); vi += __shfl_xor(vi, off);
                }
                cross += ur * vr - ui * vi;
            }
            cross = sum_block(lane == 0 ? cross : 0.0, sh_s);
        }
        s2 = dn2 >= 0.0 ? dn2 : s2 + 2.0 * cross + nu2 * nv2;
        ++rank;
        if (nu2 * nv2 <= tol * tol * fabs(s2)) break;
        if (nx.v < 0.0) break;
        irow = nx.i;
        __syncthreads();
    }
    if (tid == 0) J.rank_out[0] = rank;
}

template <typename T>
void aca_product_batched(hipStream_t s, int njobs, const AcaProdJob<T>* d_jobs, double tol) {
    if (njobs <= 0) return;
    k_aca_prod<T><<<njobs, 256, 0, s>>>(d_jobs, njobs, tol);
    check_launch("k_aca_prod");
}

// copy the first rank columns of the recompressed factors back (batched)
template <typename T>
__global__ void k_aca_copyback(const AcaProdJob<T>* __restrict__ jobs, int njobs) {
    const int jb = blockIdx.y;
    if (jb >= njobs) return;
    const AcaProdJob<T> J = jobs[jb];
    const int r = J.rank_out[0];
    const int64_t mu = (int64_t)J.m * r, nv = (int64_t)J.n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < mu + nv; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < mu) J.dstU[e] = J.U[e];
        else J.dstV[e - mu] = J.V[e - mu];
    }
}

template <typename T>
void aca_copyback_batched(hipStream_t s, int njobs, const AcaProdJob<T>* d_jobs) {
    if (njobs <= 0) return;
    k_aca_copyback<T><<<dim3(16, njobs), 256, 0, s>>>(d_jobs, njobs);
    check_launch("k_aca_copyback");
}

// ------------------------------------------------- leaf triangle inverses
// After P A = L U: LP = L^{-1} P (column c = L^{-1} P e_c) and UI = U^{-1},
// thread per column, loops uniform over rows so that the reads of L and U
// are wave-wide broadcasts.
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_inverse(int n, const cplx<T>* __restrict__ LU, int ld,
                                                      const int* __restrict__ piv, cplx<T>* __restrict__ LP,
                                                      cplx<T>* __restrict__ UI) {
    __shared__ int perm[1024];
    if (threadIdx.x == 0) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int j = 0; j < n; ++j) {            // P e_c: row positions after the swaps
            const int p = piv[j];
            const int t = perm[j]; perm[j] = perm[p]; perm[p] = t;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        // P e_c = e_s with s the position holding row c after the swaps
        int sidx = 0;
        for (int i = 0; i < n; ++i)
            if (perm[i] == c) sidx = i;
        cplx<T>* x = LP + (int64_t)c * n;
        for (int i = 0; i < n; ++i) {
            cplx<T> v = cplx<T>{(T)(i == sidx ? 1 : 0), (T)0};
            for (int t = 0; t < i; ++t) cfma(v, -LU[i + (int64_t)t * ld], x[t]);
            x[i] = (i < sidx) ? cplx<T>{(T)0, (T)0} : v;
        }
        cplx<T>* y = UI + (int64_t)c * n;
        for (int i = n - 1; i >= 0; --i) {
            cplx<T> v = cplx<T>{(T)(i == c ? 1 : 0), (T)0};
            for (int t = i + 1; t < n; ++t) cfma(v, -LU[i + (int64_t)t * ld], y[t]);
            y[i] = (i > c) ? cplx<T>{(T)0, (T)0} : cdiv(v, LU[i + (int64_t)i * ld]);
        }
    }
}

template <typename T>
void leaf_inverse(hipStream_t s, int n, const cplx<T>* LU, int ld, const int* piv, cplx<T>* LP, cplx<T>* UI) {
    CBIE_REQUIRE(n <= 1024, -7, "diagonal leaf larger than 1024 unknowns");
    k_leaf_inverse<T><<<1, 256, 0, s>>>(n, LU, ld, piv, LP, UI);
    check_launch("k_leaf_inverse");
}

// ----------------------------------------------------------- instances
#define CBIE_LINALG_INST(T)                                                                                   \
    template void gemm<T>(hipStream_t, char, char, int, int, int, cplx<T>, const cplx<T>*, int, const cplx<T>*, \
                          int, cplx<T>, cplx<T>*, int);                                                          \
    template void getrf<T>(hipStream_t, int, cplx<T>*, int, int*, int*);                                        \
    template void trsm_llnu_piv<T>(hipStream_t, int, int, const cplx<T>*, int, const int*, cplx<T>*, int);      \
    template void trsm_lunn<T>(hipStream_t, int, int, const cplx<T>*, int, cplx<T>*, int);                      \
    template void trsm_runn<T>(hipStream_t, int, int, const cplx<T>*, int, cplx<T>*, int);                      \
    template void transpose<T>(hipStream_t, int, int, const cplx<T>*, int, cplx<T>*, int);                      \
    template void copy_scale<T>(hipStream_t, int, int, cplx<T>, const cplx<T>*, int, cplx<T>*, int);            \
    template void aca_product_batched<T>(hipStream_t, int, const AcaProdJob<T>*, double);                      \
    template void aca_copyback_batched<T>(hipStream_t, int, const AcaProdJob<T>*);                             \
    template void leaf_inverse<T>(hipStream_t, int, const cplx<T>*, int, const int*, cplx<T>*, cplx<T>*);
CBIE_LINALG_INST(double)
CBIE_LINALG_INST(float)
template void convert_batched<double, float>(hipStream_t, const std::vector<ConvDesc<double, float>>&);
template void convert_batched<double, double>(hipStream_t, const std::vector<ConvDesc<double, double>>&);
template void slice_batched<double, float>(hipStream_t, const std::vector<SliceDesc<double, float>>&);
template void slice_batched<double, double>(hipStream_t, const std::vector<SliceDesc<double, double>>&);
template void convert_batched_dev<float, double>(hipStream_t, const ConvDesc<float, double>*, const ConvTile*, int);
template void convert_batched_dev<double, float>(hipStream_t, const ConvDesc<double, float>*, const ConvTile*, int);
template void convert<double, float>(hipStream_t, int64_t, const zd*, zf*);
template void convert<float, double>(hipStream_t, int64_t, const zf*, zd*);
template void convert<double, double>(hipStream_t, int64_t, const zd*, zd*);

}  // namespace cbie

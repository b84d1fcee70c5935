// Batched GEMM / copy / leaf-LU kernels driven by descriptor and tile lists.
#include "batch.hpp"

namespace cbie {

template <typename T> __device__ inline cplx<T> bz() { return cplx<T>{(T)0, (T)0}; }

// Operand pointers read from descriptors carry no address space, so their
// loads would be flat instructions, which count against the LDS wait
// counter as well: a wait for LDS reads would then also wait for every
// global load in flight (the prefetch of the next slice).  These casts say
// the memory is global.
template <typename T> using gptr = __attribute__((address_space(1))) cplx<T>*;
template <typename T> using gcptr = const __attribute__((address_space(1))) cplx<T>*;
template <typename T> __device__ inline gcptr<T> as_global(const cplx<T>* p) { return (gcptr<T>)p; }
template <typename T> __device__ inline gptr<T> as_global(cplx<T>* p) { return (gptr<T>)p; }
template <typename T> __device__ inline cplx<T> gld(gcptr<T> p) { return cplx<T>{p->re, p->im}; }
template <typename T> __device__ inline cplx<T> gld(gptr<T> p) { return cplx<T>{p->re, p->im}; }
template <typename T> __device__ inline void gst(gptr<T> p, cplx<T> v) {
    p->re = v.re;
    p->im = v.im;
}

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
// K3: the complex product by three real MFMAs (Karatsuba / "3M"):
//   P1 += Ar Br,  P2 += Ai Bi,  P3 += (Ar + Ai)(Br + Bi);
//   Cr = P1 - P2,  Ci = P3 - P1 - P2
// a quarter fewer matrix-core operations for one more accumulator set; the
// imaginary part is formed as a difference, so its rounding error grows with
// |Ar Br| + |Ai Bi| instead of |Ar Bi| + |Ai Br| (a small factor for
// operands of unrelated phases).
template <typename T, int BM, int BN, int WGM, int BK, bool K3 = false>
__global__ __launch_bounds__(256, K3 ? 4 : 1) void k_zgemm(const GemmDesc<T>* __restrict__ descs,
                                               const GemmTile* __restrict__ tiles, int ntiles) {
    constexpr int WGN = 4 / WGM, WM = BM / WGM, WN = BN / WGN, FM = WM / 16, FN = WN / 16;
    // one-element row padding: rows written lane by lane (transposing
    // stores) start two (complex64) or four (complex128) banks apart
    constexpr int PAD = 1;
    constexpr int NA = BM * BK / 256, NB = BK * BN / 256;
    static_assert(NA >= 1 && NB >= 1 && FM >= 1 && FN >= 1, "tile shape");
    typedef typename Mfma<T>::v4 v4;
    // two buffers per operand: slice i is read from one while slice i+1 is
    // written to the other, one barrier per slice
    __shared__ cplx<T> As[2][BK][BM + PAD];
    __shared__ cplx<T> Bs[2][BK][BN + PAD];
    // consecutive tiles (which share operand panels) go to one XCD: the
    // hardware deals work-groups round-robin over the 8 XCDs
    const int per = (int)gridDim.x >> 3;
    const int t = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (t >= ntiles) return;
    const GemmTile tl = tiles[t];
    const GemmDesc<T> D = descs[tl.desc];
    const int m = D.m, n = D.n, k = D.k;
    const int tn = (n + BN - 1) / BN;
    const int m0 = (tl.lt / tn) * BM, n0 = (tl.lt % tn) * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int r = lane & 15, kq = lane >> 4;

    v4 cr[FM][FN], ci[FM][FN], c3[K3 ? FM : 1][K3 ? FN : 1];
    for (int i = 0; i < FM; ++i)
        for (int j = 0; j < FN; ++j)
            for (int v = 0; v < 4; ++v) { cr[i][j][v] = (T)0; ci[i][j][v] = (T)0; }
    if (K3)
        for (int i = 0; i < FM; ++i)
            for (int j = 0; j < FN; ++j)
                for (int v = 0; v < 4; ++v) c3[K3 ? i : 0][K3 ? j : 0][v] = (T)0;

    // The next slice is fetched into registers while the current one is
    // multiplied: every load is issued unconditionally (out-of-range
    // elements read element 0 of the operand, which always exists), and the
    // range mask and the conjugation are applied only when the registers
    // are written to LDS, so no wait for the loads sits before the MFMAs.
    cplx<T> ra[NA], rb[NB];
    unsigned ma = 0, mb = 0;
    // element q of a slice: operand row i (column j) and depth kk, fixed for
    // the whole product; its offset is i ri + (k0 + kk) rk with the strides
    // of the operand's storage order, so no branch sits in the loop
    const gcptr<T> Ag = as_global(D.A);
    const gcptr<T> Bg = as_global(D.B);
    const int64_t a_ri = D.ta == 0 ? 1 : D.lda, a_rk = D.ta == 0 ? D.lda : 1;
    const int64_t b_rj = D.tb == 0 ? D.ldb : 1, b_rk = D.tb == 0 ? 1 : D.ldb;
    int ai[NA], ak[NA], bj[NB], bk[NB];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int e = tid + 256 * q;
        ai[q] = D.ta == 0 ? e % BM : e / BK;
        ak[q] = D.ta == 0 ? e / BM : e % BK;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = tid + 256 * q;
        bk[q] = D.tb == 0 ? e % BK : e / BN;
        bj[q] = D.tb == 0 ? e / BK : e % BN;
    }
    auto load = [&](int k0) {
        ma = 0;
        mb = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int gi = m0 + ai[q], gk = k0 + ak[q];
            const bool ok = gi < m && gk < k;
            ra[q] = gld<T>(Ag + (ok ? gi * a_ri + gk * a_rk : 0));
            ma |= (unsigned)ok << q;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int gj = n0 + bj[q], gk = k0 + bk[q];
            const bool ok = gj < n && gk < k;
            rb[q] = gld<T>(Bg + (ok ? gj * b_rj + gk * b_rk : 0));
            mb |= (unsigned)ok << q;
        }
    };
    auto stash = [&](int buf) {
        const T sa = D.ta == 2 ? (T)-1 : (T)1, sb = D.tb == 2 ? (T)-1 : (T)1;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const bool ok = (ma >> q) & 1u;
            As[buf][ak[q]][ai[q]] = cplx<T>{ok ? ra[q].re : (T)0, ok ? sa * ra[q].im : (T)0};
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const bool ok = (mb >> q) & 1u;
            Bs[buf][bk[q]][bj[q]] = cplx<T>{ok ? rb[q].re : (T)0, ok ? sb * rb[q].im : (T)0};
        }
    };
    load(0);
    stash(0);
    __syncthreads();
    for (int k0 = 0, cur = 0; k0 < k; k0 += BK, cur ^= 1) {
        // every wave finished the previous slice (last barrier), so buffer
        // cur ^ 1 is free; slice k0 is complete in buffer cur
        const bool more = k0 + BK < k;
        if (more) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            cplx<T> a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[cur][kk + kq][wm * WM + 16 * i + r];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = Bs[cur][kk + kq][wn * WN + 16 * j + r];
            if constexpr (K3) {
                // P1 in cr, P2 in ci, P3 in c3
                T sa[FM], sb[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) sa[i] = a[i].re + a[i].im;
#pragma unroll
                for (int j = 0; j < FN; ++j) sb[j] = b[j].re + b[j].im;
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        cr[i][j] = Mfma<T>::op(a[i].re, b[j].re, cr[i][j]);
                        ci[i][j] = Mfma<T>::op(a[i].im, b[j].im, ci[i][j]);
                        c3[K3 ? i : 0][K3 ? j : 0] = Mfma<T>::op(sa[i], sb[j], c3[K3 ? i : 0][K3 ? j : 0]);
                    }
            } else {
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
        if (more) stash(cur ^ 1);
        __syncthreads();
    }
    if constexpr (K3) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const T p1 = cr[i][j][v], p2 = ci[i][j][v];
                    cr[i][j][v] = p1 - p2;
                    ci[i][j][v] = c3[K3 ? i : 0][K3 ? j : 0][v] - p1 - p2;
                }
    }
    // Epilogue, one column group j at a time: every C value of the group is
    // loaded before any is stored (C is read and written through the same
    // pointer, so loads would otherwise wait for each preceding store).
    const bool zb = (D.beta.re == (T)0 && D.beta.im == (T)0);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn * WN + 16 * j + r;
        const bool cin = col < n;
        const gptr<T> ccol = as_global(D.C) + (int64_t)(cin ? col : 0) * D.ldc;
        cplx<T> old[FM][4];
        if (!zb) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = m0 + wm * WM + 16 * i + Mfma<T>::row(kq, v);
                    old[i][v] = gld<T>(ccol + ((cin && row < m) ? row : 0));   // masked below
                }
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm * WM + 16 * i + Mfma<T>::row(kq, v);
                if (!cin || row >= m) continue;
                cplx<T> o = D.alpha * cplx<T>{cr[i][j][v], ci[i][j][v]};
                if (!zb) cfma(o, D.beta, old[i][v]);
                gst<T>(ccol + row, o);
            }
    }
}

bool gemm_three_mult() {
    static const bool on = [] {
        const char* e = getenv("CBIE_GEMM_3M");
        return !e || atoi(e) != 0;
    }();
    return on;
}

template <typename T>
void gemm_batched(hipStream_t s, const GemmDesc<T>* d_desc, const GemmTile* d_tiles, int ntiles, int shape) {
    if (ntiles <= 0) return;
    const int grid = (ntiles + 7) / 8 * 8;
    constexpr int BKW = sizeof(T) == 4 ? 16 : 8;   // deep slices of the wide tiles fit LDS
    constexpr int BK64 = 16;
    const bool k3 = sizeof(T) == 4 && gemm_three_mult();
    switch (shape) {
        case kTile64x64:
            if constexpr (sizeof(T) == 4) {
                if (k3) {
                    k_zgemm<T, 64, 64, 2, BK64, true><<<grid, 256, 0, s>>>(d_desc, d_tiles, ntiles);
                    break;
                }
            }
            k_zgemm<T, 64, 64, 2, BK64><<<grid, 256, 0, s>>>(d_desc, d_tiles, ntiles);
            break;
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
    // sizes stay below 2^31 entries: 32-bit index arithmetic
    const unsigned m = (unsigned)D.m, tot = m * (unsigned)D.n;
    const unsigned e1 = min(tot, (unsigned)tl.e0 + (unsigned)kCopyChunk);
    for (unsigned e = (unsigned)tl.e0 + threadIdx.x; e < e1; e += 256) {
        const int i = (int)(e % m), j = (int)(e / m);
        cplx<T> v = bz<T>();
        if (D.A) {
            const gcptr<T> A = as_global(D.A);
            v = D.alpha * gld<T>(A + (D.trans ? j + (int64_t)i * D.lda : i + (int64_t)j * D.lda));
        }
        gst<T>(as_global(D.B) + i + (int64_t)j * D.ldb, v);
    }
}

template <typename T>
void copy_batched(hipStream_t s, const CopyDesc<T>* d_desc, const CopyTile* d_tiles, int ntiles) {
    if (ntiles <= 0) return;
    k_copy_b<T><<<ntiles, 256, 0, s>>>(d_desc, d_tiles, ntiles);
    check_launch("k_copy_b");
}

// ------------------------------------------------------ split-k reduction
template <typename T>
__global__ __launch_bounds__(256) void k_reduce_b(const ReduceDesc<T>* __restrict__ descs,
                                                  const CopyTile* __restrict__ tiles, int ntiles) {
    if ((int)blockIdx.x >= ntiles) return;
    const CopyTile tl = tiles[blockIdx.x];
    const ReduceDesc<T> D = descs[tl.desc];
    const unsigned m = (unsigned)D.m, tot = m * (unsigned)D.n;   // below 2^31 entries
    const unsigned e1 = min(tot, (unsigned)tl.e0 + (unsigned)kCopyChunk);
    const bool zb = D.beta.re == (T)0 && D.beta.im == (T)0;
    for (unsigned e = (unsigned)tl.e0 + threadIdx.x; e < e1; e += 256) {
        cplx<T> acc = bz<T>();
        const gcptr<T> W = as_global(D.W);
        for (int q = 0; q < D.nsplit; ++q) acc = acc + gld<T>(W + e + (size_t)q * tot);
        const int i = (int)(e % m), j = (int)(e / m);
        const gptr<T> cp = as_global(D.C) + i + (int64_t)j * D.ldc;
        cplx<T> o = D.alpha * acc;
        if (!zb) cfma(o, D.beta, gld<T>(cp));
        gst<T>(cp, o);
    }
}
template <typename T>
void reduce_batched(hipStream_t s, const ReduceDesc<T>* d_desc, const CopyTile* d_tiles, int ntiles) {
    if (ntiles <= 0) return;
    k_reduce_b<T><<<ntiles, 256, 0, s>>>(d_desc, d_tiles, ntiles);
    check_launch("k_reduce_b");
}

// ------------------------------------------------------- leaf LU + inverse
struct AMx {
    double v;
    int i;
};
__device__ inline AMx amx_better(AMx a, AMx b) { return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a; }

// One work-group of 256 threads per diagonal leaf (n <= 256).
// LU with partial pivoting, right-looking by 16-column panels: the panel
// is factored in LDS (column-major, one row per thread), its row swaps are
// applied to the other columns as one permutation of the rows they touch,
// U12 := L11^{-1} A12 by one thread per column, and A22 -= L21 U12 reads
// both factors from LDS with the global loads of 8 entries in flight.
template <typename T>
__global__ __launch_bounds__(256) void k_leaf_lu(const LeafDesc<T>* __restrict__ descs, int nd) {
    constexpr int NB = 16, NMAX = 256, UNR = 8;
    __shared__ cplx<T> PT[NB * NMAX];   // PT[t * NMAX + r] = A[j0 + r, j0 + t]
    __shared__ cplx<T> S[NB * NMAX];    // S[t * NMAX + c] = U12[t, c]
    __shared__ unsigned wmax[4];
    __shared__ int spiv[NB];
    __shared__ int aff[2 * NB], src[2 * NB];
    if ((int)blockIdx.x >= nd) return;
    const LeafDesc<T> D = descs[blockIdx.x];
    const int n = D.n, lda = D.lda;
    const gptr<T> A = as_global(D.A);
    const int tid = threadIdx.x;
    int first_zero = 0;
    for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0), R0 = n - j0, R1 = R0 - jb;
        for (int e = tid; e < R0 * jb; e += 256) {
            const int r = e % R0, t = e / R0;
            PT[t * NMAX + r] = gld<T>(A + j0 + r + (int64_t)(j0 + t) * lda);
        }
        __syncthreads();
        for (int jj = 0; jj < jb; ++jj) {
            // pivot: the largest |a|^2 in column jj; key = the top 24 bits of
            // its double (sign, exponent, 12 mantissa bits) above the
            // complemented row, so one wave maximum picks it (lowest row on
            // ties)
            unsigned key = 0u;
            if (tid >= jj && tid < R0) {
                const double v = (double)abs2(PT[jj * NMAX + tid]);
                key = ((unsigned)(__double_as_longlong(v) >> 40) << 8) | (unsigned)(255 - tid);
            }
            key = __ockl_wfred_max_u32(key);
            if ((tid & 63) == 0) wmax[tid >> 6] = key;
            __syncthreads();
            const unsigned best = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
            const int p = 255 - (int)(best & 255u);
            if (tid == 0) spiv[jj] = j0 + p;   // global stores stall a barrier: written per panel
            if (p != jj && tid < jb) {
                const cplx<T> x = PT[tid * NMAX + jj];
                PT[tid * NMAX + jj] = PT[tid * NMAX + p];
                PT[tid * NMAX + p] = x;
            }
            __syncthreads();
            const cplx<T> d = PT[jj * NMAX + jj];
            const bool nz = d.re != (T)0 || d.im != (T)0;
            if (!nz && first_zero == 0) first_zero = j0 + jj + 1;
            if (tid > jj && tid < R0 && nz) {
                const cplx<T> l = cdiv(PT[jj * NMAX + tid], d);
                cplx<T> pr[NB], my[NB];
#pragma unroll
                for (int t = 0; t < NB; ++t)
                    if (t > jj && t < jb) {
                        pr[t] = PT[t * NMAX + jj];
                        my[t] = PT[t * NMAX + tid];
                    }
                PT[jj * NMAX + tid] = l;
#pragma unroll
                for (int t = 0; t < NB; ++t)
                    if (t > jj && t < jb) {
                        cfma(my[t], -l, pr[t]);
                        PT[t * NMAX + tid] = my[t];
                    }
            }
            __syncthreads();
        }
        // the panel's swaps as one permutation of the rows they touch: slot q
        // moves original row src[q] to row aff[q] (src[q] < 0: unused); the
        // candidates are the panel rows and the first use of each pivot row
        // below the panel
        if (tid < 2 * NB) {
            int o = -1;
            if (tid < jb) {
                o = j0 + tid;
            } else if (tid >= NB && tid - NB < jb) {
                const int q = tid - NB, r = spiv[q];
                bool first = r >= j0 + jb;
                for (int u = 0; u < q; ++u)
                    if (spiv[u] == r) first = false;
                if (first) o = r;
            }
            int pos = o;
            if (o >= 0)
                for (int u = 0; u < jb; ++u) {
                    const int ra = j0 + u, rb = spiv[u];
                    if (pos == ra) pos = rb;
                    else if (pos == rb) pos = ra;
                }
            src[tid] = o;
            aff[tid] = pos;
        }
        for (int e = tid; e < R0 * jb; e += 256) {
            const int r = e % R0, t = e / R0;
            gst<T>(A + j0 + r + (int64_t)(j0 + t) * lda, PT[t * NMAX + r]);
        }
        if (tid < jb) D.piv[j0 + tid] = spiv[tid];
        __syncthreads();
        for (int c = tid; c < n; c += 256) {
            if (c >= j0 && c < j0 + jb) continue;
            cplx<T> v[2 * NB];
#pragma unroll
            for (int q = 0; q < 2 * NB; ++q)
                if (src[q] >= 0) v[q] = gld<T>(A + src[q] + (int64_t)c * lda);
#pragma unroll
            for (int q = 0; q < 2 * NB; ++q)
                if (src[q] >= 0) gst<T>(A + aff[q] + (int64_t)c * lda, v[q]);
        }
        __syncthreads();
        // U12 := L11^{-1} A12, one column per thread
        if (tid < R1) {
            const int c = j0 + jb + tid;
            cplx<T> v[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t)
                if (t < jb) v[t] = gld<T>(A + j0 + t + (int64_t)c * lda);
#pragma unroll
            for (int t = 1; t < NB; ++t)
#pragma unroll
                for (int u = 0; u < t; ++u)
                    if (t < jb) cfma(v[t], -PT[u * NMAX + t], v[u]);
#pragma unroll
            for (int t = 0; t < NB; ++t)
                if (t < jb) {
                    S[t * NMAX + tid] = v[t];
                    gst<T>(A + j0 + t + (int64_t)c * lda, v[t]);
                }
        }
        __syncthreads();
        // A22 -= L21 U12 on the matrix cores: 16 x 16 tiles, operands from
        // LDS, each wave updating 4 tiles at a time (their loads in flight
        // together)
        {
            typedef typename Mfma<T>::v4 v4;
            const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, cl = lane & 15;
            const int nt = (R1 + 15) / 16, ntt = nt * nt;
            for (int tb = 4 * wave; tb < ntt; tb += 16) {
                cplx<T> cv[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int tile = tb + q, r0 = 16 * (tile % nt), col = 16 * (tile / nt) + cl;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = r0 + Mfma<T>::row(g, v);
                        cv[q][v] = (tile < ntt && row < R1 && col < R1)
                                       ? gld<T>(A + j0 + jb + row + (int64_t)(j0 + jb + col) * lda)
                                       : bz<T>();
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int tile = tb + q;
                    if (tile >= ntt) break;
                    const int r0 = 16 * (tile % nt), c0 = 16 * (tile / nt), col = c0 + cl;
                    v4 cr, ci;
                    for (int v = 0; v < 4; ++v) { cr[v] = (T)0; ci[v] = (T)0; }
#pragma unroll
                    for (int k0 = 0; k0 < NB; k0 += 4) {
                        const int kk = k0 + g;
                        const cplx<T> x = (kk < jb && r0 + cl < R1) ? PT[kk * NMAX + jb + r0 + cl] : bz<T>();
                        const cplx<T> y = (kk < jb && col < R1) ? S[kk * NMAX + col] : bz<T>();
                        cr = Mfma<T>::op(x.re, y.re, cr);
                        cr = Mfma<T>::op(-x.im, y.im, cr);
                        ci = Mfma<T>::op(x.re, y.im, ci);
                        ci = Mfma<T>::op(x.im, y.re, ci);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = r0 + Mfma<T>::row(g, v);
                        if (row < R1 && col < R1)
                            gst<T>(A + j0 + jb + row + (int64_t)(j0 + jb + col) * lda,
                                   cplx<T>{cv[q][v].re - cr[v], cv[q][v].im - ci[v]});
                    }
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) D.info[0] = first_zero;
}

// Explicit inverses of a factored leaf, one work-group per column chunk:
// blockIdx.y = 0: chunk of UI = U^{-1} (column c is zero below row c);
// blockIdx.y = 1: chunk of LP = L^{-1} P (column j of L^{-1}, zero above
// row j, goes to column perm[j], perm = the row swaps applied to 0..n-1).
// The chunk is held row-major in LDS and built by block substitution over
// 16-row blocks: an update of all chunk columns by the finished blocks,
// then a 16 x 16 triangular solve per column; the 16 rows of the triangle
// in use are staged in LDS.
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_leaf_inv(const LeafDesc<T>* __restrict__ descs, int nd) {
    constexpr int NMAX = 256;
    __shared__ cplx<T> X[NMAX * CH];   // X[i * CH + cc]
    __shared__ cplx<T> B[16 * NMAX];   // B[r * NMAX + k]
    __shared__ int perm[NMAX];
    const int leaf = (int)blockIdx.x / (NMAX / CH), chunk = (int)blockIdx.x % (NMAX / CH);
    if (leaf >= nd) return;
    const LeafDesc<T> D = descs[leaf];
    const int n = D.n, lda = D.lda, c0 = chunk * CH;
    if (c0 >= n) return;
    const gcptr<T> A = as_global(D.A);
    const int tid = threadIdx.x, cw = min(CH, n - c0);
    for (int e = tid; e < n * CH; e += 256) X[e] = bz<T>();
    if (blockIdx.y == 0) {
        const int rows = min(n, c0 + cw);
        for (int I = (rows - 1) / 16; I >= 0; --I) {
            const int i0 = 16 * I, i1 = min(i0 + 16, rows);
            __syncthreads();
            for (int e = tid; e < 16 * (rows - i0); e += 256) {
                const int r = e % 16, k = i0 + e / 16;
                if (i0 + r < i1) B[r * NMAX + k] = gld<T>(A + i0 + r + (int64_t)k * lda);
            }
            __syncthreads();
            for (int e = tid; e < 16 * CH; e += 256) {
                const int r = e / CH, cc = e % CH, i = i0 + r;
                if (i >= i1 || cc >= cw) continue;
                cplx<T> v = cplx<T>{(T)(i == c0 + cc ? 1 : 0), (T)0};
                for (int k = i1; k < rows; ++k) cfma(v, -B[r * NMAX + k], X[k * CH + cc]);
                X[i * CH + cc] = v;
            }
            __syncthreads();
            if (tid < cw) {
                for (int i = i1 - 1; i >= i0; --i) {
                    const int r = i - i0;
                    cplx<T> v = X[i * CH + tid];
                    for (int k = i + 1; k < i1; ++k) cfma(v, -B[r * NMAX + k], X[k * CH + tid]);
                    X[i * CH + tid] = cdiv(v, B[r * NMAX + i]);
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < n * cw; e += 256) {
            const int i = e % n, cc = e / n;
            gst<T>(as_global(D.UI) + i + (int64_t)(c0 + cc) * n, X[i * CH + cc]);
        }
        return;
    }
    if (tid == 0) {
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int j = 0; j < n; ++j) {
            const int p = D.piv[j];
            const int t = perm[j];
            perm[j] = perm[p];
            perm[p] = t;
        }
    }
    const int nblk = (n + 15) / 16;
    for (int I = c0 / 16; I < nblk; ++I) {
        const int i0 = 16 * I, i1 = min(i0 + 16, n);
        __syncthreads();
        for (int e = tid; e < 16 * (i1 - c0); e += 256) {
            const int r = e % 16, k = c0 + e / 16;
            if (i0 + r < i1) B[r * NMAX + k] = gld<T>(A + i0 + r + (int64_t)k * lda);
        }
        __syncthreads();
        for (int e = tid; e < 16 * CH; e += 256) {
            const int r = e / CH, cc = e % CH, i = i0 + r;
            if (i >= i1 || cc >= cw) continue;
            cplx<T> v = cplx<T>{(T)(i == c0 + cc ? 1 : 0), (T)0};
            for (int k = c0; k < i0; ++k) cfma(v, -B[r * NMAX + k], X[k * CH + cc]);
            X[i * CH + cc] = v;
        }
        __syncthreads();
        if (tid < cw) {
            for (int i = i0 + 1; i < i1; ++i) {
                const int r = i - i0;
                cplx<T> v = X[i * CH + tid];
                for (int k = i0; k < i; ++k) cfma(v, -B[r * NMAX + k], X[k * CH + tid]);
                X[i * CH + tid] = v;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < n * cw; e += 256) {
        const int i = e % n, cc = e / n;
        gst<T>(as_global(D.LP) + i + (int64_t)perm[c0 + cc] * n, X[i * CH + cc]);
    }
}

template <typename T>
void leaf_batched(hipStream_t s, const LeafDesc<T>* d_desc, int n) {
    if (n <= 0) return;
    constexpr int CH = sizeof(T) == 4 ? 32 : 16;
    k_leaf_lu<T><<<n, 256, 0, s>>>(d_desc, n);
    check_launch("k_leaf_lu");
    k_leaf_inv<T, CH><<<dim3(n * (256 / CH), 2), 256, 0, s>>>(d_desc, n);
    check_launch("k_leaf_inv");
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
// LDS path (p <= PL): the Hermitian Gram matrix is copied to LDS as its
// upper triangle in physical indices, packed by columns (entry (a, b),
// a <= b, at a + b (b + 1) / 2; (b, a) is its conjugate), and factored
// there.  Pivoting permutes logical indices (perm) instead of moving data;
// pivots are chosen by one wave maximum of packed keys.  Row j of R is
// written over the slots {perm[j], perm[t]} (t > j), which no later step
// reads as Gram entries, and the downdate touches each remaining unordered
// pair once.  R^{-1} is then formed one column per wave: back substitution
// with lane-parallel sums.
template <typename T> struct PcholLds {
    // packed triangle plus four back-substitution vectors within 160 KB of LDS
    static constexpr int PL = sizeof(T) == 4 ? 128 : 132;
    static constexpr int SLOTS = PL * (PL + 1) / 2;
};
__device__ inline int tri_slot(int a, int b) {
    const int lo = min(a, b), hi = max(a, b);
    return lo + hi * (hi + 1) / 2;
}
template <typename T>
__device__ void pchol_lds(const PcholDesc<T>& D, cplx<T>* G, int* perm, unsigned* wmax, double* red,
                          cplx<T>* xs) {
    const int p = D.p, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const gcptr<T> Gg = as_global((const cplx<T>*)D.G);
    for (int b = wave; b < p; b += 4)
        for (int a = lane; a <= b; a += 64) G[a + b * (b + 1) / 2] = gld<T>(Gg + a + (int64_t)b * p);
    for (int i = tid; i < p; i += 256) perm[i] = i;
    __syncthreads();
    double m0 = 0.0;
    for (int i = tid; i < p; i += 256) m0 = fmax(m0, (double)G[i + i * (i + 1) / 2].re);
    for (int off = 32; off > 0; off >>= 1) m0 = fmax(m0, __shfl_xor(m0, off));
    if (lane == 0) red[wave] = m0;
    __syncthreads();
    const double dmax0 = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int k = p;
    for (int j = 0; j < p; ++j) {
        unsigned key = 0u;
        for (int t = j + tid; t < p; t += 256) {
            const int q = perm[t];
            const double v = fmax((double)G[q + q * (q + 1) / 2].re, 0.0);
            key = max(key, ((unsigned)(__double_as_longlong(v) >> 40) << 8) | (unsigned)(255 - t));
        }
        key = __ockl_wfred_max_u32(key);
        if (lane == 0) wmax[wave] = key;
        __syncthreads();
        const unsigned best = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
        const int bi = 255 - (int)(best & 255u);
        const int pj = perm[bi], pjo = perm[j];
        const double bv = (double)G[pj + pj * (pj + 1) / 2].re;
        if (!(bv > D.thr * dmax0) || bv <= 0.0) {
            k = j;
            break;
        }
        __syncthreads();   // every thread has read perm[j] and perm[bi]
        if (tid == 0) {
            perm[bi] = pjo;
            perm[j] = pj;
        }
        const T rjj = sqrt((T)bv);
        // row j of R: R[j, t] = G(pj, q) / rjj with q the physical index of
        // logical t > j (thread 0 changes only perm[j] and perm[bi])
        for (int t = j + 1 + tid; t < p; t += 256) {
            const int q = bi == t ? pjo : perm[t];
            const int sl = tri_slot(pj, q);
            const cplx<T> g = pj <= q ? G[sl] : conj(G[sl]);
            G[sl] = (T(1) / rjj) * g;
        }
        if (tid == 0) G[pj + pj * (pj + 1) / 2] = cplx<T>{rjj, (T)0};
        __syncthreads();
        // downdate G(a, b) -= conj(R[j, a]) R[j, b] over the unordered pairs of
        // the remaining logical indices, stored at (min, max)
        const int R = p - j - 1;
        for (int u = wave; u < R; u += 4) {
            const int b = perm[j + 1 + u];
            const cplx<T> rb = G[tri_slot(pj, b)];
            for (int t = lane; t <= u; t += 64) {
                const int a = perm[j + 1 + t];
                const cplx<T> ra = G[tri_slot(pj, a)];
                if (a <= b) cfma(G[tri_slot(a, b)], -conj(ra), rb);
                else cfma(G[tri_slot(a, b)], -conj(rb), ra);
            }
        }
        __syncthreads();
    }
    // S = Pi R^{-1}: column j of R^{-1} solves R x = e_j (x zero below j);
    // R[t, u] (t < u) sits in slot {perm[t], perm[u]}
    cplx<T>* x = xs + wave * PcholLds<T>::PL;
    const gptr<T> Sg = as_global(D.S);
    for (int e = tid; e < p * p; e += 256) gst<T>(Sg + e, bz<T>());
    __syncthreads();
    for (int j = wave; j < k; j += 4) {
        for (int t = j; t >= 0; --t) {
            cplx<T> acc = bz<T>();
            const int pt = perm[t];
            for (int u = t + 1 + lane; u <= j; u += 64) cfma(acc, G[tri_slot(pt, perm[u])], x[u]);
            for (int off = 32; off > 0; off >>= 1) {
                acc.re += __shfl_xor(acc.re, off);
                acc.im += __shfl_xor(acc.im, off);
            }
            const cplx<T> num = cplx<T>{(T)(t == j ? 1 : 0), (T)0} - acc;
            const cplx<T> xt = cdiv(num, G[pt + pt * (pt + 1) / 2]);
            if (lane == 0) x[t] = xt;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        }
        for (int t = lane; t <= j; t += 64) gst<T>(Sg + perm[t] + (int64_t)j * p, x[t]);
        __builtin_amdgcn_wave_barrier();
    }
    if (tid == 0) D.k_out[0] = k;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pchol_b(const PcholDesc<T>* __restrict__ descs, int nd) {
    if ((int)blockIdx.x >= nd) return;
    const PcholDesc<T> D = descs[blockIdx.x];
    const int p = D.p;
    constexpr int PL = PcholLds<T>::PL;
    static_assert(PcholLds<T>::SLOTS >= 4 * 512, "back-substitution vectors");
    __shared__ int perm[512];
    // the packed matrix when p <= PL; on the global path the pivot row
    // during the factorization, then R packed (rank <= PL) or the vectors
    // of the back substitution
    __shared__ cplx<T> Gl[PcholLds<T>::SLOTS];
    __shared__ cplx<T> xs[4 * PL];
    {
        __shared__ unsigned wmax[4];
        __shared__ double red[4];
        if (p <= PL) {
            pchol_lds<T>(D, Gl, perm, wmax, red, xs);
            return;
        }
    }
    // larger matrices in global memory, rows and columns swapped in place
    const gptr<T> G = as_global(D.G);
    __shared__ double dv[4];
    __shared__ int di[4];
    __shared__ double dmax0;
    __shared__ int kk;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < p; i += 256) perm[i] = i;
    if (tid == 0) {
        double m0 = 0.0;
        for (int i = 0; i < p; ++i) m0 = fmax(m0, (double)G[i + (int64_t)i * p].re);
        dmax0 = m0;
        kk = p;
    }
    __syncthreads();
    cplx<T>* rrow = Gl;   // row j of R, indexed by column
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
                const cplx<T> a = gld<T>(G + j + (int64_t)t * p);
                gst<T>(G + j + (int64_t)t * p, gld<T>(G + bi + (int64_t)t * p));
                gst<T>(G + bi + (int64_t)t * p, a);
            }
            __syncthreads();
            for (int t = tid; t < p; t += 256) {
                const cplx<T> a = gld<T>(G + t + (int64_t)j * p);
                gst<T>(G + t + (int64_t)j * p, gld<T>(G + t + (int64_t)bi * p));
                gst<T>(G + t + (int64_t)bi * p, a);
            }
            if (tid == 0) { const int x = perm[j]; perm[j] = perm[bi]; perm[bi] = x; }
            __syncthreads();
        }
        // row j of R: R[j, j] = sqrt(G[j, j]), R[j, t] = G[j, t] / R[j, j],
        // kept in LDS for the downdate
        const T rjj = sqrt((T)bv);
        for (int t = j + 1 + tid; t < p; t += 256) {
            const cplx<T> v = (T(1) / rjj) * gld<T>(G + j + (int64_t)t * p);
            gst<T>(G + j + (int64_t)t * p, v);
            rrow[t] = v;
        }
        if (tid == 0) gst<T>(G + j + (int64_t)j * p, cplx<T>{rjj, (T)0});
        __syncthreads();
        // trailing downdate G[t, u] -= conj(R[j, t]) R[j, u], t, u > j: lanes
        // along columns (coalesced), four elements in flight per thread
        const unsigned R = (unsigned)(p - j - 1), RR = R * R;
        for (unsigned e0 = tid; e0 < RR; e0 += 4 * 256) {
            cplx<T> v[4];
            gptr<T> g[4];
            cplx<T> rt[4], ru[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned e = e0 + 256u * q;
                const unsigned t = e < RR ? e % R : 0u, u = e < RR ? e / R : 0u;
                g[q] = G + (j + 1 + (int)t) + (int64_t)(j + 1 + (int)u) * p;
                rt[q] = rrow[j + 1 + t];
                ru[q] = rrow[j + 1 + u];
                if (e < RR) v[q] = gld<T>(g[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (e0 + 256u * q < RR) {
                    cfma(v[q], -conj(rt[q]), ru[q]);
                    gst<T>(g[q], v[q]);
                }
        }
        __syncthreads();
    }
    __syncthreads();
    const int k = kk;
    // S = Pi R_kk^{-1}: column j solves R x = e_j by back substitution, one
    // wave per column with its lanes over the inner sums.  R (upper, k x k)
    // is staged in LDS, packed by columns, when it fits; x in LDS
    const gptr<T> Sg = as_global(D.S);
    for (int64_t e = tid; e < (int64_t)p * p; e += 256) gst<T>(Sg + e, bz<T>());
    const bool rl = k <= PL;
    if (rl)
        for (int u = wave; u < k; u += 4)
            for (int t = lane; t <= u; t += 64) Gl[t + u * (u + 1) / 2] = gld<T>(G + t + (int64_t)u * p);
    __syncthreads();
    cplx<T>* x = rl ? xs + wave * PL : Gl + wave * 512;
    for (int j = wave; j < k; j += 4) {
        for (int t = j; t >= 0; --t) {
            cplx<T> acc = bz<T>();
            if (rl)
                for (int u = t + 1 + lane; u <= j; u += 64) cfma(acc, Gl[t + u * (u + 1) / 2], x[u]);
            else
                for (int u = t + 1 + lane; u <= j; u += 64) cfma(acc, gld<T>(G + t + (int64_t)u * p), x[u]);
            for (int off = 32; off > 0; off >>= 1) {
                acc.re += __shfl_xor(acc.re, off);
                acc.im += __shfl_xor(acc.im, off);
            }
            const cplx<T> num = cplx<T>{(T)(t == j ? 1 : 0), (T)0} - acc;
            const cplx<T> xt = cdiv(num, rl ? Gl[t + t * (t + 1) / 2] : gld<T>(G + t + (int64_t)t * p));
            if (lane == 0) x[t] = xt;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        }
        for (int t = lane; t <= j; t += 64) gst<T>(Sg + perm[t] + (int64_t)j * p, x[t]);
        __builtin_amdgcn_wave_barrier();
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
    template void reduce_batched<T>(hipStream_t, const ReduceDesc<T>*, const CopyTile*, int);  \
    template void leaf_batched<T>(hipStream_t, const LeafDesc<T>*, int);                       \
    template void rand_batched<T>(hipStream_t, const RandDesc<T>*, int);                       \
    template void pchol_batched<T>(hipStream_t, const PcholDesc<T>*, int);                     \
    template void eig_batched<T>(hipStream_t, const EigDesc<T>*, int);
CBIE_BATCH_INST(double)
CBIE_BATCH_INST(float)

}  // namespace cbie

// H-LU factorization and H forward/back substitution (Sec. III, eqs. 23-28)
// with formatted (truncated) low-rank arithmetic, complex64 or complex128.
//
// Recursion over the block cluster tree.  For a diagonal block with
// children (t1, t2):
//   HLU(A11);  A12 := L11^{-1} A12;  A21 := A21 U11^{-1};
//   A22 := A22 - A21 A12 (formatted);  HLU(A22).
// Leaves: LU with partial pivoting inside the diagonal leaf (P A = L U),
// no pivoting across blocks.  Updates of low-rank blocks are accumulated as
// low-rank terms and recompressed once, by ACA of the summed factors, when
// the block is next read ("lazy" formatted addition).
#include <algorithm>
#include <cmath>
#include <functional>

#include "ctx.hpp"
#include "linalg.hpp"
#include "ops.hpp"

namespace cbie {

// bump allocator over device chunks; pointers stay valid until reset
template <typename T> struct Arena {
    std::vector<DBuf<cplx<T>>> chunks;
    std::vector<size_t> used;
    size_t chunk_elems = size_t(1) << 26;   // 1 GiB of complex128 per chunk
    int cur = -1;
    size_t total = 0;
    cplx<T>* alloc(size_t n) {
        n = (n + 31) & ~size_t(31);
        if (n == 0) n = 32;
        if (cur < 0 && !chunks.empty()) cur = 0;   // chunks kept by a release to the empty mark
        while (cur >= 0 && cur + 1 < (int)chunks.size() && used[cur] + n > chunks[cur].n) {
            ++cur;   // reuse a chunk kept by an earlier release
        }
        if (cur < 0 || used[cur] + n > chunks[cur].n) {
            DBuf<cplx<T>> b;
            b.alloc(std::max(n, chunk_elems));
            chunks.push_back(std::move(b));
            used.push_back(0);
            cur = (int)chunks.size() - 1;
        }
        cplx<T>* p = chunks[cur].p + used[cur];
        used[cur] += n;
        total += n;
        return p;
    }
    struct Mark {
        int cur;
        size_t used;
    };
    Mark mark() const { return Mark{cur, cur >= 0 ? used[cur] : 0}; }
    // stream ordering makes reuse safe: later kernels run after earlier ones
    void release(Mark m) {
        for (int k = m.cur + 1; k <= cur; ++k) used[k] = 0;
        cur = m.cur;
        if (cur >= 0) used[cur] = m.used;
    }
};

template <typename T> struct HF {
    Ctx& c;
    hipStream_t s;
    const Tree& T_;
    double tol;
    DBuf<cplx<T>> dense;
    std::vector<int64_t> piv_off;   // per dense block (diagonal leaves), -1 otherwise
    DBuf<int> piv, info;
    // A low-rank block U V^T.  The factors live in accumulation buffers of
    // `cap` columns: columns [0, r) hold the current factors, columns
    // [r, K) hold pending update terms (zero outside their row / column
    // ranges), recompressed together when the block is next read.
    struct LR {
        cplx<T>* U;
        cplx<T>* V;
        int m, n, r;
        int K = 0, cap = 0;
    };
    std::vector<LR> lr;
    Arena<T> arena, scratch;
    DBuf<unsigned char> used;
    DBuf<int> d_rank;
    int64_t launches = 0;
    double flops = 0.0;

    struct View {
        int blk = -1;        // block node, or -1 for a raw dense buffer
        int r0 = 0, c0 = 0;  // offset inside a leaf block
        int m = 0, n = 0;
        int rc = -1, cc = -1;   // row / column cluster (-1: not split)
        cplx<T>* p = nullptr;   // raw buffer (already offset)
        int ld = 0;
    };
    enum Kind { RAW, DENSE, LRK, HIER };

    HF(Ctx& cc, double t) : c(cc), s(cc.stream), T_(cc.tree), tol(t) {}

    // ------------------------------------------------------------- helpers
    int kind(const View& v) const {
        if (v.blk < 0) return RAW;
        const int ty = T_.blocks[v.blk].type;
        return ty == BLK_DENSE ? DENSE : (ty == BLK_LR ? LRK : HIER);
    }
    int nunk(int cl) const { return (int)T_.clusters[cl].nunk(); }
    View full(int blk) const {
        const Block& b = T_.blocks[blk];
        View v;
        v.blk = blk;
        v.rc = b.t;
        v.cc = b.s;
        v.m = nunk(b.t);
        v.n = nunk(b.s);
        return v;
    }
    View raw(cplx<T>* p, int ld, int m, int n, int rc, int cc) const {
        View v;
        v.p = p; v.ld = ld; v.m = m; v.n = n; v.rc = rc; v.cc = cc;
        return v;
    }
    View sub(const View& v, int ri, int ci) const {
        if (kind(v) == HIER) {
            const Block& b = T_.blocks[v.blk];
            return full(b.child[ri * 2 + ci]);
        }
        View w = v;
        if (ri >= 0) {
            const Cluster& cl = T_.clusters[v.rc];
            const int ch = cl.child[ri];
            const int off = ri == 0 ? 0 : nunk(cl.child[0]);
            w.rc = ch;
            w.m = nunk(ch);
            if (v.blk < 0) w.p += off; else w.r0 += off;
        }
        if (ci >= 0) {
            const Cluster& cl = T_.clusters[v.cc];
            const int ch = cl.child[ci];
            const int off = ci == 0 ? 0 : nunk(cl.child[0]);
            w.cc = ch;
            w.n = nunk(ch);
            if (v.blk < 0) w.p += (int64_t)off * v.ld; else w.c0 += off;
        }
        return w;
    }
    // dense pointer / leading dimension of a RAW or DENSE view
    cplx<T>* dptr(const View& v, int& ld) const {
        if (v.blk < 0) { ld = v.ld; return v.p; }
        const DenseBlockDev& d = c.dblk[T_.blocks[v.blk].leaf_index];
        ld = d.ld;
        return dense.p + d.offset + (int64_t)v.c0 * d.ld + v.r0;
    }
    LR& lrb(const View& v) { return lr[T_.blocks[v.blk].leaf_index]; }

    // counted launches
    void g(char ta, char tb, int m, int n, int k, cplx<T> al, const cplx<T>* A, int lda, const cplx<T>* B, int ldb,
           cplx<T> be, cplx<T>* C, int ldc) {
        if (m <= 0 || n <= 0) return;
        gemm<T>(s, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc);
        ++launches;
        flops += 8.0 * m * n * std::max(k, 0);
    }
    static cplx<T> one() { return cplx<T>{(T)1, (T)0}; }
    static cplx<T> zero() { return cplx<T>{(T)0, (T)0}; }
    static cplx<T> neg() { return cplx<T>{(T)-1, (T)0}; }

    // ------------------------------------------------- lazy low-rank sums
    void flush_block(int leaf) {
        LR& L = lr[leaf];
        if (L.K == L.r) return;
        const int m = L.m, n = L.n, K = L.K;
        auto mk = scratch.mark();
        const int cap = std::min({m, n, K, 1024});
        cplx<T>* U = scratch.alloc((size_t)m * cap);
        cplx<T>* V = scratch.alloc((size_t)n * cap);
        aca_product<T>(s, m, n, K, L.U, L.V, tol, cap, U, V, used.p, d_rank.p);
        ++launches;
        int r = 0;
        CBIE_HIP(hipMemcpyAsync(&r, d_rank.p, sizeof(int), hipMemcpyDeviceToHost, s));
        CBIE_HIP(hipStreamSynchronize(s));
        flops += 8.0 * (double)(m + n) * K * r;   // entries of r rows and columns
        copy_scale<T>(s, m, r, one(), U, m, L.U, m);
        copy_scale<T>(s, n, r, one(), V, n, L.V, n);
        launches += 2;
        scratch.release(mk);
        L.r = L.K = r;
    }
    void flush(const View& v) {
        if (v.blk >= 0 && kind(v) == LRK) flush_block(T_.blocks[v.blk].leaf_index);
    }
    // room for k more term columns of block C; returns the first new column
    // (zeroed).  X goes to U + col m + r0, Y to V + col n + c0.
    int reserve(const View& C, int k) {
        const int leaf = T_.blocks[C.blk].leaf_index;
        LR& L = lr[leaf];
        if (L.K + k > 1024) flush_block(leaf);
        if (L.K + k > L.cap) {
            const int nc = std::max(L.K + k, 2 * L.cap);
            cplx<T>* U = arena.alloc((size_t)L.m * nc);
            cplx<T>* V = arena.alloc((size_t)L.n * nc);
            if (L.K > 0) {
                copy_scale<T>(s, L.m, L.K, one(), L.U, L.m, U, L.m);
                copy_scale<T>(s, L.n, L.K, one(), L.V, L.n, V, L.n);
                launches += 2;
            }
            L.U = U;
            L.V = V;
            L.cap = nc;
        }
        const int col = L.K;
        copy_scale<T>(s, L.m, k, zero(), nullptr, L.m, L.U + (int64_t)col * L.m, L.m);
        copy_scale<T>(s, L.n, k, zero(), nullptr, L.n, L.V + (int64_t)col * L.n, L.n);
        launches += 2;
        L.K += k;
        return col;
    }

    // ------------------------------------------------------ C += alpha A B
    void update(const View& C, const View& A, const View& B, cplx<T> al) {
        const bool hc = kind(C) == HIER, ha = kind(A) == HIER, hb = kind(B) == HIER;
        if (hc || ha || hb) {
            const bool sr = hc || ha, sm = ha || hb, sc = hc || hb;
            for (int i = (sr ? 0 : -1); i < (sr ? 2 : 0); ++i)
                for (int j = (sc ? 0 : -1); j < (sc ? 2 : 0); ++j)
                    for (int k = (sm ? 0 : -1); k < (sm ? 2 : 0); ++k)
                        update(sub(C, i, j), sub(A, i, k), sub(B, k, j), al);
            return;
        }
        flush(A);
        flush(B);
        const int kA = kind(A), kB = kind(B), kC = kind(C);
        const bool dA = kA != LRK, dB = kB != LRK;
        auto mk = scratch.mark();
        if (kC != LRK) {
            int ldc;
            cplx<T>* Cp = dptr(C, ldc);
            if (dA && dB) {
                int lda, ldb;
                cplx<T>* Ap = dptr(A, lda);
                cplx<T>* Bp = dptr(B, ldb);
                g('N', 'N', C.m, C.n, A.n, al, Ap, lda, Bp, ldb, one(), Cp, ldc);
            } else if (!dA) {
                LR& La = lrb(A);
                const int ra = La.r;
                if (ra > 0) {
                    const cplx<T>* Ua = La.U + A.r0;
                    const cplx<T>* Va = La.V + A.c0;
                    cplx<T>* Tm = scratch.alloc((size_t)ra * C.n);
                    if (dB) {
                        int ldb;
                        cplx<T>* Bp = dptr(B, ldb);
                        g('T', 'N', ra, C.n, B.m, one(), Va, La.n, Bp, ldb, zero(), Tm, ra);
                    } else {
                        LR& Lb = lrb(B);
                        const int rb = Lb.r;
                        cplx<T>* W = scratch.alloc((size_t)ra * std::max(rb, 1));
                        if (rb > 0) {
                            g('T', 'N', ra, rb, B.m, one(), Va, La.n, Lb.U + B.r0, Lb.m, zero(), W, ra);
                            g('N', 'T', ra, C.n, rb, one(), W, ra, Lb.V + B.c0, Lb.n, zero(), Tm, ra);
                        } else {
                            copy_scale<T>(s, ra, C.n, zero(), nullptr, ra, Tm, ra);
                            ++launches;
                        }
                    }
                    g('N', 'N', C.m, C.n, ra, al, Ua, La.m, Tm, ra, one(), Cp, ldc);
                }
            } else {
                LR& Lb = lrb(B);
                const int rb = Lb.r;
                if (rb > 0) {
                    int lda;
                    cplx<T>* Ap = dptr(A, lda);
                    cplx<T>* Tm = scratch.alloc((size_t)C.m * rb);
                    g('N', 'N', C.m, rb, A.n, one(), Ap, lda, Lb.U + B.r0, Lb.m, zero(), Tm, C.m);
                    g('N', 'T', C.m, C.n, rb, al, Tm, C.m, Lb.V + B.c0, Lb.n, one(), Cp, ldc);
                }
            }
            scratch.release(mk);
            return;
        }
        // C low rank: append the product as X Y^T, recompressed when C is read
        scratch.release(mk);
        LR& Lc = lrb(C);
        if (!dA) {
            LR& La = lrb(A);
            const int ra = La.r;
            if (ra == 0) return;
            const cplx<T>* Va = La.V + A.c0;
            if (!dB && lrb(B).r == 0) return;
            const int col = reserve(C, ra);
            cplx<T>* X = Lc.U + (int64_t)col * Lc.m + C.r0;
            cplx<T>* Y = Lc.V + (int64_t)col * Lc.n + C.c0;
            copy_scale<T>(s, C.m, ra, al, La.U + A.r0, La.m, X, Lc.m);
            ++launches;
            if (dB) {
                int ldb;
                cplx<T>* Bp = dptr(B, ldb);
                g('T', 'N', C.n, ra, B.m, one(), Bp, ldb, Va, La.n, zero(), Y, Lc.n);
            } else {
                LR& Lb = lrb(B);
                const int rb = Lb.r;
                auto mk2 = scratch.mark();
                cplx<T>* W = scratch.alloc((size_t)rb * ra);
                g('T', 'N', rb, ra, B.m, one(), Lb.U + B.r0, Lb.m, Va, La.n, zero(), W, rb);
                g('N', 'N', C.n, ra, rb, one(), Lb.V + B.c0, Lb.n, W, rb, zero(), Y, Lc.n);
                scratch.release(mk2);
            }
        } else if (!dB) {
            LR& Lb = lrb(B);
            const int rb = Lb.r;
            if (rb == 0) return;
            int lda;
            cplx<T>* Ap = dptr(A, lda);
            const int col = reserve(C, rb);
            cplx<T>* X = Lc.U + (int64_t)col * Lc.m + C.r0;
            cplx<T>* Y = Lc.V + (int64_t)col * Lc.n + C.c0;
            g('N', 'N', C.m, rb, A.n, al, Ap, lda, Lb.U + B.r0, Lb.m, zero(), X, Lc.m);
            copy_scale<T>(s, C.n, rb, one(), Lb.V + B.c0, Lb.n, Y, Lc.n);
            ++launches;
        } else {
            int lda, ldb;
            cplx<T>* Ap = dptr(A, lda);
            cplx<T>* Bp = dptr(B, ldb);
            const int k = A.n;
            const int col = reserve(C, k);
            cplx<T>* X = Lc.U + (int64_t)col * Lc.m + C.r0;
            cplx<T>* Y = Lc.V + (int64_t)col * Lc.n + C.c0;
            copy_scale<T>(s, C.m, k, al, Ap, lda, X, Lc.m);
            transpose<T>(s, B.m, B.n, Bp, ldb, Y, Lc.n);
            launches += 2;
        }
    }

    // --------------------------------------------------- triangular solves
    // X (|d| x ncol) := L_dd^{-1} X   (L includes the leaf pivots)
    void solveL(int d, cplx<T>* X, int ldx, int ncol) {
        const Block& D = T_.blocks[d];
        if (D.type == BLK_DENSE) {
            const DenseBlockDev& db = c.dblk[D.leaf_index];
            trsm_llnu_piv<T>(s, db.ld, ncol, dense.p + db.offset, db.ld, piv.p + piv_off[D.leaf_index], X, ldx);
            ++launches;
            flops += 4.0 * db.ld * db.ld * ncol;
            return;
        }
        const Cluster& ct = T_.clusters[D.t];
        const int n1 = nunk(ct.child[0]), n2 = nunk(ct.child[1]);
        solveL(D.child[0], X, ldx, ncol);
        update(raw(X + n1, ldx, n2, ncol, ct.child[1], -1), full(D.child[2]), raw(X, ldx, n1, ncol, ct.child[0], -1),
               neg());
        solveL(D.child[3], X + n1, ldx, ncol);
    }
    // X (|d| x ncol) := U_dd^{-1} X
    void solveU(int d, cplx<T>* X, int ldx, int ncol) {
        const Block& D = T_.blocks[d];
        if (D.type == BLK_DENSE) {
            const DenseBlockDev& db = c.dblk[D.leaf_index];
            trsm_lunn<T>(s, db.ld, ncol, dense.p + db.offset, db.ld, X, ldx);
            ++launches;
            flops += 4.0 * db.ld * db.ld * ncol;
            return;
        }
        const Cluster& ct = T_.clusters[D.t];
        const int n1 = nunk(ct.child[0]), n2 = nunk(ct.child[1]);
        solveU(D.child[3], X + n1, ldx, ncol);
        update(raw(X, ldx, n1, ncol, ct.child[0], -1), full(D.child[1]), raw(X + n1, ldx, n2, ncol, ct.child[1], -1),
               neg());
        solveU(D.child[0], X, ldx, ncol);
    }
    // X (nrow x |d|) := X U_dd^{-1}
    void solveUr(int d, cplx<T>* X, int ldx, int nrow) {
        const Block& D = T_.blocks[d];
        if (D.type == BLK_DENSE) {
            const DenseBlockDev& db = c.dblk[D.leaf_index];
            trsm_runn<T>(s, nrow, db.ld, dense.p + db.offset, db.ld, X, ldx);
            ++launches;
            flops += 4.0 * db.ld * db.ld * nrow;
            return;
        }
        const Cluster& ct = T_.clusters[D.t];
        const int n1 = nunk(ct.child[0]), n2 = nunk(ct.child[1]);
        solveUr(D.child[0], X, ldx, nrow);
        update(raw(X + (int64_t)n1 * ldx, ldx, nrow, n2, -1, ct.child[1]), raw(X, ldx, nrow, n1, -1, ct.child[0]),
               full(D.child[1]), neg());
        solveUr(D.child[3], X + (int64_t)n1 * ldx, ldx, nrow);
    }

    // block X (row cluster of d) := L_dd^{-1} X
    void trsmL(int d, const View& X) {
        const int k = kind(X);
        if (k == DENSE) {
            int ld;
            cplx<T>* p = dptr(X, ld);
            solveL(d, p, ld, X.n);
        } else if (k == LRK) {
            flush(X);
            LR& L = lrb(X);
            if (L.r > 0) solveL(d, L.U, L.m, L.r);
        } else {
            const Block& D = T_.blocks[d];
            for (int j = 0; j < 2; ++j) {
                const View X1 = sub(X, 0, j), X2 = sub(X, 1, j);
                trsmL(D.child[0], X1);
                update(X2, full(D.child[2]), X1, neg());
                trsmL(D.child[3], X2);
            }
        }
    }
    // block X (column cluster of d) := X U_dd^{-1}
    void trsmU(int d, const View& X) {
        const int k = kind(X);
        if (k == DENSE) {
            int ld;
            cplx<T>* p = dptr(X, ld);
            solveUr(d, p, ld, X.m);
        } else if (k == LRK) {
            flush(X);
            LR& L = lrb(X);
            if (L.r > 0) {
                // U (V^T U_dd^{-1}): solve on W = V^T, then V = W^T
                auto mk = scratch.mark();
                cplx<T>* W = scratch.alloc((size_t)L.r * L.n);
                transpose<T>(s, L.n, L.r, L.V, L.n, W, L.r);
                solveUr(d, W, L.r, L.r);
                transpose<T>(s, L.r, L.n, W, L.r, L.V, L.n);
                launches += 2;
                scratch.release(mk);
            }
        } else {
            const Block& D = T_.blocks[d];
            for (int i = 0; i < 2; ++i) {
                const View X1 = sub(X, i, 0), X2 = sub(X, i, 1);
                trsmU(D.child[0], X1);
                update(X2, X1, full(D.child[1]), neg());
                trsmU(D.child[3], X2);
            }
        }
    }

    void hlu(int d) {
        const Block& D = T_.blocks[d];
        if (D.type == BLK_DENSE) {
            const DenseBlockDev& db = c.dblk[D.leaf_index];
            getrf<T>(s, db.ld, dense.p + db.offset, db.ld, piv.p + piv_off[D.leaf_index], info.p + D.leaf_index);
            ++launches;
            flops += 8.0 / 3.0 * (double)db.ld * db.ld * db.ld;
            return;
        }
        CBIE_REQUIRE(D.type == BLK_HIER, -7, "low-rank diagonal block");
        hlu(D.child[0]);
        trsmL(D.child[0], full(D.child[1]));
        trsmU(D.child[0], full(D.child[2]));
        update(full(D.child[3]), full(D.child[2]), full(D.child[1]), neg());
        hlu(D.child[3]);
    }
};

struct HMat {
    int prec = 0;
    std::shared_ptr<HF<double>> f64;
    std::shared_ptr<HF<float>> f32;
};

Ctx::Ctx() {}
Ctx::~Ctx() {}

template <typename T> static std::shared_ptr<HF<T>> make_factor(Ctx& c) {
    auto f = std::make_shared<HF<T>>(c, c.aca_tol);
    hipStream_t s = c.stream;
    const Tree& T_ = c.tree;
    // copy of the operator in the working precision
    f->dense.alloc(std::max<int64_t>(c.stats.dense_entries, 1));
    convert<double, T>(s, c.stats.dense_entries, c.dense.p, f->dense.p);
    f->lr.resize(c.lblk.size());
    for (size_t b = 0; b < c.lblk.size(); ++b) {
        auto& L = f->lr[b];
        L.m = 2 * c.lblk[b].row_nodes;
        L.n = 2 * c.lblk[b].col_nodes;
        L.r = L.K = c.lr.rank[b];
        L.cap = std::max(L.r, 1);
        L.U = f->arena.alloc((size_t)L.m * L.cap);
        L.V = f->arena.alloc((size_t)L.n * L.cap);
        convert<double, T>(s, (int64_t)L.m * L.r, c.lr.mem.p + c.lr.u_off[b], L.U);
        convert<double, T>(s, (int64_t)L.n * L.r, c.lr.mem.p + c.lr.v_off[b], L.V);
    }
    // pivots of the diagonal leaves
    f->piv_off.assign(c.dblk.size(), -1);
    int64_t np = 0;
    for (size_t b = 0; b < T_.dense_blocks.size(); ++b) {
        const Block& B = T_.blocks[T_.dense_blocks[b]];
        if (B.t == B.s) {
            f->piv_off[b] = np;
            np += c.dblk[b].ld;
        }
    }
    f->piv.alloc(std::max<int64_t>(np, 1));
    f->info.alloc(std::max<size_t>(c.dblk.size(), 1));
    CBIE_HIP(hipMemsetAsync(f->info.p, 0, sizeof(int) * std::max<size_t>(c.dblk.size(), 1), s));
    int maxm = 1;
    for (auto& d : c.lblk) maxm = std::max(maxm, 2 * d.row_nodes);
    f->used.alloc(maxm);
    f->d_rank.alloc(1);
    return f;
}

template <typename T> static void run_factor(Ctx& c, HF<T>& f) {
    for (int root : c.tree.block_roots) f.hlu(root);
    for (size_t b = 0; b < f.lr.size(); ++b) f.flush_block((int)b);
    std::vector<int> info(c.dblk.size());
    if (!info.empty()) f.info.download(info.data(), info.size(), c.stream);
    c.sync();
    for (size_t b = 0; b < info.size(); ++b)
        CBIE_REQUIRE(info[b] == 0, CBIE_ESINGULAR, "zero pivot in diagonal leaf " + std::to_string(b));
    c.stats.factor_flops = (int64_t)f.flops;
    c.stats.n_kernel_launches = f.launches;
}

void stage_factor(Ctx& c, int prec) {
    const double t0 = now_s();
    auto hm = std::make_shared<HMat>();
    hm->prec = prec;
    if (prec == CBIE_PREC_C128) {
        hm->f64 = make_factor<double>(c);
        run_factor(c, *hm->f64);
    } else {
        hm->f32 = make_factor<float>(c);
        run_factor(c, *hm->f32);
    }
    c.hm = hm;
    c.stats.t_factor = now_s() - t0;
}

// X (tree order, N x nrhs, ld N) := LU^{-1} X in the working precision
template <typename T> static void lu_solve_tree(Ctx& c, HF<T>& f, cplx<T>* X, int nrhs) {
    const int ld = (int)c.n_unk;
    for (int root : c.tree.block_roots) {
        const Cluster& cl = c.tree.clusters[c.tree.blocks[root].t];
        cplx<T>* Xo = X + cl.unk0();
        f.solveL(root, Xo, ld, nrhs);
        f.solveU(root, Xo, ld, nrhs);
    }
}

// column norms |r_j|^2 and |b_j|^2
__global__ void k_colnorm2(int64_t n, int nrhs, const zd* __restrict__ a, double* __restrict__ out) {
    const int r = blockIdx.x;
    if (r >= nrhs) return;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += abs2(a[(int64_t)r * n + i]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = sh[0] + sh[1] + sh[2] + sh[3];
}
__global__ void k_axpy_sub(int64_t n, const zd* __restrict__ b, zd* __restrict__ r) {   // r = b - r
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) r[e] = b[e] - r[e];
}
__global__ void k_add(int64_t n, const zd* __restrict__ d, zd* __restrict__ x) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) x[e] = x[e] + d[e];
}

void stage_solve(Ctx& c, int nrhs, const zd* b, zd* x, long ld, double tol, int maxit, int* iters) {
    const double t0 = now_s();
    CBIE_REQUIRE(c.hm, CBIE_ESTATE, "no factorization");
    const int64_t N = c.n_unk, NN = N * nrhs;
    hipStream_t s = c.stream;
    DBuf<zd> bt, xt, rt;
    bt.alloc(NN);
    xt.alloc(NN);
    rt.alloc(NN);
    const unsigned g = ceil_div(NN, 256);
    k_to_tree<double><<<g, 256, 0, s>>>(c.d_tree_node.p, N, nrhs, b, ld, bt.p);
    check_launch("k_to_tree");
    DBuf<double> nrm;
    nrm.alloc(2 * (size_t)nrhs);
    std::vector<double> hn(2 * (size_t)nrhs);
    k_colnorm2<<<nrhs, 256, 0, s>>>(N, nrhs, bt.p, nrm.p + nrhs);
    check_launch("k_colnorm2");

    DBuf<zf> w;
    if (c.hm->prec != CBIE_PREC_C128) w.alloc(NN);
    auto correction = [&](const zd* rhs, zd* out) {   // out = LU^{-1} rhs
        if (c.hm->prec == CBIE_PREC_C128) {
            if (out != rhs) CBIE_HIP(hipMemcpyAsync(out, rhs, sizeof(zd) * NN, hipMemcpyDeviceToDevice, s));
            lu_solve_tree(c, *c.hm->f64, out, nrhs);
        } else {
            convert<double, float>(s, NN, rhs, w.p);
            lu_solve_tree(c, *c.hm->f32, w.p, nrhs);
            convert<float, double>(s, NN, w.p, out);
        }
    };
    correction(bt.p, xt.p);
    int it = 0;
    bool ok = (maxit == 0);
    for (; it < maxit; ++it) {
        apply_operator_tree(c, nrhs, xt.p, rt.p);
        k_axpy_sub<<<g, 256, 0, s>>>(NN, bt.p, rt.p);
        check_launch("k_axpy_sub");
        k_colnorm2<<<nrhs, 256, 0, s>>>(N, nrhs, rt.p, nrm.p);
        check_launch("k_colnorm2");
        nrm.download(hn.data(), hn.size(), s);
        c.sync();
        double worst = 0.0;
        for (int r = 0; r < nrhs; ++r) worst = std::max(worst, std::sqrt(hn[r] / std::max(hn[nrhs + r], 1e-300)));
        if (worst <= tol) { ok = true; break; }
        correction(rt.p, rt.p);
        k_add<<<g, 256, 0, s>>>(NN, rt.p, xt.p);
        check_launch("k_add");
    }
    k_from_tree<double><<<g, 256, 0, s>>>(c.d_tree_node.p, N, nrhs, xt.p, x, ld);
    check_launch("k_from_tree");
    c.sync();
    if (iters) *iters = it;
    c.stats.ir_iterations = it;
    c.stats.t_solve = now_s() - t0;
    CBIE_REQUIRE(ok, CBIE_ENOCONV, "iterative refinement did not reach the tolerance");
}

}  // namespace cbie

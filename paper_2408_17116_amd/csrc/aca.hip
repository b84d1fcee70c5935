// Batched adaptive cross approximation of the admissible blocks (Sec. III;
// ACA with partial pivoting, the paper's ref. [22]) and the low-rank store.
#include <algorithm>
#include <cmath>

#include "ctx.hpp"
#include "lowrank.hpp"
#include "mlp.hpp"
#include "linalg.hpp"

namespace cbie {

// ---------------------------------------------------------------- reductions
struct ArgMax {
    double v;
    int i;
};
__device__ inline ArgMax better(ArgMax a, ArgMax b) {
    // larger value wins; ties go to the lower index
    if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
    return a;
}
__device__ inline ArgMax wave_argmax(ArgMax a) {
    for (int off = 32; off > 0; off >>= 1) {
        ArgMax o;
        o.v = __shfl_xor(a.v, off);
        o.i = __shfl_xor(a.i, off);
        a = better(a, o);
    }
    return a;
}
__device__ inline double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}
// block of 256 threads (4 waves)
__device__ inline ArgMax block_argmax(ArgMax a, ArgMax* sh) {
    a = wave_argmax(a);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = a;
    __syncthreads();
    ArgMax r = sh[0];
    for (int k = 1; k < 4; ++k) r = better(r, sh[k]);
    return r;
}
__device__ inline double block_sum(double x, double* sh) {
    x = wave_sum(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = x;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// MFIE entries of one (target node, source node) pair, far rule.
__device__ inline void far_pair(const NodeArrays& nd, double k, int gi, int gj, zd K[2][2]) {
    const V3 R = v3(nd.rx[gi] - nd.rx[gj], nd.ry[gi] - nd.ry[gj], nd.rz[gi] - nd.rz[gj]);
    mfie_kernel(k, R, v3(nd.aux[gi], nd.auy[gi], nd.auz[gi]), v3(nd.avx[gi], nd.avy[gi], nd.avz[gi]),
                v3(nd.aux[gj], nd.auy[gj], nd.auz[gj]), v3(nd.avx[gj], nd.avy[gj], nd.avz[gj]), K);
    const double w = nd.w[gj];
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) K[b][a] = zd{w * K[b][a].re, w * K[b][a].im};
}

// N-Mueller far entries of one (target node, source node) pair: the twelve
// kernel values times the source weight, and the weighted divergence
// weights w phi[b] (eqs. 7-9, 19; rows H_u, H_v, E_u, E_v).
__device__ inline void nm_far_pair(const NmMat& M, const NodeArrays& nd, int gi, int gj, NmVals& K, double& w) {
    nm_kernel(M, v3(nd.rx[gi] - nd.rx[gj], nd.ry[gi] - nd.ry[gj], nd.rz[gi] - nd.rz[gj]),
              v3(nd.aux[gi], nd.auy[gi], nd.auz[gi]), v3(nd.avx[gi], nd.avy[gi], nd.avz[gi]),
              v3(nd.aux[gj], nd.auy[gj], nd.auz[gj]), v3(nd.avx[gj], nd.avy[gj], nd.avz[gj]), K);
    w = nd.w[gj];
}
__device__ inline int nm_dmat_offset(int q) { return (q - 1) * q * (2 * q - 1) / 6; }

// One work-group of 256 threads per admissible block M (m x n, m = 2 row
// nodes, n = 2 column nodes), M ~ sum_k u_k v_k^T:
//   row i_k -> residual row r (written into V[:, k]); pivot j_k = argmax |r|
//   (lowest index on ties), skipping rows whose residual vanishes;
//   v_k = r / r[j_k]; u_k = residual column j_k (written into U[:, k]);
//   |S_k|^2 += 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k) + |u_k|^2 |v_k|^2;
//   stop when |u_k| |v_k| <= tol |S_k|, else i_{k+1} = argmax |u_k| over
//   unused rows.  Entries are generated on the fly from the far rule (an
//   admissible block holds no near pair), or, for an N-Mueller block with
//   J.a_off >= 0, read from its explicit copy (column-major m x n in
//   `dense`).  N-Mueller entries on the fly: the surface divergence of the
//   source couples an entry of column (j = (k, l), a) to the divergence
//   weights of the nodes on the source patch's line through j, through the
//   differentiation matrix D (u: sum_m D[m][l] w phi(k, m); v: sum_m D[m][k]
//   w phi(m, l)).  A row takes one kernel evaluation per column node (the
//   weights of the row's component staged in the job's phi scratch); a
//   column takes q per row node.
__global__ __launch_bounds__(256) void k_aca(const AcaJob* __restrict__ jobs, int n_jobs,
                                             const int* __restrict__ tree_node, NodeArrays nd,
                                             const ObjDev* __restrict__ objs, double tol,
                                             zd* __restrict__ ws, unsigned char* __restrict__ used_ws,
                                             int* __restrict__ rank_out, int* __restrict__ flag_out,
                                             const zd* __restrict__ dense, const PatchDev* __restrict__ patches,
                                             const int* __restrict__ node_patch, const double* __restrict__ dmat) {
    const int jb = blockIdx.x;
    if (jb >= n_jobs) return;
    const AcaJob J = jobs[jb];
    const int m = J.upn * J.row_nodes, n = J.upn * J.col_nodes;
    const zd* A = (dense && J.a_off >= 0) ? dense + J.a_off : nullptr;
    const bool nm = J.upn == 4;
    const NmMat M = nm_mat(objs[J.obj]);
    zd* phi = ws + J.phi_off;   // N-Mueller row step: w phi of the row's component per column node
    zd* U = ws + J.u_off;   // m x cap
    zd* V = ws + J.v_off;   // n x cap
    unsigned char* used = used_ws + J.used_off;
    const double k0 = objs[J.obj].k0;
    __shared__ ArgMax sh_am[4];
    __shared__ double sh_s[4];
    __shared__ zd s_coef[1024];       // U[i, l] (row step) or V[j, l] (column step)
    __shared__ double s_cross[2];
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += 256) used[i] = 0;
    __syncthreads();

    int irow = 0;
    int rank = 0;
    double s2 = 0.0;
    int converged = 0;
    const int cap = J.cap;
    while (rank < cap) {
        // residual row irow into V[:, rank]
        for (int l = tid; l < rank; l += 256) s_coef[l] = U[(int64_t)l * m + irow];
        if (tid == 0) used[irow] = 1;
        __syncthreads();
        zd* vk = V + (int64_t)rank * n;
        ArgMax am{-1.0, 0x7fffffff};
        if (A) {
            for (int j = tid; j < n; j += 256) {
                zd r = A[(int64_t)j * m + irow];
                for (int l = 0; l < rank; ++l) r = r - s_coef[l] * V[(int64_t)l * n + j];
                vk[j] = r;
                am = better(am, ArgMax{abs2(r), j});
            }
        } else if (nm) {
            const int gi = tree_node[J.row_node0 + irow / 4];
            const int cr = irow & 3, b = cr & 1;
            const bool isE = cr >= 2;
            // pass 1: the entries without the divergence term, and w phi[b]
            for (int jn = tid; jn < J.col_nodes; jn += 256) {
                const int gj = tree_node[J.col_node0 + jn];
                NmVals K;
                double w;
                nm_far_pair(M, nd, gi, gj, K, w);
                phi[jn] = w * K.phi[b];
                for (int a = 0; a < 2; ++a) {
                    vk[4 * jn + a] = w * (isE ? K.X0[b][a] : K.CH[b][a]);
                    vk[4 * jn + 2 + a] = w * (isE ? K.CE[b][a] : K.X0[b][a]);
                }
            }
            __syncthreads();
            // pass 2: divergence terms on the X entries, residual, pivot
            for (int jn = tid; jn < J.col_nodes; jn += 256) {
                const int gj = tree_node[J.col_node0 + jn];
                const PatchDev P = patches[node_patch[gj]];
                const int q = P.q, loc = gj - P.node0, kk = loc / q, ll = loc % q, base = jn - loc;
                const double* Dq = dmat + nm_dmat_offset(q);
                zd su{0.0, 0.0}, sv{0.0, 0.0};
                for (int mm = 0; mm < q; ++mm) {
                    cfma(su, zd{Dq[mm * q + ll], 0.0}, phi[base + kk * q + mm]);
                    cfma(sv, zd{Dq[mm * q + kk], 0.0}, phi[base + mm * q + ll]);
                }
                const int xs = isE ? 0 : 2;   // slots of the X entries (a = 0, 1)
                vk[4 * jn + xs] = vk[4 * jn + xs] + su;
                vk[4 * jn + xs + 1] = vk[4 * jn + xs + 1] + sv;
                for (int a = 0; a < 4; ++a) {
                    const int j = 4 * jn + a;
                    zd r = vk[j];
                    for (int l = 0; l < rank; ++l) r = r - s_coef[l] * V[(int64_t)l * n + j];
                    vk[j] = r;
                    am = better(am, ArgMax{abs2(r), j});
                }
            }
        } else {
            const int gi = tree_node[J.row_node0 + irow / 2];
            const int b = irow & 1;
            for (int jn = tid; jn < J.col_nodes; jn += 256) {
                const int gj = tree_node[J.col_node0 + jn];
                zd K[2][2];
                far_pair(nd, k0, gi, gj, K);
                for (int a = 0; a < 2; ++a) {
                    const int j = 2 * jn + a;
                    zd r = K[b][a];
                    for (int l = 0; l < rank; ++l) r = r - s_coef[l] * V[(int64_t)l * n + j];
                    vk[j] = r;
                    am = better(am, ArgMax{abs2(r), j});
                }
            }
        }
        am = block_argmax(am, sh_am);
        if (am.v <= 0.0) {
            // zero residual row: try the next unused row, stop if none
            __syncthreads();
            ArgMax nx{-1.0, 0x7fffffff};
            for (int i = tid; i < m; i += 256)
                if (!used[i]) nx = better(nx, ArgMax{0.0, i});
            nx = block_argmax(nx, sh_am);
            if (nx.v < 0.0) { converged = 1; break; }
            irow = nx.i;
            continue;
        }
        const int jp = am.i;
        const zd piv = vk[jp];
        __syncthreads();
        // v_k = r / pivot
        for (int j = tid; j < n; j += 256) vk[j] = cdiv(vk[j], piv);
        for (int l = tid; l < rank; l += 256) s_coef[l] = V[(int64_t)l * n + jp];
        __syncthreads();
        // residual column jp into U[:, rank]
        zd* uk = U + (int64_t)rank * m;
        ArgMax nx{-1.0, 0x7fffffff};
        double nu2 = 0.0;
        if (A) {
            for (int i = tid; i < m; i += 256) {
                zd c = A[(int64_t)jp * m + i];
                for (int l = 0; l < rank; ++l) c = c - s_coef[l] * U[(int64_t)l * m + i];
                uk[i] = c;
                nu2 += abs2(c);
                if (!used[i]) nx = better(nx, ArgMax{abs2(c), i});
            }
        } else if (nm) {
            const int gj = tree_node[J.col_node0 + jp / 4];
            const int a = jp & 3, ap = a & 1;
            const bool isM = a >= 2;
            const PatchDev P = patches[node_patch[gj]];
            const int q = P.q, loc = gj - P.node0, kk = loc / q, ll = loc % q;
            const double* Dq = dmat + nm_dmat_offset(q);
            for (int in = tid; in < J.row_nodes; in += 256) {
                const int gi2 = tree_node[J.row_node0 + in];
                NmVals K;
                double w;
                nm_far_pair(M, nd, gi2, gj, K, w);
                // divergence terms of both row components b: the weights on
                // the source patch's line through j (direction ap)
                zd d0{0.0, 0.0}, d1{0.0, 0.0};
                for (int mm = 0; mm < q; ++mm) {
                    const int lm = ap == 0 ? kk * q + mm : mm * q + ll;
                    const double dc = Dq[mm * q + (ap == 0 ? ll : kk)];
                    zd p0, p1;
                    if (lm == loc) {
                        p0 = w * K.phi[0];
                        p1 = w * K.phi[1];
                    } else {
                        NmVals Km;
                        double wm;
                        nm_far_pair(M, nd, gi2, P.node0 + lm, Km, wm);
                        p0 = wm * Km.phi[0];
                        p1 = wm * Km.phi[1];
                    }
                    cfma(d0, zd{dc, 0.0}, p0);
                    cfma(d1, zd{dc, 0.0}, p1);
                }
                const int ac = isM ? a - 2 : a;
                for (int cr = 0; cr < 4; ++cr) {
                    const int b = cr & 1;
                    const bool isE = cr >= 2;
                    zd c;
                    if (!isM) c = isE ? w * K.X0[b][ac] + (b ? d1 : d0) : w * K.CH[b][ac];
                    else c = isE ? w * K.CE[b][ac] : w * K.X0[b][ac] + (b ? d1 : d0);
                    const int i = 4 * in + cr;
                    for (int l = 0; l < rank; ++l) c = c - s_coef[l] * U[(int64_t)l * m + i];
                    uk[i] = c;
                    nu2 += abs2(c);
                    if (!used[i]) nx = better(nx, ArgMax{abs2(c), i});
                }
            }
        } else {
            const int gj = tree_node[J.col_node0 + jp / 2];
            const int a = jp & 1;
            for (int in = tid; in < J.row_nodes; in += 256) {
                const int gi2 = tree_node[J.row_node0 + in];
                zd K[2][2];
                far_pair(nd, k0, gi2, gj, K);
                for (int bb = 0; bb < 2; ++bb) {
                    const int i = 2 * in + bb;
                    zd c = K[bb][a];
                    for (int l = 0; l < rank; ++l) c = c - s_coef[l] * U[(int64_t)l * m + i];
                    uk[i] = c;
                    nu2 += abs2(c);
                    if (!used[i]) nx = better(nx, ArgMax{abs2(c), i});
                }
            }
        }
        double nv2 = 0.0;
        for (int j = tid; j < n; j += 256) nv2 += abs2(vk[j]);
        nu2 = block_sum(nu2, sh_s);
        nv2 = block_sum(nv2, sh_s);
        nx = block_argmax(nx, sh_am);
        // cross terms 2 Re sum_l (u_l^H u_k)(v_l^H v_k): wave w handles l = w, w+4, ...
        double cross = 0.0;
        {
            const int w = tid >> 6, lane = tid & 63;
            for (int l = w; l < rank; l += 4) {
                double ur = 0, ui = 0, vr = 0, vi = 0;
                for (int i = lane; i < m; i += 64) {
                    const zd x = U[(int64_t)l * m + i], y = uk[i];
                    ur += x.re * y.re + x.im * y.im;
                    ui += x.re * y.im - x.im * y.re;
                }
                for (int j = lane; j < n; j += 64) {
                    const zd x = V[(int64_t)l * n + j], y = vk[j];
                    vr += x.re * y.re + x.im * y.im;
                    vi += x.re * y.im - x.im * y.re;
                }
                ur = wave_sum(ur); ui = wave_sum(ui); vr = wave_sum(vr); vi = wave_sum(vi);
                cross += ur * vr - ui * vi;
            }
            if (lane == 0) sh_s[w] = cross;
            __syncthreads();
            if (tid == 0) s_cross[0] = sh_s[0] + sh_s[1] + sh_s[2] + sh_s[3];
            __syncthreads();
            cross = s_cross[0];
        }
        s2 += 2.0 * cross + nu2 * nv2;
        ++rank;
        if (nu2 * nv2 <= tol * tol * fabs(s2)) { converged = 1; break; }
        if (nx.v < 0.0) { converged = 1; break; }   // every row used
        irow = nx.i;
        __syncthreads();
    }
    if (tid == 0) {
        rank_out[jb] = rank;
        flag_out[jb] = converged;
    }
}

// Copy the first `rank` columns of the ACA workspace into the compact store.
__global__ void k_lr_compact(const AcaJob* __restrict__ jobs, int n_jobs, const zd* __restrict__ ws,
                             const int* __restrict__ rank, const int64_t* __restrict__ u_dst,
                             const int64_t* __restrict__ v_dst, zd* __restrict__ store) {
    const int jb = blockIdx.y;
    if (jb >= n_jobs) return;
    const AcaJob J = jobs[jb];
    const int64_t m = J.upn * (int64_t)J.row_nodes, n = J.upn * (int64_t)J.col_nodes, r = rank[jb];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (m + n) * r;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < m * r) store[u_dst[jb] + e] = ws[J.u_off + e];
        else store[v_dst[jb] + (e - m * r)] = ws[J.v_off + (e - m * r)];
    }
}

// Entries U V^T of each low-rank block, written in the original order.
__global__ void k_export_lr(const DenseBlockDev* __restrict__ blocks, int n_blocks,
                            const int64_t* __restrict__ u_off, const int64_t* __restrict__ v_off,
                            const int* __restrict__ rank, const int* __restrict__ tree_node,
                            const zd* __restrict__ store, zd* __restrict__ A, int64_t lda) {
    const int bid = blockIdx.y;
    if (bid >= n_blocks) return;
    const DenseBlockDev B = blocks[bid];
    const int64_t m = B.upn * (int64_t)B.row_nodes, n = B.upn * (int64_t)B.col_nodes;
    const int r = rank[bid];
    const zd* U = store + u_off[bid];
    const zd* V = store + v_off[bid];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % m, j = e / m;
        zd s{0.0, 0.0};
        for (int l = 0; l < r; ++l) cfma(s, U[l * m + i], V[l * n + j]);
        const int64_t gr = B.upn * (int64_t)tree_node[B.row_node0 + i / B.upn] + (i % B.upn);
        const int64_t gc = B.upn * (int64_t)tree_node[B.col_node0 + j / B.upn] + (j % B.upn);
        A[gc * lda + gr] = s;
    }
}

// ACA of the given blocks with the given widths, in rounds whose workspace
// (U: m x width and V: n x width per block) stays within a budget
// (CBIE_ACA_BUDGET elements; default a quarter of the device memory free at
// the start, at most 2^32 elements); each round's factors are packed (U then
// V, rank columns each) into a buffer of their own before the workspace is
// reused.  N-Mueller blocks whose shorter side is below CBIE_NM_OTF_MIN
// unknowns (default 2048) are filled explicitly per round, within a budget
// of their own (CBIE_ACA_DENSE entries; default an eighth of the free
// memory, at most kAcaDense), and compressed from their copies; larger ones
// get their entries on the fly (a column costs q kernel evaluations per
// row: the surface divergence couples the source patch's line, so the
// explicit copy is cheaper for small blocks).  A round lasts as long as its
// slowest block (one work-group each), so fewer, larger rounds finish
// sooner.
struct AcaPass {
    std::vector<int> rank, flag;
    std::vector<int> round;        // per block: the buffer holding its factors
    std::vector<int64_t> off;      // per block: offset of its factors there
    std::vector<DBuf<zd>> fac;     // packed factors, one buffer per round
    double ws_elems = 0.0;         // workspace the widths ask for, all rounds
    int rounds = 0;
};
static void aca_pass(Ctx& c, double tol, const std::vector<int>& blocks, const std::vector<int>& width, AcaPass& P) {
    const int nb = (int)blocks.size();
    size_t mfree = 0, mtot = 0;
    if (hipMemGetInfo(&mfree, &mtot) != hipSuccess) mfree = size_t(64) << 30;
    const int64_t free_elems = (int64_t)(mfree / sizeof(zd));
    const char* eb = getenv("CBIE_ACA_BUDGET");
    const int64_t budget = eb ? std::max<int64_t>(1, atoll(eb))
                              : std::max<int64_t>(int64_t(1) << 26, std::min<int64_t>(int64_t(1) << 32, free_elems / 4));
    const char* ed = getenv("CBIE_ACA_DENSE");
    const int64_t dense_budget = ed ? std::max<int64_t>(1, atoll(ed))
                                    : std::max<int64_t>(int64_t(1) << 24, std::min<int64_t>(kAcaDense, free_elems / 8));
    const char* eo = getenv("CBIE_NM_OTF_MIN");
    const int64_t otf_min = eo ? std::max<int64_t>(0, atoll(eo)) : 2048;
    P.rank.assign(nb, 0);
    P.flag.assign(nb, 0);
    P.round.assign(nb, -1);
    P.off.assign(nb, 0);
    P.fac.clear();
    P.ws_elems = 0.0;
    DBuf<zd> ws, dense;
    DBuf<unsigned char> used;
    int q0 = 0;
    while (q0 < nb) {
        // the round: blocks [q0, q1)
        std::vector<AcaJob> jobs;
        std::vector<DenseBlockDev> blk;
        int64_t off = 0, uoff = 0, doff = 0;
        int q1 = q0;
        while (q1 < nb) {
            const DenseBlockDev& d = c.lblk[blocks[q1]];
            const int m = d.upn * d.row_nodes, n = d.upn * d.col_nodes;
            const bool explicit_nm = c.upn == 4 && std::min(m, n) < otf_min;
            const bool otf_nm = c.upn == 4 && !explicit_nm;
            const int64_t w = (int64_t)(m + n) * width[q1] + (otf_nm ? d.col_nodes : 0);
            const int64_t e = explicit_nm ? (int64_t)m * n : 0;
            if (q1 > q0 && (off + w > budget || doff + e > dense_budget)) break;
            AcaJob J{};
            J.row_node0 = d.row_node0;
            J.row_nodes = d.row_nodes;
            J.col_node0 = d.col_node0;
            J.col_nodes = d.col_nodes;
            J.obj = d.obj;
            J.upn = d.upn;
            J.cap = width[q1];
            J.u_off = off;
            off += (int64_t)m * J.cap;
            J.v_off = off;
            off += (int64_t)n * J.cap;
            J.phi_off = 0;
            if (otf_nm) {
                J.phi_off = off;
                off += d.col_nodes;
            }
            J.used_off = uoff;
            uoff += m;
            J.a_off = -1;
            if (explicit_nm) {
                DenseBlockDev x = d;
                x.offset = doff;
                x.ld = m;
                blk.push_back(x);
                J.a_off = doff;
                doff += e;
            }
            jobs.push_back(J);
            ++q1;
        }
        const int nq = q1 - q0;
        P.ws_elems += (double)off;
        if ((int64_t)ws.n < off) ws.alloc(off);
        if ((int64_t)used.n < uoff) used.alloc(uoff);
        DBuf<AcaJob> d_jobs;
        d_jobs.upload(jobs, c.stream);
        DBuf<int> d_rank, d_flag;
        d_rank.alloc(nq);
        d_flag.alloc(nq);
        const zd* src = nullptr;
        DBuf<DenseBlockDev> d_blk;
        if (!blk.empty()) {
            if ((int64_t)dense.n < doff) dense.alloc(doff);
            d_blk.upload(blk, c.stream);
            fill_blocks_nm(c, blk, d_blk.p, dense.p);
            src = dense.p;
        }
        k_aca<<<nq, 256, 0, c.stream>>>(d_jobs.p, nq, c.d_tree_node.p, c.nd, c.d_objs.p, tol, ws.p, used.p, d_rank.p,
                                        d_flag.p, src, c.d_patches.p, c.d_node_patch.p, c.d_dmat.p);
        check_launch("k_aca");
        d_rank.download(P.rank.data() + q0, nq, c.stream);
        d_flag.download(P.flag.data() + q0, nq, c.stream);
        c.sync();
        // pack the round's factors
        std::vector<int64_t> uo(nq), vo(nq);
        int64_t tot = 0;
        for (int q = 0; q < nq; ++q) {
            const DenseBlockDev& d = c.lblk[blocks[q0 + q]];
            const int64_t m = d.upn * (int64_t)d.row_nodes, n = d.upn * (int64_t)d.col_nodes, r = P.rank[q0 + q];
            P.round[q0 + q] = (int)P.fac.size();
            P.off[q0 + q] = tot;
            uo[q] = tot;
            vo[q] = tot + m * r;
            tot += (m + n) * r;
        }
        DBuf<zd> packed;
        packed.alloc(std::max<int64_t>(tot, 1));
        DBuf<int64_t> du, dv;
        du.upload(uo, c.stream);
        dv.upload(vo, c.stream);
        k_lr_compact<<<dim3(32, nq), 256, 0, c.stream>>>(d_jobs.p, nq, ws.p, d_rank.p, du.p, dv.p, packed.p);
        check_launch("k_lr_compact");
        c.sync();
        P.fac.push_back(std::move(packed));
        ++P.rounds;
        q0 = q1;
    }
}

void stage_compress(Ctx& c, double tol, int mode) {
    const double t0 = now_s();
    const int nb = (int)c.lblk.size();
    CBIE_REQUIRE(mode != CBIE_RANK_PREDICTED || c.rank_model.set, CBIE_EINVAL, "predicted ranks without a rank model");
    c.aca_tol = tol;
    c.lr_prefix.assign(nb + 1, 0);
    c.lr.u_off.assign(nb, 0);
    c.lr.v_off.assign(nb, 0);
    c.lr.rank.assign(nb, 0);
    c.lr.cap.assign(nb, 0);
    int64_t lr_entries = 0, max_rank = 0, sum_rank = 0;
    c.stats.aca_fallbacks = 0;
    c.stats.aca_workspace_bytes = 0.0;
    c.stats.aca_unconverged = 0;
    if (nb > 0) {
        std::vector<int> all(nb), full(nb), width(nb);
        for (int b = 0; b < nb; ++b) {
            all[b] = b;
            full[b] = std::min({c.upn * c.lblk[b].row_nodes, c.upn * c.lblk[b].col_nodes, kAcaMaxRank});
        }
        width = full;
        if (mode == CBIE_RANK_PREDICTED) {
            // widths from the network's predicted log-ranks
            std::vector<float> f;
            block_features(c, tol, f);
            const auto& M = c.rank_model;
            DBuf<float> dp, dm, ds, dx, dy;
            dp.upload(M.params, c.stream);
            dm.upload(M.mean, c.stream);
            ds.upload(M.sdev, c.stream);
            dx.upload(f, c.stream);
            dy.alloc(nb);
            mlp_forward(c.stream, dp.p, dm.p, ds.p, dx.p, nb, dy.p);
            std::vector<float> y(nb);
            dy.download(y.data(), nb, c.stream);
            c.sync();
            for (int b = 0; b < nb; ++b) {
                const double r = std::ceil(std::exp((double)std::min(y[b], 20.f)) * (1.0 + M.margin)) + 2.0;
                width[b] = (int)std::min<double>(full[b], std::max(8.0, r));
            }
        }
        AcaPass P;
        aca_pass(c, tol, all, width, P);
        double ws_elems = P.ws_elems;
        // blocks that filled a predicted width without converging: full width
        std::vector<int> redo, redo_w;
        for (int b = 0; b < nb; ++b)
            if (!P.flag[b] && P.rank[b] == width[b] && width[b] < full[b]) {
                redo.push_back(b);
                redo_w.push_back(full[b]);
            }
        AcaPass R;
        std::vector<int> src(nb, -1);   // block -> job in the redo pass
        if (!redo.empty()) {
            aca_pass(c, tol, redo, redo_w, R);
            ws_elems += R.ws_elems;
            for (size_t q = 0; q < redo.size(); ++q) src[redo[q]] = (int)q;
        }
        c.stats.aca_fallbacks = (int64_t)redo.size();
        c.stats.aca_workspace_bytes = ws_elems * sizeof(zd);
        int64_t so = 0;
        std::vector<ConvDesc<double, double>> place;   // packed factors -> final offsets
        place.reserve(nb);
        for (int b = 0; b < nb; ++b) {
            const int64_t m = c.upn * (int64_t)c.lblk[b].row_nodes, n = c.upn * (int64_t)c.lblk[b].col_nodes;
            const AcaPass& Q = src[b] >= 0 ? R : P;
            const int qb = src[b] >= 0 ? src[b] : b;
            const int r = Q.rank[qb];
            c.lr.rank[b] = r;
            c.lr.cap[b] = r;
            c.lr.u_off[b] = so;
            c.lr.v_off[b] = so + m * r;
            if (r > 0) place.push_back(ConvDesc<double, double>{Q.fac[Q.round[qb]].p + Q.off[qb], nullptr, (m + n) * r});
            so += (m + n) * r;
            lr_entries += (m + n) * r;
            max_rank = std::max<int64_t>(max_rank, r);
            sum_rank += r;
            // a block that stopped at its full width min(m, n) is reproduced
            // exactly (every column interpolated); one stopped by the rank cap
            // below that may miss the tolerance
            c.stats.aca_unconverged += (!Q.flag[qb] && r < std::min(m, n)) ? 1 : 0;
        }
        c.lr.mem.alloc(std::max<int64_t>(so, 1));
        for (int b = 0, i = 0; b < nb; ++b)
            if (c.lr.rank[b] > 0) place[i++].b = c.lr.mem.p + c.lr.u_off[b];
        convert_batched<double, double>(c.stream, place);
        c.lr.d_u_off.upload(c.lr.u_off, c.stream);
        c.lr.d_v_off.upload(c.lr.v_off, c.stream);
        c.lr.d_rank.upload(c.lr.rank, c.stream);
        for (int b = 0; b < nb; ++b) c.lr_prefix[b + 1] = c.lr_prefix[b] + c.lr.rank[b];
        c.d_lr_prefix.upload(c.lr_prefix, c.stream);
        c.sync();
    }
    cbie_stats& st = c.stats;
    st.lr_entries = lr_entries;
    st.max_rank = max_rank;
    st.sum_rank = sum_rank;
    const double N = (double)c.n_unk;
    double full = 0.0;
    for (size_t o = 0; o < c.objs.size(); ++o) full += (double)c.upn * c.upn * c.obj_nodes[o] * c.obj_nodes[o];
    st.compression_rate = 1.0 - (double)(st.dense_entries + lr_entries) / full;
    (void)N;
    st.t_compress = now_s() - t0;
}

void export_lowrank(Ctx& c, zd* A, long ld) {
    const int nb = (int)c.lblk.size();
    if (nb == 0) return;
    dim3 grid(64, nb);
    k_export_lr<<<grid, 256, 0, c.stream>>>(c.d_lblk.p, nb, c.lr.d_u_off.p, c.lr.d_v_off.p, c.lr.d_rank.p,
                                            c.d_tree_node.p, c.lr.mem.p, A, ld);
    check_launch("k_export_lr");
}

}  // namespace cbie

// Operator application in FP64 (matvec, iterative-refinement residual),
// plane-wave right-hand sides (eq. 22) and the far field of a solution.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "ops.hpp"

namespace cbie {

// x (original order, ld) -> xt (tree order, ld_t = n_unk), nrhs columns
template <typename T>
__global__ void k_to_tree(const int* __restrict__ tree_node, int upn, int64_t n_unk, int nrhs,
                          const zd* __restrict__ x, int64_t ld, cplx<T>* __restrict__ xt) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n_unk * nrhs) return;
    const int64_t r = e / n_unk, u = e % n_unk;
    const zd v = x[r * ld + upn * (int64_t)tree_node[u / upn] + (u % upn)];
    xt[e] = cplx<T>{(T)v.re, (T)v.im};
}

template <typename T>
__global__ void k_from_tree(const int* __restrict__ tree_node, int upn, int64_t n_unk, int nrhs,
                            const cplx<T>* __restrict__ yt, zd* __restrict__ y, int64_t ld) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n_unk * nrhs) return;
    const int64_t r = e / n_unk, u = e % n_unk;
    const cplx<T> v = yt[e];
    y[r * ld + upn * (int64_t)tree_node[u / upn] + (u % upn)] = zd{(double)v.re, (double)v.im};
}

template __global__ void k_to_tree<double>(const int*, int, int64_t, int, const zd*, int64_t, zd*);
template __global__ void k_to_tree<float>(const int*, int, int64_t, int, const zd*, int64_t, zf*);
template __global__ void k_from_tree<double>(const int*, int, int64_t, int, const zd*, zd*, int64_t);
template __global__ void k_from_tree<float>(const int*, int, int64_t, int, const zf*, zd*, int64_t);

__device__ inline void atomic_add_z(zd* p, zd v) {
    atomicAdd(&p->re, v.re);
    atomicAdd(&p->im, v.im);
}

// y[rows] += D x[cols] for every dense block; work-group = (block, 64-row
// slice), rhs processed 8 at a time with x staged in LDS; FP64 accumulation.
__global__ __launch_bounds__(256) void k_dense_mv(const DenseBlockDev* __restrict__ blocks, int nb,
                                                  const zd* __restrict__ store, const zd* __restrict__ xt,
                                                  zd* __restrict__ yt, int64_t n_unk, int nrhs) {
    const int bid = blockIdx.y;
    if (bid >= nb) return;
    const DenseBlockDev B = blocks[bid];
    const int m = B.upn * B.row_nodes, n = B.upn * B.col_nodes;
    const int r0 = blockIdx.x * 64;
    if (r0 >= m) return;
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;   // 4 groups split the columns
    const int row = r0 + lane;
    __shared__ zd sx[8][256];
    __shared__ zd red[4][64][8];
    const zd* D = store + B.offset;
    const int64_t c0 = B.upn * (int64_t)B.col_node0, rr0 = B.upn * (int64_t)B.row_node0;
    for (int rb = 0; rb < nrhs; rb += 8) {
        const int nr = min(8, nrhs - rb);
        zd acc[8];
        for (int t = 0; t < 8; ++t) acc[t] = zd{0.0, 0.0};
        for (int cb = 0; cb < n; cb += 256) {
            const int nc = min(256, n - cb);
            __syncthreads();
            for (int t = threadIdx.x; t < nr * 256; t += 256) {
                const int rr = t / 256, cc = t % 256;
                sx[rr][cc] = cc < nc ? xt[(int64_t)(rb + rr) * n_unk + c0 + cb + cc] : zd{0.0, 0.0};
            }
            __syncthreads();
            if (row < m) {
                for (int cc = grp; cc < nc; cc += 4) {
                    const zd a = D[(int64_t)(cb + cc) * B.ld + row];
                    for (int t = 0; t < nr; ++t) cfma(acc[t], a, sx[t][cc]);
                }
            }
        }
        __syncthreads();
        for (int t = 0; t < 8; ++t) red[grp][lane][t] = acc[t];
        __syncthreads();
        if (grp == 0 && row < m) {
            for (int t = 0; t < nr; ++t) {
                zd s = red[0][lane][t] + red[1][lane][t] + red[2][lane][t] + red[3][lane][t];
                atomic_add_z(&yt[(int64_t)(rb + t) * n_unk + rr0 + row], s);
            }
        }
    }
}

// tmp[l, r] = sum_j V[j, l] x[c0 + j, r] for each low-rank block (one
// work-group per (block, l)); block b's tmp starts at prefix[b] * nrhs.
__global__ __launch_bounds__(256) void k_lr_vt(const DenseBlockDev* __restrict__ blocks, int nb,
                                               const int64_t* __restrict__ v_off, const int* __restrict__ rank,
                                               const int64_t* __restrict__ prefix, const zd* __restrict__ store,
                                               const zd* __restrict__ xt, zd* __restrict__ tmp, int64_t n_unk,
                                               int nrhs) {
    const int bid = blockIdx.y;
    if (bid >= nb) return;
    const int l = blockIdx.x;
    const int r = rank[bid];
    if (l >= r) return;
    const DenseBlockDev B = blocks[bid];
    const int n = B.upn * B.col_nodes;
    const zd* V = store + v_off[bid] + (int64_t)l * n;
    const int64_t c0 = B.upn * (int64_t)B.col_node0;
    __shared__ double sh[2][4];
    for (int rr = 0; rr < nrhs; ++rr) {
        double sr = 0.0, si = 0.0;
        for (int j = threadIdx.x; j < n; j += 256) {
            const zd a = V[j], b = xt[(int64_t)rr * n_unk + c0 + j];
            sr += a.re * b.re - a.im * b.im;
            si += a.re * b.im + a.im * b.re;
        }
        for (int off = 32; off > 0; off >>= 1) { sr += __shfl_xor(sr, off); si += __shfl_xor(si, off); }
        __syncthreads();
        if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = sr; sh[1][threadIdx.x >> 6] = si; }
        __syncthreads();
        if (threadIdx.x == 0)
            tmp[prefix[bid] * nrhs + (int64_t)rr * r + l] =
                zd{sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3], sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]};
    }
}

// y[r0 + i, r] += sum_l U[i, l] tmp[l, r]
__global__ __launch_bounds__(256) void k_lr_u(const DenseBlockDev* __restrict__ blocks, int nb,
                                              const int64_t* __restrict__ u_off, const int* __restrict__ rank,
                                              const int64_t* __restrict__ prefix, const zd* __restrict__ store,
                                              const zd* __restrict__ tmp, zd* __restrict__ yt, int64_t n_unk,
                                              int nrhs) {
    const int bid = blockIdx.y;
    if (bid >= nb) return;
    const DenseBlockDev B = blocks[bid];
    const int m = B.upn * B.row_nodes;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int r = rank[bid];
    const zd* U = store + u_off[bid];
    const zd* T = tmp + prefix[bid] * nrhs;
    const int64_t r0 = B.upn * (int64_t)B.row_node0;
    for (int rr = 0; rr < nrhs; ++rr) {
        zd s{0.0, 0.0};
        for (int l = 0; l < r; ++l) cfma(s, U[(int64_t)l * m + i], T[(int64_t)rr * r + l]);
        atomic_add_z(&yt[(int64_t)rr * n_unk + r0 + i], s);
    }
}

__global__ void k_zero_z(int64_t n, zd* __restrict__ y) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) y[e] = zd{0.0, 0.0};
}

// y_t = A x_t in tree order (FP64), y_t overwritten; tmp holds
// lr_prefix[nl] * nrhs elements (V^T x of every low-rank block).  Launches
// only: no allocation, no memset (a fill kernel clears y_t).
static void apply_operator_tree_into(Ctx& c, int nrhs, const zd* xt, zd* yt, zd* tmp) {
    const int64_t N = c.n_unk;
    k_zero_z<<<ceil_div(N * nrhs, 256), 256, 0, c.stream>>>(N * nrhs, yt);
    check_launch("k_zero_z");
    const int nd = (int)c.dblk.size();
    if (nd > 0) {
        int maxm = 0;
        for (const auto& d : c.dblk) maxm = std::max(maxm, c.upn * d.row_nodes);
        k_dense_mv<<<dim3(ceil_div(maxm, 64), nd), 256, 0, c.stream>>>(c.d_dblk.p, nd, c.dense.p, xt, yt, N, nrhs);
        check_launch("k_dense_mv");
    }
    const int nl = (int)c.lblk.size();
    if (nl > 0) {
        int maxr = 1, maxm = 0;
        for (int b = 0; b < nl; ++b) {
            maxr = std::max(maxr, c.lr.rank[b]);
            maxm = std::max(maxm, c.upn * c.lblk[b].row_nodes);
        }
        k_lr_vt<<<dim3(maxr, nl), 256, 0, c.stream>>>(
            c.d_lblk.p, nl, c.lr.d_v_off.p, c.lr.d_rank.p, c.d_lr_prefix.p, c.lr.mem.p, xt, tmp, N, nrhs);
        check_launch("k_lr_vt");
        k_lr_u<<<dim3(ceil_div(maxm, 256), nl), 256, 0, c.stream>>>(
            c.d_lblk.p, nl, c.lr.d_u_off.p, c.lr.d_rank.p, c.d_lr_prefix.p, c.lr.mem.p, tmp, yt, N, nrhs);
        check_launch("k_lr_u");
    }
}

void apply_operator_tree(Ctx& c, int nrhs, const zd* xt, zd* yt) {
    const int64_t need = std::max<int64_t>(c.lr_prefix.empty() ? 0 : c.lr_prefix.back() * nrhs, 1);
    if ((int64_t)c.mv_tmp.n < need) c.mv_tmp.alloc(need);
    apply_operator_tree_into(c, nrhs, xt, yt, c.mv_tmp.p);
}

void stage_matvec(Ctx& c, int nrhs, const zd* x, zd* y, long ld) {
    const int64_t N = c.n_unk;
    DBuf<zd> xt, yt;
    xt.alloc(N * nrhs);
    yt.alloc(N * nrhs);
    const unsigned g = ceil_div(N * nrhs, 256);
    k_to_tree<double><<<g, 256, 0, c.stream>>>(c.d_tree_node.p, c.upn, N, nrhs, x, ld, xt.p);
    check_launch("k_to_tree");
    apply_operator_tree(c, nrhs, xt.p, yt.p);
    k_from_tree<double><<<g, 256, 0, c.stream>>>(c.d_tree_node.p, c.upn, N, nrhs, yt.p, y, ld);
    check_launch("k_from_tree");
    c.sync();
}

// ------------------------------------------------ allocation-free matvec
// One scratch array per GPU for callers that cannot allocate.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): its device address is resolved once per device by
// resolve_scratch() and kept in g_scratch.
static __device__ __align__(256) zd scratch[kScratchElems];

static std::mutex g_scratch_mu;
static std::vector<zd*> g_scratch;   // device -> address of that device's scratch

void resolve_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= device) g_scratch.resize(device + 1, nullptr);
    if (g_scratch[device]) return;
    void* p = nullptr;
    CBIE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CBIE_REQUIRE(p != nullptr, CBIE_EHIP, "scratch symbol has no device address");
    g_scratch[device] = (zd*)p;
}

int64_t matvec_scratch_elems(const Ctx& c, int nrhs) {
    return (2 * c.n_unk + (c.lr_prefix.empty() ? 0 : c.lr_prefix.back())) * (int64_t)nrhs;
}

void stage_matvec_noalloc(Ctx& c, int nrhs, const zd* x, zd* y, long ld) {
    const int64_t N = c.n_unk;
    const int64_t need = matvec_scratch_elems(c, nrhs);
    CBIE_REQUIRE(need <= kScratchElems, CBIE_EINVAL,
                 "matvec_noalloc: needs " + std::to_string(need) + " complex128 scratch elements, the limit is " +
                     std::to_string(kScratchElems) + " (fewer right-hand sides per call, or cbie_matvec)");
    zd* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (c.device < (int)g_scratch.size()) base = g_scratch[c.device];
    }
    CBIE_REQUIRE(base != nullptr, CBIE_EHIP, "scratch address not resolved for this device");
    zd* xt = base;
    zd* yt = base + N * nrhs;
    zd* tmp = yt + N * nrhs;
    const unsigned g = ceil_div(N * nrhs, 256);
    k_to_tree<double><<<g, 256, 0, c.stream>>>(c.d_tree_node.p, c.upn, N, nrhs, x, ld, xt);
    check_launch("k_to_tree");
    apply_operator_tree_into(c, nrhs, xt, yt, tmp);
    k_from_tree<double><<<g, 256, 0, c.stream>>>(c.d_tree_node.p, c.upn, N, nrhs, yt, y, ld);
    check_launch("k_from_tree");
    c.sync();
}

// ------------------------------------------------------ RHS (eqs. 19, 22)
// MFIE: b_u = -a_v . H_inc, b_v = a_u . H_inc.  N-Mueller (rows H_u, H_v,
// E_u, E_v of a node): -a_v . H_inc, a_u . H_inc, -a_v . E_inc, a_u . E_inc.
// E_inc = pol e^{-j k khat.r}, H_inc = khat x E_inc (exterior vacuum).
__global__ void k_rhs(NodeArrays nd, const int* __restrict__ node_patch, const PatchDev* __restrict__ patches,
                      const ObjDev* __restrict__ objs, int n_nodes, int upn, int nw, const double* __restrict__ kp,
                      zd* __restrict__ b, int64_t ld) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n_nodes * nw) return;
    const int w = (int)(e / n_nodes), i = (int)(e % n_nodes);
    const double k = objs[patches[node_patch[i]].obj].k0;
    const V3 kh = v3(kp[6 * w], kp[6 * w + 1], kp[6 * w + 2]);
    const V3 po = v3(kp[6 * w + 3], kp[6 * w + 4], kp[6 * w + 5]);
    const V3 r = v3(nd.rx[i], nd.ry[i], nd.rz[i]);
    double s, cs;
    sincos(k * dot(kh, r), &s, &cs);        // e^{-j phi} = cos - j sin
    const V3 h = cross(kh, po);
    const V3 au = v3(nd.aux[i], nd.auy[i], nd.auz[i]);
    const V3 av = v3(nd.avx[i], nd.avy[i], nd.avz[i]);
    const double cu = -dot(av, h), cv = dot(au, h);
    zd* bi = b + (int64_t)w * ld + (int64_t)upn * i;
    bi[0] = zd{cu * cs, -cu * s};
    bi[1] = zd{cv * cs, -cv * s};
    if (upn == 4) {
        const double eu = -dot(av, po), ev = dot(au, po);
        bi[2] = zd{eu * cs, -eu * s};
        bi[3] = zd{ev * cs, -ev * s};
    }
}

void stage_rhs(Ctx& c, int nw, const double* khat, const double* pol, zd* b, long ld) {
    std::vector<double> kp(6 * (size_t)nw);
    for (int w = 0; w < nw; ++w)
        for (int d = 0; d < 3; ++d) { kp[6 * w + d] = khat[3 * w + d]; kp[6 * w + 3 + d] = pol[3 * w + d]; }
    DBuf<double> d_kp;
    d_kp.upload(kp, c.stream);
    k_rhs<<<ceil_div((int64_t)c.n_nodes * nw, 256), 256, 0, c.stream>>>(
        c.nd, c.d_node_patch.p, c.d_patches.p, c.d_objs.p, c.n_nodes, c.upn, nw, d_kp.p, b, ld);
    check_launch("k_rhs");
    c.sync();
}

// Right-hand sides for point electric dipoles in free space (the feed of
// the spiral antenna, Sec. IV-A): the dipole's E and H replace the plane
// wave's in the rows of eq. 22 (and eq. 19).  Moment m (I l) at r0; with
// d = r - r0, R = |d|, e = d / R and G = e^{-jkR} / (4 pi R):
//   H = (1 + j k R) (G / R) (m x e),
//   E = G [(-1/R + j (1/(k R^2) - k)) (m - (m.e) e) + (2/R - 2j/(k R^2)) (m.e) e].
// One thread per (node, dipole); dp holds (r0, m) per dipole.
__global__ void k_rhs_dipole(NodeArrays nd, const int* __restrict__ node_patch, const PatchDev* __restrict__ patches,
                             const ObjDev* __restrict__ objs, int n_nodes, int upn, int ndp,
                             const double* __restrict__ dp, zd* __restrict__ b, int64_t ld) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_nodes * ndp) return;
    const int w = (int)(t / n_nodes), i = (int)(t % n_nodes);
    const double k = objs[patches[node_patch[i]].obj].k0;
    const V3 r0 = v3(dp[6 * w], dp[6 * w + 1], dp[6 * w + 2]);
    const V3 m = v3(dp[6 * w + 3], dp[6 * w + 4], dp[6 * w + 5]);
    const V3 d = v3(nd.rx[i], nd.ry[i], nd.rz[i]) - r0;
    const double R = sqrt(dot(d, d)), iR = 1.0 / R;
    const V3 e = iR * d;
    double s, cs;
    sincos(k * R, &s, &cs);
    const double gr = cs * iR / (4.0 * M_PI), gi = -s * iR / (4.0 * M_PI);   // G
    const double hr = (gr - k * R * gi) * iR, hi = (gi + k * R * gr) * iR;    // (1 + jkR) G / R
    const double a = 1.0 / (k * R * R) - k;
    const double tr = -gr * iR - gi * a, ti = -gi * iR + gr * a;              // G (-1/R + j a)
    const double c2 = 2.0 / (k * R * R);
    const double rr = 2.0 * gr * iR + gi * c2, ri = 2.0 * gi * iR - gr * c2;  // G (2/R - j c2)
    const V3 au = v3(nd.aux[i], nd.auy[i], nd.auz[i]);
    const V3 av = v3(nd.avx[i], nd.avy[i], nd.avz[i]);
    const V3 mh = cross(m, e);
    const double me = dot(m, e);
    const V3 mt = m - me * e;
    zd* bi = b + (int64_t)w * ld + (int64_t)upn * i;
    const double hu = -dot(av, mh), hv = dot(au, mh);
    bi[0] = zd{hr * hu, hi * hu};
    bi[1] = zd{hr * hv, hi * hv};
    if (upn == 4) {
        const double tu = -dot(av, mt), tv = dot(au, mt);
        const double ru = -me * dot(av, e), rv = me * dot(au, e);
        bi[2] = zd{tr * tu + rr * ru, ti * tu + ri * ru};
        bi[3] = zd{tr * tv + rr * rv, ti * tv + ri * rv};
    }
}

void stage_rhs_dipole(Ctx& c, int ndp, const double* pos, const double* mom, zd* b, long ld) {
    const int n = c.n_nodes;
    std::vector<double> dp(6 * (size_t)ndp);
    for (int w = 0; w < ndp; ++w) {
        for (int d = 0; d < 3; ++d) { dp[6 * w + d] = pos[3 * w + d]; dp[6 * w + 3 + d] = mom[3 * w + d]; }
        for (int i = 0; i < n; ++i) {
            const double x = c.h_r[i] - pos[3 * w], y = c.h_r[(size_t)n + i] - pos[3 * w + 1],
                         z = c.h_r[2 * (size_t)n + i] - pos[3 * w + 2];
            CBIE_REQUIRE(x * x + y * y + z * z > 0.0, CBIE_EINVAL,
                         "dipole " + std::to_string(w) + " sits on node " + std::to_string(i));
        }
    }
    DBuf<double> d_dp;
    d_dp.upload(dp, c.stream);
    k_rhs_dipole<<<ceil_div((int64_t)n * ndp, 256), 256, 0, c.stream>>>(c.nd, c.d_node_patch.p, c.d_patches.p,
                                                                      c.d_objs.p, n, c.upn, ndp, d_dp.p, b, ld);
    check_launch("k_rhs_dipole");
    c.sync();
}

// ---------------------------------------------------------------- far field
// N(rhat) = sum_nodes w (F_J^u a_u + F_J^v a_v) e^{j k rhat.r}, L likewise
// from M (N-Mueller only);  E = -j k (N_perp - rhat x L) / (4 pi).
// One work-group per (direction, rhs).
__global__ __launch_bounds__(256) void k_farfield(NodeArrays nd, const int* __restrict__ node_patch,
                                                  const PatchDev* __restrict__ patches,
                                                  const ObjDev* __restrict__ objs, int n_nodes, int upn,
                                                  const zd* __restrict__ x, int64_t ld, int ndir,
                                                  const double* __restrict__ rhat, zd* __restrict__ E) {
    const int d = blockIdx.x, r = blockIdx.y;
    if (d >= ndir) return;
    const V3 rh = v3(rhat[3 * d], rhat[3 * d + 1], rhat[3 * d + 2]);
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // N (re, im per axis), then L
    double kk = 0.0;
    for (int i = threadIdx.x; i < n_nodes; i += 256) {
        const double k = objs[patches[node_patch[i]].obj].k0;
        kk = k;
        const zd* xi = x + (int64_t)r * ld + (int64_t)upn * i;
        double s, cs;
        sincos(k * dot(rh, v3(nd.rx[i], nd.ry[i], nd.rz[i])), &s, &cs);   // e^{+j phi}
        const double w = nd.w[i];
        const double au[3] = {nd.aux[i], nd.auy[i], nd.auz[i]};
        const double av[3] = {nd.avx[i], nd.avy[i], nd.avz[i]};
        for (int src = 0; src < upn / 2; ++src) {
            const zd fu = xi[2 * src], fv = xi[2 * src + 1];
            for (int c = 0; c < 3; ++c) {
                const double jr = w * (fu.re * au[c] + fv.re * av[c]);
                const double ji = w * (fu.im * au[c] + fv.im * av[c]);
                acc[6 * src + 2 * c] += jr * cs - ji * s;
                acc[6 * src + 2 * c + 1] += jr * s + ji * cs;
            }
        }
    }
    __shared__ double sh[12][4];
    __shared__ double shk[4];
    for (int c = 0; c < 12; ++c) {
        double v = acc[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0) sh[c][threadIdx.x >> 6] = v;
    }
    double km = kk;
    for (int off = 32; off > 0; off >>= 1) km = fmax(km, __shfl_xor(km, off));
    if ((threadIdx.x & 63) == 0) shk[threadIdx.x >> 6] = km;
    __syncthreads();
    if (threadIdx.x == 0) {
        double N[12];
        for (int c = 0; c < 12; ++c) N[c] = sh[c][0] + sh[c][1] + sh[c][2] + sh[c][3];
        const double* L = N + 6;
        const double k = fmax(fmax(shk[0], shk[1]), fmax(shk[2], shk[3]));
        const double rv[3] = {rh.x, rh.y, rh.z};
        const double dre = rv[0] * N[0] + rv[1] * N[2] + rv[2] * N[4];
        const double dim = rv[0] * N[1] + rv[1] * N[3] + rv[2] * N[5];
        for (int c = 0; c < 3; ++c) {
            // N_perp - rhat x L (L = 0 for a conductor)
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const double xr = rv[c1] * L[2 * c2] - rv[c2] * L[2 * c1];
            const double xim = rv[c1] * L[2 * c2 + 1] - rv[c2] * L[2 * c1 + 1];
            const double pr = N[2 * c] - rv[c] * dre - xr, pi = N[2 * c + 1] - rv[c] * dim - xim;
            // -j k / (4 pi) (pr + j pi) = (k pi - j k pr) / (4 pi)
            E[((int64_t)r * ndir + d) * 3 + c] = zd{k * pi / (4 * M_PI), -k * pr / (4 * M_PI)};
        }
    }
}

void stage_farfield(Ctx& c, int nrhs, const zd* x, long ld, int ndir, const double* rhat, zd* E) {
    DBuf<double> d_r;
    d_r.upload(rhat, 3 * (size_t)ndir, c.stream);
    DBuf<zd> d_E;
    d_E.alloc(3 * (size_t)ndir * nrhs);
    k_farfield<<<dim3(ndir, nrhs), 256, 0, c.stream>>>(c.nd, c.d_node_patch.p, c.d_patches.p, c.d_objs.p,
                                                       c.n_nodes, c.upn, x, ld, ndir, d_r.p, d_E.p);
    check_launch("k_farfield");
    d_E.download(E, 3 * (size_t)ndir * nrhs, c.stream);
    c.sync();
}

}  // namespace cbie

// Geometry, near classification, self/near change-of-variables quadrature and
// dense-block fill of the CBIE MFIE matrix (Sec. II-B, eqs. 11-20).
#include "fill.hpp"

namespace cbie {

// ------------------------------------------------------------ node geometry
// One thread per node (original order): r, a_u, a_v at the Fejer point
// (u_l, v_k) of its patch, tensor weight w_l w_k.
__global__ void k_nodes(const PatchDev* __restrict__ patches, const ObjDev* __restrict__ objs,
                        const double* __restrict__ fej_x, const double* __restrict__ fej_w,
                        const int* __restrict__ node_patch, int n_nodes, NodeArrays nd) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const PatchDev P = patches[node_patch[i]];
    const ObjDev O = objs[P.obj];
    const int loc = i - P.node0;
    const int kk = loc / P.q, ll = loc % P.q;
    const double* x = fej_x + P.q * (P.q - 1) / 2;    // rule of size q stored at offset q(q-1)/2
    const double* w = fej_w + P.q * (P.q - 1) / 2;
    const double u = x[ll], v = x[kk];
    V3 r, au, av;
    patch_eval(P, O, u, v, r, au, av);
    nd.rx[i] = r.x; nd.ry[i] = r.y; nd.rz[i] = r.z;
    nd.aux[i] = au.x; nd.auy[i] = au.y; nd.auz[i] = au.z;
    nd.avx[i] = av.x; nd.avy[i] = av.y; nd.avz[i] = av.z;
    nd.w[i] = w[ll] * w[kk];
    nd.u[i] = u; nd.v[i] = v;
}

// Per patch: centre point r(0,0), corner-diagonal diameter, and a radius
// bounding the patch around the centre (1.25 x the farthest corner or edge
// midpoint), used only to skip patches that cannot be near.
__global__ void k_patch_info(const PatchDev* __restrict__ patches, const ObjDev* __restrict__ objs,
                             int n_patches, double* __restrict__ info) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_patches) return;
    const PatchDev P = patches[p];
    const ObjDev O = objs[P.obj];
    V3 c, au, av, r[8];
    patch_eval(P, O, 0.0, 0.0, c, au, av);
    const double us[8] = {-1, 1, 1, -1, 0, 1, 0, -1};
    const double vs[8] = {-1, -1, 1, 1, -1, 0, 1, 0};
    double rad = 0.0;
    for (int t = 0; t < 8; ++t) {
        patch_eval(P, O, us[t], vs[t], r[t], au, av);
        rad = fmax(rad, norm(r[t] - c));
    }
    const double diam = fmax(norm(r[0] - r[2]), norm(r[1] - r[3]));
    info[5 * p + 0] = c.x;
    info[5 * p + 1] = c.y;
    info[5 * p + 2] = c.z;
    info[5 * p + 3] = diam;
    info[5 * p + 4] = 1.25 * rad;
}

// Closest point of the patch to `t`: Gauss-Newton on |r(u,v) - t|^2 from
// the patch centre, each iterate clamped to the square.
__device__ inline double project(const PatchDev& P, const ObjDev& O, V3 t, double& uo, double& vo) {
    double u = 0.0, v = 0.0;
    V3 r, au, av;
    for (int it = 0; it < 80; ++it) {
        patch_eval(P, O, u, v, r, au, av);
        const V3 d = r - t;
        const double g0 = dot(d, au), g1 = dot(d, av);
        const double h00 = dot(au, au), h01 = dot(au, av), h11 = dot(av, av);
        const double det = h00 * h11 - h01 * h01;
        const double du = (h11 * g0 - h01 * g1) / det;
        const double dv = (h00 * g1 - h01 * g0) / det;
        const double un = fmin(1.0, fmax(-1.0, u - du));
        const double vn = fmin(1.0, fmax(-1.0, v - dv));
        const bool done = fabs(un - u) + fabs(vn - v) < 1e-15;
        u = un; v = vn;
        if (done) break;
    }
    patch_eval(P, O, u, v, r, au, av);
    uo = u; vo = v;
    return norm(r - t);
}

// Near test of one (node, patch) pair; fills (u*, v*, dist) when near.
__device__ inline bool near_test(const PatchDev* patches, const ObjDev* objs, const double* info,
                                 const NodeArrays& nd, int i, int p, int own, double delta,
                                 double& us, double& vs, double& dist) {
    if (p == own) {
        us = nd.u[i]; vs = nd.v[i]; dist = 0.0;
        return true;
    }
    const V3 t = v3(nd.rx[i], nd.ry[i], nd.rz[i]);
    const V3 c = v3(info[5 * p], info[5 * p + 1], info[5 * p + 2]);
    const double diam = info[5 * p + 3];
    if (norm(t - c) >= delta * diam + info[5 * p + 4]) return false;
    const PatchDev P = patches[p];
    dist = project(P, objs[P.obj], t, us, vs);
    return dist < delta * diam;
}

// Pass 1: count near patches per node.  Pass 2: write them in patch order.
__global__ void k_near(const PatchDev* __restrict__ patches, const ObjDev* __restrict__ objs,
                       const double* __restrict__ info, const int* __restrict__ node_patch,
                       const int* __restrict__ obj_patch0, const int* __restrict__ obj_npatch,
                       NodeArrays nd, int n_nodes, double delta, int* __restrict__ counts,
                       const int64_t* __restrict__ offsets, NearPair* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    const int own = node_patch[i];
    const int ob = patches[own].obj;
    const int p0 = obj_patch0[ob], p1 = p0 + obj_npatch[ob];
    int cnt = 0;
    int64_t pos = offsets ? offsets[i] : 0;
    for (int p = p0; p < p1; ++p) {
        double us, vs, dist;
        if (near_test(patches, objs, info, nd, i, p, own, delta, us, vs, dist)) {
            if (out) {
                NearPair e;
                e.target = i; e.patch = p; e.us = us; e.vs = vs; e.dist = dist;
                e.self = (p == own);
                out[pos + cnt] = e;
            }
            ++cnt;
        }
    }
    if (!out) counts[i] = cnt;
}

// ------------------------------------------------- singular / near quadrature
// Barycentric Lagrange basis at first-kind Chebyshev points (ascending):
// ell_l(x) = [lam_l/(x - x_l)] / sum_m [lam_m/(x - x_m)],
// lam_l = (-1)^l sin((2l+1) pi / (2q)) (bary_weights, once per thread).
__device__ inline void bary_weights(int q, double* lam) {
    for (int l = 0; l < q; ++l) lam[l] = ((l & 1) ? -1.0 : 1.0) * sin((2 * l + 1) * M_PI / (2.0 * q));
}
__device__ inline void lagrange(int q, const double* xn, const double* lam, double x, double* L) {
    for (int l = 0; l < q; ++l) {
        if (x == xn[l]) {
            for (int m = 0; m < q; ++m) L[m] = (m == l) ? 1.0 : 0.0;
            return;
        }
    }
    double den = 0.0;
    for (int l = 0; l < q; ++l) {
        L[l] = lam[l] / (x - xn[l]);
        den += L[l];
    }
    const double inv = 1.0 / den;
    for (int l = 0; l < q; ++l) L[l] *= inv;
}

// One work-group of 256 threads per (target node, source patch) pair.
//
// Change of variables (the singularity-cancelling step of Sec. II-B, eq. 20):
// [-1,1]^2 is cut at the singular point P = (u*, v*) into up to four
// rectangles with corner P; each rectangle into two triangles along its
// diagonal; on a triangle x = P + s (a, t b) (or P + s (t a, b)) the Duffy
// Jacobian s|ab| cancels the 1/R singularity.  The angular variable uses
// t = (L1/L2) sinh(sigma asinh(L2/L1)) (L1 the leg along the axis, L2 the
// far side), which flattens the angular peak of thin rectangles.  Radially:
// self pairs use a plain Fejer rule in s; near pairs (target off the patch
// at parameter distance d) use s = e sinh(sigma asinh(s1/e)) on [0, s1],
// e = d/|ray|, s1 = min(1/2, 6e), and a plain Fejer rule on [s1, 1].
// All 1D rules are Fejer-1 on [0, 1] (tables fej_x, fej_w at offset n(n-1)/2).
//
// Contraction: wave w takes the points w, w+4, ... of each tile staged in
// LDS; its lane (k, l) accumulates, for all four (b, a),
//   sum_points w K[b][a](x) ell_k(v) ell_l(u)
// (the basis product once per point for four outputs); the four waves'
// partial sums are added through LDS at the end.
// Triangles of the change of variables around (us, vs): per triangle the
// legs a, b, L1/L2, asinh(L2/L1) and its kind (which leg carries t).
__device__ inline int quad_triangles(double us, double vs, double (*tri)[6]) {
    int nt = 0;
    for (int iu = 0; iu < 2; ++iu) {
        const double a = (iu ? 1.0 : -1.0) - us;
        if (fabs(a) < 1e-14) continue;
        for (int iv = 0; iv < 2; ++iv) {
            const double b = (iv ? 1.0 : -1.0) - vs;
            if (fabs(b) < 1e-14) continue;
            for (int kind = 0; kind < 2; ++kind) {
                const double L1 = kind ? fabs(b) : fabs(a);
                const double L2 = kind ? fabs(a) : fabs(b);
                tri[nt][0] = a;
                tri[nt][1] = b;
                tri[nt][2] = L1 / L2;
                tri[nt][3] = asinh(L2 / L1);
                tri[nt][4] = kind;
                ++nt;
            }
        }
    }
    return nt;
}

// Parameter distance of a near target from its projection point.
template <bool CHEB = true>
__device__ inline double near_param_dist(const PatchDev& P, const ObjDev& O, double us, double vs, double dist) {
    V3 r0, au0, av0;
    patch_eval<CHEB>(P, O, us, vs, r0, au0, av0);
    return dist / sqrt(norm(au0) * norm(av0));
}

// Point pidx of the rule: offset (du, dv) from the singular point and weight.
__device__ inline void quad_point(const double (*tri)[6], int nt, int nr, int self, double dpar,
                                  const QuadRule& rule, const double* fej_x, const double* fej_w, int64_t pidx,
                                  double& du, double& dv, double& wgt) {
    const int t_i = (int)(pidx / ((int64_t)nt * nr));
    const int rem = (int)(pidx % ((int64_t)nt * nr));
    const int it = rem / nr, ir = rem % nr;
    const double a = tri[t_i][0], b = tri[t_i][1];
    const double ratio = tri[t_i][2], hi = tri[t_i][3];
    const int kind = (int)tri[t_i][4];
    const double sig = fej_x[rule.off_ang + it];
    const double t = ratio * sinh(hi * sig);
    const double wt = fej_w[rule.off_ang + it] * hi * ratio * cosh(hi * sig);
    const double eu = kind ? t * a : a;
    const double ev = kind ? b : t * b;
    double s, ws;
    if (self) {
        s = fej_x[rule.off_rad + ir];
        ws = fej_w[rule.off_rad + ir];
    } else {
        const double rho = sqrt(eu * eu + ev * ev);
        const double e = dpar / rho;
        const double s1 = fmin(0.5, 6.0 * e);
        if (ir < rule.n_in) {
            const double h2 = asinh(s1 / e);
            const double sg = fej_x[rule.off_in + ir];
            s = e * sinh(h2 * sg);
            ws = fej_w[rule.off_in + ir] * h2 * e * cosh(h2 * sg);
        } else {
            const int jr = ir - rule.n_in;
            s = s1 + (1.0 - s1) * fej_x[rule.off_out + jr];
            ws = fej_w[rule.off_out + jr] * (1.0 - s1);
        }
    }
    du = s * eu;
    dv = s * ev;
    wgt = wt * ws * s * fabs(a * b);
}

// Point tile of k_quad: w K (4 complex) and the two interpolation bases of
// every point (QM: the largest order the instance handles).
template <int QM> struct QuadPointLDS {
    double kw[256][8];
    double lu[256][QM];
    double lv[256][QM];
};

// QM = 8: lane kl of each wave owns node kl (q^2 <= 64).  QM = 11: lane kl
// owns nodes kl and kl + 64 (q^2 <= 121, up to 242 unknowns per patch, the
// most a 256-unknown leaf holds).
template <int QM, bool CHEB>
__global__ __launch_bounds__(256) void k_quad(
    const PatchDev* __restrict__ patches, const ObjDev* __restrict__ objs, NodeArrays nd,
    const NearPair* __restrict__ pairs, int64_t n_pairs, const double* __restrict__ fej11_x,
    const double* __restrict__ fej_x, const double* __restrict__ fej_w, QuadRule rule,
    int64_t stride, zd* __restrict__ out) {
    constexpr int NPL = (QM * QM + 63) / 64;   // nodes per lane
    __shared__ QuadPointLDS<QM> S;
    __shared__ double s_tri[8][6];   // per triangle: a, b, L1/L2, hi, kind(0/1), valid
    __shared__ int s_ntri;
    const int64_t pid = blockIdx.x;
    if (pid >= n_pairs) return;
    const NearPair E = pairs[pid];
    const PatchDev P = patches[E.patch];
    const ObjDev O = objs[P.obj];
    const int q = P.q;
    const int i = E.target;
    const V3 rt = v3(nd.rx[i], nd.ry[i], nd.rz[i]);
    const V3 aut = v3(nd.aux[i], nd.auy[i], nd.auz[i]);
    const V3 avt = v3(nd.avx[i], nd.avy[i], nd.avz[i]);
    const double us = E.us, vs = E.vs;
    const double* xq = fej11_x + q * (q - 1) / 2;   // the patch's own Chebyshev points
    const int tid = threadIdx.x;
    double lam[QM];
    bary_weights(q, lam);

    if (tid == 0) s_ntri = quad_triangles(us, vs, s_tri);
    __syncthreads();
    const int ntri = s_ntri;
    const double dpar = E.self ? 0.0 : near_param_dist<CHEB>(P, O, us, vs, E.dist);
    const int nt = rule.n_ang;
    const int nr = E.self ? rule.n_rad : (rule.n_in + rule.n_out);
    const int64_t npts = (int64_t)ntri * nt * nr;

    // output ownership: lane (k, l) (and (k, l) + 64), every (b, a), a
    // quarter of the points
    const int q2 = q * q;
    const int wave = tid >> 6, kl = tid & 63;
    int ok[NPL], ol[NPL];
    bool owner[NPL];
#pragma unroll
    for (int h = 0; h < NPL; ++h) {
        const int nn = kl + 64 * h;
        owner[h] = nn < q2;
        ok[h] = owner[h] ? nn / q : 0;
        ol[h] = owner[h] ? nn % q : 0;
    }
    double acc[NPL][8];   // (re, im) for ba = 0..3
#pragma unroll
    for (int h = 0; h < NPL; ++h)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[h][c] = 0.0;

    for (int64_t base = 0; base < npts; base += 256) {
        const int64_t pidx = base + tid;
        double kw[8];
        double Lu[QM], Lv[QM];
        for (int c = 0; c < 8; ++c) kw[c] = 0.0;
        for (int c = 0; c < QM; ++c) { Lu[c] = 0.0; Lv[c] = 0.0; }
        if (pidx < npts) {
            double du, dv, wgt;
            quad_point(s_tri, nt, nr, E.self, dpar, rule, fej_x, fej_w, pidx, du, dv, wgt);
            const double u = us + du, v = vs + dv;
            V3 r, au, av;
            patch_eval<CHEB>(P, O, u, v, r, au, av);
            const V3 R = E.self ? patch_delta<CHEB>(P, O, us, vs, du, dv) : (rt - r);
            zd K[2][2];
            mfie_kernel(O.k0, R, aut, avt, au, av, K);
            kw[0] = wgt * K[0][0].re; kw[1] = wgt * K[0][0].im;
            kw[2] = wgt * K[0][1].re; kw[3] = wgt * K[0][1].im;
            kw[4] = wgt * K[1][0].re; kw[5] = wgt * K[1][0].im;
            kw[6] = wgt * K[1][1].re; kw[7] = wgt * K[1][1].im;
            lagrange(q, xq, lam, u, Lu);
            lagrange(q, xq, lam, v, Lv);
        }
        __syncthreads();
        for (int c = 0; c < 8; ++c) S.kw[tid][c] = kw[c];
        for (int c = 0; c < QM; ++c) {
            S.lu[tid][c] = Lu[c];
            S.lv[tid][c] = Lv[c];
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)256, npts - base);
#pragma unroll
        for (int h = 0; h < NPL; ++h) {
            if (!owner[h]) continue;
            for (int pnt = wave; pnt < cnt; pnt += 4) {
                const double bb = S.lv[pnt][ok[h]] * S.lu[pnt][ol[h]];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[h][c] = fma(S.kw[pnt][c], bb, acc[h][c]);
            }
        }
    }
    // sum the four waves' partials (the point tile is no longer needed)
    __syncthreads();
    double (*red)[64 * NPL][8] = reinterpret_cast<double (*)[64 * NPL][8]>(&S.kw[0][0]);   // [wave][node][8]
    static_assert(sizeof(double) * 4 * 64 * NPL * 8 <= sizeof(QuadPointLDS<QM>), "reduction buffer");
#pragma unroll
    for (int h = 0; h < NPL; ++h)
#pragma unroll
        for (int c = 0; c < 8; ++c) red[wave][kl + 64 * h][c] = acc[h][c];
    __syncthreads();
    for (int o = tid; o < 4 * q2; o += 256) {
        // thread -> (ba, kl2): output (b, a) of node kl2
        const int ba = o / q2, kl2 = o % q2;
        const int b = ba >> 1, a = ba & 1;
        double re = 0.0, im = 0.0;
        for (int w = 0; w < 4; ++w) {
            re += red[w][kl2][2 * ba];
            im += red[w][kl2][2 * ba + 1];
        }
        // identity term 1/2 F^b at the target node itself
        if (E.self && a == b && (P.node0 + kl2) == i) re += 0.5;
        out[pid * stride + ((int64_t)b * q2 + kl2) * 2 + a] = zd{re, im};
    }
}
#define CBIE_KQUAD_INST(QM, CH)                                                                                \
    template __global__ void k_quad<QM, CH>(const PatchDev*, const ObjDev*, NodeArrays, const NearPair*, int64_t, \
                                            const double*, const double*, const double*, QuadRule, int64_t, zd*);
CBIE_KQUAD_INST(8, false)
CBIE_KQUAD_INST(11, false)
CBIE_KQUAD_INST(8, true)
CBIE_KQUAD_INST(11, true)

// ------------------------------------------------------------- far fill
// Dense block tile: 64 row nodes x 16 column nodes per work-group; thread
// (ti, tj4) handles row node ti and four column nodes.  Entries use the
// plain Fejer rule  A[(i,b),(j,a)] = w_j K[b][a](r_i - r_j).  Column-major
// storage: rows 2i, 2i+1 of column 2j+a are adjacent, so a wave writes
// 64 x 32 contiguous bytes per column.
template <typename T>
__global__ __launch_bounds__(256) void k_far_fill(const DenseTile* __restrict__ tiles, int n_tiles,
                                                  const DenseBlockDev* __restrict__ blocks,
                                                  const int* __restrict__ tree_node, NodeArrays nd,
                                                  const ObjDev* __restrict__ objs,
                                                  cplx<T>* __restrict__ store) {
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const DenseTile Tl = tiles[tile];
    const DenseBlockDev B = blocks[Tl.block];
    const int ti = Tl.row0 + (threadIdx.x & 63);
    if (ti >= B.row_nodes) return;
    const int gi = tree_node[B.row_node0 + ti];
    const V3 ri = v3(nd.rx[gi], nd.ry[gi], nd.rz[gi]);
    const V3 aui = v3(nd.aux[gi], nd.auy[gi], nd.auz[gi]);
    const V3 avi = v3(nd.avx[gi], nd.avy[gi], nd.avz[gi]);
    const double k = objs[B.obj].k0;
    cplx<T>* base = store + B.offset;
    for (int c = 0; c < 4; ++c) {
        const int tj = Tl.col0 + (threadIdx.x >> 6) * 4 + c;
        if (tj >= B.col_nodes) break;
        const int gj = tree_node[B.col_node0 + tj];
        zd K[2][2];
        if (gi == gj) {
            K[0][0] = K[0][1] = K[1][0] = K[1][1] = zd{0.0, 0.0};
        } else {
            const V3 R = ri - v3(nd.rx[gj], nd.ry[gj], nd.rz[gj]);
            mfie_kernel(k, R, aui, avi, v3(nd.aux[gj], nd.auy[gj], nd.auz[gj]),
                        v3(nd.avx[gj], nd.avy[gj], nd.avz[gj]), K);
        }
        const double w = nd.w[gj];
        for (int a = 0; a < 2; ++a) {
            cplx<T>* col = base + (int64_t)(2 * tj + a) * B.ld + 2 * ti;
            col[0] = cplx<T>{(T)(w * K[0][a].re), (T)(w * K[0][a].im)};
            col[1] = cplx<T>{(T)(w * K[1][a].re), (T)(w * K[1][a].im)};
        }
    }
}

// Overwrite the near/self entries of each pair in its dense block.
template <typename T>
__global__ void k_near_scatter(const NearDest* __restrict__ dest, int64_t n_pairs, int64_t stride,
                               const zd* __restrict__ vals, const DenseBlockDev* __restrict__ blocks,
                               cplx<T>* __restrict__ store) {
    const int64_t pid = blockIdx.x;
    if (pid >= n_pairs) return;
    const NearDest D = dest[pid];
    const int q2 = D.q2;
    const DenseBlockDev B = blocks[D.block];
    const int upn = B.upn;
    for (int t = threadIdx.x; t < upn * upn * q2; t += blockDim.x) {
        const int b = t / (upn * q2);
        const int rem = t % (upn * q2);
        const int jl = rem / upn, a = rem % upn;
        const zd v = vals[pid * stride + t];
        const int64_t row = upn * (int64_t)D.row_node + b;
        const int64_t col = upn * (int64_t)(D.col_node0 + jl) + a;
        store[B.offset + col * B.ld + row] = cplx<T>{(T)v.re, (T)v.im};
    }
}

// ============================================================ N-Mueller
// Lagrange basis at first-kind Chebyshev points and its derivative at x:
// with t_k = lam_k / (x - x_k), S = sum_k t_k,
//   ell_m(x) = t_m / S,
//   ell_m'(x) = (t_m / S^2) sum_{k != m} t_k (x_k - x_m) / ((x - x_k)(x - x_m)),
// a form without cancellation next to a node (every term is a product).
// At a node the derivative row comes from the differentiation matrix D.
__device__ inline void lagrange_d(int q, const double* xn, const double* lam, const double* D, double x, double* L,
                                  double* dL) {
    for (int l = 0; l < q; ++l) {
        if (x == xn[l]) {
            for (int m = 0; m < q; ++m) {
                L[m] = (m == l) ? 1.0 : 0.0;
                dL[m] = D[l * q + m];
            }
            return;
        }
    }
    double t[8], S = 0.0;
    for (int l = 0; l < q; ++l) {
        t[l] = lam[l] / (x - xn[l]);
        S += t[l];
    }
    const double iS = 1.0 / S;
    for (int m = 0; m < q; ++m) {
        double acc = 0.0;
        for (int k = 0; k < q; ++k)
            if (k != m) acc += t[k] * (xn[k] - xn[m]) / ((x - xn[k]) * (x - xn[m]));
        L[m] = t[m] * iS;
        dL[m] = t[m] * iS * iS * acc;
    }
}

__device__ inline int dmat_offset(int q) { return (q - 1) * q * (2 * q - 1) / 6; }

// Self/near integrals of the sixteen N-Mueller entries: one work-group per
// (target node, source patch) pair, the same change of variables as k_quad.
// Per point: the twelve distinct kernel values (X0, CH, CE) and the two
// divergence weights phi.  Wave w takes the points w, w+4, ... of each
// tile; its lane (k, l) accumulates the twelve outputs of that node:
//   X:  sum w (X0[b][a] ell_k(v) ell_l(u) + phi[b] d_a(ell_k(v) ell_l(u)))
//   CH: sum w CH[b][a] ell_k(v) ell_l(u),   CE likewise,
// and the four waves' partials are added through LDS.  Written as
// (4, q^2, 4) [row c, source node, column a]; the identity terms
// (mu_1 + mu_2)/2 and -(eps_1 + eps_2)/2 are added at the target node.
constexpr int kNmTile = 128;
struct QuadNmLDS {
    double val[kNmTile][28];
    double lu[kNmTile][8], lv[kNmTile][8], dlu[kNmTile][8], dlv[kNmTile][8];
};

__global__ __launch_bounds__(256) void k_quad_nm(
    const PatchDev* __restrict__ patches, const ObjDev* __restrict__ objs, NodeArrays nd,
    const NearPair* __restrict__ pairs, int64_t n_pairs, const double* __restrict__ fej11_x,
    const double* __restrict__ fej_x, const double* __restrict__ fej_w, const double* __restrict__ dmat,
    QuadRule rule, int64_t stride, zd* __restrict__ out) {
    __shared__ QuadNmLDS S;
    __shared__ double s_tri[8][6];
    __shared__ int s_ntri;
    const int64_t pid = blockIdx.x;
    if (pid >= n_pairs) return;
    const NearPair E = pairs[pid];
    const PatchDev P = patches[E.patch];
    const ObjDev O = objs[P.obj];
    const NmMat M = nm_mat(O);
    const int q = P.q;
    const int i = E.target;
    const V3 rt = v3(nd.rx[i], nd.ry[i], nd.rz[i]);
    const V3 aut = v3(nd.aux[i], nd.auy[i], nd.auz[i]);
    const V3 avt = v3(nd.avx[i], nd.avy[i], nd.avz[i]);
    const double us = E.us, vs = E.vs;
    const double* xq = fej11_x + q * (q - 1) / 2;
    const double* Dq = dmat + dmat_offset(q);
    const int tid = threadIdx.x;
    double lam[8];
    bary_weights(q, lam);
    if (tid == 0) s_ntri = quad_triangles(us, vs, s_tri);
    __syncthreads();
    const int ntri = s_ntri;
    const double dpar = E.self ? 0.0 : near_param_dist(P, O, us, vs, E.dist);
    const int nt = rule.n_ang;
    const int nr = E.self ? rule.n_rad : (rule.n_in + rule.n_out);
    const int64_t npts = (int64_t)ntri * nt * nr;
    const int q2 = q * q;
    const int wave = tid >> 6, kl = tid & 63;
    const bool owner = kl < q2;
    const int ok = owner ? kl / q : 0, ol = owner ? kl % q : 0;
    double acc[24];   // (re, im) of X[ba], CH[ba], CE[ba], ba = 2b + a
    for (int c = 0; c < 24; ++c) acc[c] = 0.0;

    for (int64_t base = 0; base < npts; base += kNmTile) {
        const int64_t pidx = base + tid;
        double vals[28];
        double Lu[8], Lv[8], dLu[8], dLv[8];
        for (int c = 0; c < 28; ++c) vals[c] = 0.0;
        for (int c = 0; c < 8; ++c) { Lu[c] = Lv[c] = dLu[c] = dLv[c] = 0.0; }
        if (tid < kNmTile && pidx < npts) {
            double du, dv, wgt;
            quad_point(s_tri, nt, nr, E.self, dpar, rule, fej_x, fej_w, pidx, du, dv, wgt);
            const double u = us + du, v = vs + dv;
            V3 r, au, av;
            patch_eval(P, O, u, v, r, au, av);
            const V3 R = E.self ? patch_delta(P, O, us, vs, du, dv) : (rt - r);
            NmVals K;
            nm_kernel(M, R, aut, avt, au, av, K);
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    const int e = 2 * (2 * b + a);
                    vals[e] = wgt * K.X0[b][a].re;
                    vals[e + 1] = wgt * K.X0[b][a].im;
                    vals[8 + e] = wgt * K.CH[b][a].re;
                    vals[8 + e + 1] = wgt * K.CH[b][a].im;
                    vals[16 + e] = wgt * K.CE[b][a].re;
                    vals[16 + e + 1] = wgt * K.CE[b][a].im;
                }
            for (int b = 0; b < 2; ++b) {
                vals[24 + 2 * b] = wgt * K.phi[b].re;
                vals[24 + 2 * b + 1] = wgt * K.phi[b].im;
            }
            lagrange_d(q, xq, lam, Dq, u, Lu, dLu);
            lagrange_d(q, xq, lam, Dq, v, Lv, dLv);
        }
        __syncthreads();
        if (tid < kNmTile) {
            for (int c = 0; c < 28; ++c) S.val[tid][c] = vals[c];
            for (int c = 0; c < 8; ++c) {
                S.lu[tid][c] = Lu[c];
                S.lv[tid][c] = Lv[c];
                S.dlu[tid][c] = dLu[c];
                S.dlv[tid][c] = dLv[c];
            }
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)kNmTile, npts - base);
        if (owner) {
            for (int pnt = wave; pnt < cnt; pnt += 4) {
                const double lv = S.lv[pnt][ok], lu = S.lu[pnt][ol];
                const double bas = lv * lu;
                const double du = lv * S.dlu[pnt][ol], dv = S.dlv[pnt][ok] * lu;   // d_u, d_v of the basis
                const double* V = S.val[pnt];
#pragma unroll
                for (int ba = 0; ba < 4; ++ba) {
                    const int b = ba >> 1;
                    const double db = (ba & 1) ? dv : du;
                    acc[2 * ba] = fma(V[2 * ba], bas, fma(V[24 + 2 * b], db, acc[2 * ba]));
                    acc[2 * ba + 1] = fma(V[2 * ba + 1], bas, fma(V[25 + 2 * b], db, acc[2 * ba + 1]));
                    acc[8 + 2 * ba] = fma(V[8 + 2 * ba], bas, acc[8 + 2 * ba]);
                    acc[9 + 2 * ba] = fma(V[9 + 2 * ba], bas, acc[9 + 2 * ba]);
                    acc[16 + 2 * ba] = fma(V[16 + 2 * ba], bas, acc[16 + 2 * ba]);
                    acc[17 + 2 * ba] = fma(V[17 + 2 * ba], bas, acc[17 + 2 * ba]);
                }
            }
        }
    }
    // sum the four waves' partials (the point tile is no longer needed)
    __syncthreads();
    double (*red)[64][24] = reinterpret_cast<double (*)[64][24]>(&S);   // [wave][lane][24]
    static_assert(sizeof(double) * 4 * 64 * 24 <= sizeof(QuadNmLDS), "reduction buffer");
    for (int c = 0; c < 24; ++c) red[wave][kl][c] = acc[c];
    __syncthreads();
    zd* dst = out + pid * stride;
    for (int o = tid; o < 12 * q2; o += 256) {
        const int type = o / (4 * q2), rem = o % (4 * q2);
        const int ba = rem / q2, kl2 = rem % q2;
        const int b = ba >> 1, a = ba & 1;
        const int c = 8 * type + 2 * ba;
        double re = 0.0, im = 0.0;
        for (int w = 0; w < 4; ++w) {
            re += red[w][kl2][c];
            im += red[w][kl2][c + 1];
        }
        const int kl = kl2;
        const bool diag = E.self && a == b && (P.node0 + kl) == i;
        const zd v{re, im};
        if (type == 0) {
            dst[((int64_t)b * q2 + kl) * 4 + 2 + a] = v;            // H_b x M^a
            dst[((int64_t)(2 + b) * q2 + kl) * 4 + a] = v;          // E_b x J^a
        } else if (type == 1) {
            dst[((int64_t)b * q2 + kl) * 4 + a] = zd{v.re + (diag ? 0.5 * (1.0 + M.m2) : 0.0), v.im};
        } else {
            dst[((int64_t)(2 + b) * q2 + kl) * 4 + 2 + a] = zd{v.re - (diag ? 0.5 * (1.0 + M.e2) : 0.0), v.im};
        }
    }
}

// Far (Fejer-rule) entries of N-Mueller blocks, column-major with leading
// dimension ld = 4 row_nodes.  A work-group takes 32 row nodes against one
// source patch (tile.col0: its first local column node, tile.pad: q).  The
// surface divergence of the source is the derivative of its Chebyshev
// interpolant: the weight phi of node (k, l) reaches column (k, m) of the
// u-component through D[l][m] and column (m, l) of the v-component through
// D[k][m].  Pass 1 stages w phi in LDS, pass 2 writes all sixteen entries.
// Self pairs are left zero (near pairs are overwritten by k_quad_nm).
template <typename T>
__global__ __launch_bounds__(256) void k_far_fill_nm(const DenseTile* __restrict__ tiles, int n_tiles,
                                                     const DenseBlockDev* __restrict__ blocks,
                                                     const int* __restrict__ tree_node, NodeArrays nd,
                                                     const ObjDev* __restrict__ objs,
                                                     const double* __restrict__ dmat, cplx<T>* __restrict__ store) {
    __shared__ zd s_phi[2][32][65];
    __shared__ double s_D[64];
    const int tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const DenseTile Tl = tiles[tile];
    const DenseBlockDev B = blocks[Tl.block];
    const int q = Tl.pad, q2 = q * q;
    const NmMat M = nm_mat(objs[B.obj]);
    const double* Dq = dmat + dmat_offset(q);
    for (int e = threadIdx.x; e < q2; e += 256) s_D[e] = Dq[e];
    const int nrow = min(32, B.row_nodes - Tl.row0);
    for (int p = threadIdx.x; p < 32 * q2; p += 256) {
        const int il = p & 31, j = p >> 5;
        zd ph[2] = {zd{0.0, 0.0}, zd{0.0, 0.0}};
        if (il < nrow) {
            const int gi = tree_node[B.row_node0 + Tl.row0 + il];
            const int gj = tree_node[B.col_node0 + Tl.col0 + j];
            if (gi != gj) {
                NmVals K;
                nm_kernel(M, v3(nd.rx[gi] - nd.rx[gj], nd.ry[gi] - nd.ry[gj], nd.rz[gi] - nd.rz[gj]),
                          v3(nd.aux[gi], nd.auy[gi], nd.auz[gi]), v3(nd.avx[gi], nd.avy[gi], nd.avz[gi]),
                          v3(nd.aux[gj], nd.auy[gj], nd.auz[gj]), v3(nd.avx[gj], nd.avy[gj], nd.avz[gj]), K);
                const double w = nd.w[gj];
                ph[0] = w * K.phi[0];
                ph[1] = w * K.phi[1];
            }
        }
        s_phi[0][il][j] = ph[0];
        s_phi[1][il][j] = ph[1];
    }
    __syncthreads();
    cplx<T>* base = store + B.offset;
    for (int p = threadIdx.x; p < 32 * q2; p += 256) {
        const int il = p & 31, j = p >> 5;
        if (il >= nrow) continue;
        const int ti = Tl.row0 + il;
        const int gi = tree_node[B.row_node0 + ti];
        const int gj = tree_node[B.col_node0 + Tl.col0 + j];
        NmVals K;
        double w = 0.0;
        if (gi != gj) {
            nm_kernel(M, v3(nd.rx[gi] - nd.rx[gj], nd.ry[gi] - nd.ry[gj], nd.rz[gi] - nd.rz[gj]),
                      v3(nd.aux[gi], nd.auy[gi], nd.auz[gi]), v3(nd.avx[gi], nd.avy[gi], nd.avz[gi]),
                      v3(nd.aux[gj], nd.auy[gj], nd.auz[gj]), v3(nd.avx[gj], nd.avy[gj], nd.avz[gj]), K);
            w = nd.w[gj];
        } else {
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) K.X0[b][a] = K.CH[b][a] = K.CE[b][a] = zd{0.0, 0.0};
        }
        const int kk = j / q, ll = j % q;
        zd dvu[2], dvv[2];
        for (int b = 0; b < 2; ++b) {
            zd su{0.0, 0.0}, sv{0.0, 0.0};
            for (int m = 0; m < q; ++m) {
                cfma(su, zd{s_D[m * q + ll], 0.0}, s_phi[b][il][kk * q + m]);
                cfma(sv, zd{s_D[m * q + kk], 0.0}, s_phi[b][il][m * q + ll]);
            }
            dvu[b] = su;
            dvv[b] = sv;
        }
        const int64_t row = 4 * (int64_t)ti;
        for (int a = 0; a < 2; ++a) {
            const int64_t cj = 4 * (int64_t)(Tl.col0 + j) + a, cm = cj + 2;
            cplx<T>* colJ = base + cj * B.ld + row;
            cplx<T>* colM = base + cm * B.ld + row;
            for (int b = 0; b < 2; ++b) {
                const zd X = w * K.X0[b][a] + (a ? dvv[b] : dvu[b]);
                const zd ch = w * K.CH[b][a], ce = w * K.CE[b][a];
                colJ[b] = cplx<T>{(T)ch.re, (T)ch.im};
                colJ[2 + b] = cplx<T>{(T)X.re, (T)X.im};
                colM[b] = cplx<T>{(T)X.re, (T)X.im};
                colM[2 + b] = cplx<T>{(T)ce.re, (T)ce.im};
            }
        }
    }
}

template __global__ void k_far_fill_nm<double>(const DenseTile*, int, const DenseBlockDev*, const int*, NodeArrays,
                                               const ObjDev*, const double*, zd*);

template __global__ void k_far_fill<double>(const DenseTile*, int, const DenseBlockDev*, const int*,
                                            NodeArrays, const ObjDev*, zd*);
template __global__ void k_far_fill<float>(const DenseTile*, int, const DenseBlockDev*, const int*,
                                           NodeArrays, const ObjDev*, zf*);
template __global__ void k_near_scatter<double>(const NearDest*, int64_t, int64_t, const zd*,
                                                const DenseBlockDev*, zd*);
template __global__ void k_near_scatter<float>(const NearDest*, int64_t, int64_t, const zd*,
                                               const DenseBlockDev*, zf*);

}  // namespace cbie

namespace cbie {

// ----------------------------------------------------------- dense export
// Scatter a dense block (tree order, column-major) into an N x N matrix in
// the original unknown order.
__global__ void k_export_dense_block(const DenseBlockDev* __restrict__ blocks, int n_blocks,
                                     const int* __restrict__ tree_node, const zd* __restrict__ store,
                                     zd* __restrict__ A, int64_t lda) {
    const int bid = blockIdx.y;
    if (bid >= n_blocks) return;
    const DenseBlockDev B = blocks[bid];
    const int upn = B.upn;
    const int64_t m = upn * (int64_t)B.row_nodes, n = upn * (int64_t)B.col_nodes;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % m, c = e / m;
        const int64_t gr = upn * (int64_t)tree_node[B.row_node0 + r / upn] + (r % upn);
        const int64_t gc = upn * (int64_t)tree_node[B.col_node0 + c / upn] + (c % upn);
        A[gc * lda + gr] = store[B.offset + c * B.ld + r];
    }
}

// Plain-rule entries of a block (used for admissible blocks before
// compression), written in the original order.
__global__ void k_export_far(const DenseBlockDev* __restrict__ blocks, int n_blocks,
                             const int* __restrict__ tree_node, NodeArrays nd,
                             const ObjDev* __restrict__ objs, zd* __restrict__ A, int64_t lda) {
    const int bid = blockIdx.y;
    if (bid >= n_blocks) return;
    const DenseBlockDev B = blocks[bid];
    const int64_t np = (int64_t)B.row_nodes * B.col_nodes;
    const double k = objs[B.obj].k0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int gi = tree_node[B.row_node0 + e % B.row_nodes];
        const int gj = tree_node[B.col_node0 + e / B.row_nodes];
        const V3 R = v3(nd.rx[gi] - nd.rx[gj], nd.ry[gi] - nd.ry[gj], nd.rz[gi] - nd.rz[gj]);
        zd K[2][2];
        mfie_kernel(k, R, v3(nd.aux[gi], nd.auy[gi], nd.auz[gi]), v3(nd.avx[gi], nd.avy[gi], nd.avz[gi]),
                    v3(nd.aux[gj], nd.auy[gj], nd.auz[gj]), v3(nd.avx[gj], nd.avy[gj], nd.avz[gj]), K);
        const double w = nd.w[gj];
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                A[(2 * (int64_t)gj + a) * lda + 2 * (int64_t)gi + b] = zd{w * K[b][a].re, w * K[b][a].im};
    }
}

}  // namespace cbie

// Patch geometry and the MFIE kernel on the device (FP64).
//
// Equiangular cube-sphere patch on an ellipsoid (the paper gives no map for
// its spheres): xi = (2i+1+u)/s - 1, eta = (2j+1+v)/s - 1,
// c = e_n + tan(pi xi/4) e_1 + tan(pi eta/4) e_2, r = center + diag(axes) c/|c|.
// Covariant basis a_u = dr/du, a_v = dr/dv (eq. 14).
//
// Chebyshev-interpolated patch (generic surface input, e.g. from CAD):
// r(u, v) = sum_{n, m <= deg} C[c][n][m] T_n(u) T_m(v) per coordinate c,
// a_u and a_v from T_n'(x) = n U_{n-1}(x).
#pragma once
#include "common.hpp"

namespace cbie {

struct PatchDev {
    int face, i, j, split;   // Chebyshev-interpolated objects: i = the patch's index in the coefficient table
    int obj;          // object index
    int node0;        // first node (original order)
    int q;
    int pad;
};

constexpr int kChebMaxDeg = 16;   // highest degree of a Chebyshev-interpolated patch

struct ObjDev {
    double axes[3];
    double center[3];
    double k0;
    int q;
    int form;
    double eps_r, mu_r;   // interior material (N-Mueller)
    const double* coef;   // Chebyshev-interpolated patches: device table [patch][3][deg+1][deg+1]
    int deg;              // their degree (0: cube-sphere patches on the ellipsoid)
    int pad;
};

__device__ __constant__ static const double kFaceFrames[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, 0, 1}, {0, 1, 0}},
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 0}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {1, 0, 0}, {0, 1, 0}},
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

struct V3 { double x, y, z; };
__device__ inline V3 v3(double x, double y, double z) { return V3{x, y, z}; }
__device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline double norm(V3 a) { return sqrt(dot(a, a)); }
__device__ inline V3 mulc(const double* s, V3 a) { return {s[0] * a.x, s[1] * a.y, s[2] * a.z}; }

__device__ inline V3 frame(int f, int row) {
    return v3(kFaceFrames[f][row][0], kFaceFrames[f][row][1], kFaceFrames[f][row][2]);
}

// Chebyshev-interpolated patch: every T_n and its derivative n U_{n-1} by
// running recurrences (no tables), so the evaluation needs few registers
// and no stack inside the quadrature kernels.
__device__ inline void cheb_patch_eval(const double* __restrict__ C, int deg, double u, double v, V3& r, V3& au,
                                       V3& av) {
    const int d1 = deg + 1;
    double x[3] = {0.0, 0.0, 0.0}, xu[3] = {0.0, 0.0, 0.0}, xv[3] = {0.0, 0.0, 0.0};
    double tn = 1.0, tp = u, un = 0.0, up = 1.0;   // T_n(u), T_{n-1}(u) (T_{-1} = T_1), U_{n-1}(u), U_{n-2}(u)
    for (int n = 0; n < d1; ++n) {
        const double dtn = n * un;                   // T_n'(u) = n U_{n-1}(u)
        for (int c = 0; c < 3; ++c) {
            const double* row = C + ((size_t)c * d1 + n) * d1;
            double s0 = 0.0, s1 = 0.0;
            double tm = 1.0, tq = v, um = 0.0, uq = 1.0;
            for (int m = 0; m < d1; ++m) {
                s0 += row[m] * tm;
                s1 += row[m] * (m * um);
                const double t2 = (m == 0 ? v : 2.0 * v * tm - tq);
                tq = tm;
                tm = t2;
                const double u2 = (m == 0 ? 1.0 : 2.0 * v * um - uq);
                uq = um;
                um = u2;
            }
            x[c] += tn * s0;
            xu[c] += dtn * s0;
            xv[c] += tn * s1;
        }
        const double t2 = (n == 0 ? u : 2.0 * u * tn - tp);
        tp = tn;
        tn = t2;
        const double u2 = (n == 0 ? 1.0 : 2.0 * u * un - up);
        up = un;
        un = u2;
    }
    r = v3(x[0], x[1], x[2]);
    au = v3(xu[0], xu[1], xu[2]);
    av = v3(xv[0], xv[1], xv[2]);
}

// r(u0, v0) - r(u0 + du, v0 + dv) of a Chebyshev-interpolated patch without
// cancellation: T_n(u0) T_m(v0) - T_n(u1) T_m(v1) =
// (T_n(u0) - T_n(u1)) T_m(v0) + T_n(u1) (T_m(v0) - T_m(v1)); each difference
// D_n = T_n(a) - T_n(b), b = a - d, runs D_0 = 0, D_1 = d,
// D_{n+1} = 2 a D_n + 2 d T_n(b) - D_{n-1}, with the step d as given.
__device__ inline V3 cheb_patch_delta(const double* __restrict__ C, int deg, double u0, double v0, double du,
                                      double dv) {
    const int d1 = deg + 1;
    const double du_ = -du, dv_ = -dv, u1 = u0 + du, v1 = v0 + dv;
    double x[3] = {0.0, 0.0, 0.0};
    double Dn = 0.0, Dp = 0.0, bn = 1.0, bp = 0.0;   // D_n, D_{n-1}, T_n(u1), T_{n-1}(u1)
    for (int n = 0; n < d1; ++n) {
        for (int c = 0; c < 3; ++c) {
            const double* row = C + ((size_t)c * d1 + n) * d1;
            double s0 = 0.0, s1 = 0.0;
            double Em = 0.0, Eq = 0.0, am = 1.0, aq = 0.0, cm = 1.0, cq = 0.0;   // D_m(v), T_m(v0), T_m(v1)
            for (int m = 0; m < d1; ++m) {
                s0 += row[m] * am;
                s1 += row[m] * Em;
                const double E2 = (m == 0 ? dv_ : 2.0 * v0 * Em + 2.0 * dv_ * cm - Eq);
                Eq = Em;
                Em = E2;
                const double a2 = (m == 0 ? v0 : 2.0 * v0 * am - aq);
                aq = am;
                am = a2;
                const double c2 = (m == 0 ? v1 : 2.0 * v1 * cm - cq);
                cq = cm;
                cm = c2;
            }
            x[c] += Dn * s0 + bn * s1;
        }
        const double D2 = (n == 0 ? du_ : 2.0 * u0 * Dn + 2.0 * du_ * bn - Dp);
        Dp = Dn;
        Dn = D2;
        const double b2 = (n == 0 ? u1 : 2.0 * u1 * bn - bp);
        bp = bn;
        bn = b2;
    }
    return v3(x[0], x[1], x[2]);
}

__device__ inline const double* cheb_coef(const PatchDev& P, const ObjDev& O) {
    return O.coef + (size_t)P.i * 3 * (O.deg + 1) * (O.deg + 1);
}

// r, a_u, a_v of a cube-sphere patch at (u, v)
__device__ inline void sphere_patch_eval(const PatchDev& P, const ObjDev& O, double u, double v, V3& r, V3& au,
                                         V3& av) {
    const double s = (double)P.split;
    const double xi = (2.0 * P.i + 1.0 + u) / s - 1.0;
    const double eta = (2.0 * P.j + 1.0 + v) / s - 1.0;
    const double tx = tan(M_PI * 0.25 * xi);
    const double ty = tan(M_PI * 0.25 * eta);
    const V3 en = frame(P.face, 0), e1 = frame(P.face, 1), e2 = frame(P.face, 2);
    const V3 c = en + tx * e1 + ty * e2;
    const double cn = norm(c);
    const V3 p = (1.0 / cn) * c;
    const V3 dcu = (M_PI / (4.0 * s)) * (1.0 + tx * tx) * e1;
    const V3 dcv = (M_PI / (4.0 * s)) * (1.0 + ty * ty) * e2;
    const V3 dpu = (1.0 / cn) * (dcu - dot(p, dcu) * p);
    const V3 dpv = (1.0 / cn) * (dcv - dot(p, dcv) * p);
    r = v3(O.center[0], O.center[1], O.center[2]) + mulc(O.axes, p);
    au = mulc(O.axes, dpu);
    av = mulc(O.axes, dpv);
}

// r(u0, v0) - r(u0 + du, v0 + dv) formed without cancellation: the tangent
// difference uses tan a - tan b = sin(a - b)/(cos a cos b) and the
// normalisation difference uses |c1|^2 - |c0|^2 = (c1 - c0).(c1 + c0).
__device__ inline V3 sphere_patch_delta(const PatchDev& P, const ObjDev& O, double u0, double v0, double du,
                                        double dv) {
    const double s = (double)P.split;
    const double q4 = M_PI * 0.25 / s;
    const double a0 = M_PI * 0.25 * ((2.0 * P.i + 1.0 + u0) / s - 1.0);
    const double b0 = M_PI * 0.25 * ((2.0 * P.j + 1.0 + v0) / s - 1.0);
    const double a1 = a0 + q4 * du, b1 = b0 + q4 * dv;
    const double ca0 = cos(a0), ca1 = cos(a1), cb0 = cos(b0), cb1 = cos(b1);
    const double dtx = -sin(q4 * du) / (ca0 * ca1);   // tan a0 - tan a1
    const double dty = -sin(q4 * dv) / (cb0 * cb1);
    const V3 en = frame(P.face, 0), e1 = frame(P.face, 1), e2 = frame(P.face, 2);
    const V3 dc = dtx * e1 + dty * e2;               // c0 - c1
    const V3 c0 = en + tan(a0) * e1 + tan(b0) * e2;
    const V3 c1 = en + tan(a1) * e1 + tan(b1) * e2;
    const double n0 = norm(c0), n1 = norm(c1);
    const double d2 = -dot(dc, c0 + c1);             // |c1|^2 - |c0|^2
    const V3 dp = (1.0 / n0) * dc + (d2 / (n0 * n1 * (n0 + n1))) * c1;
    return mulc(O.axes, dp);
}

// Either patch kind.  CHEB = false leaves the Chebyshev branch out, for
// the hot quadrature kernel of contexts without such patches.
template <bool CHEB = true>
__device__ inline void patch_eval(const PatchDev& P, const ObjDev& O, double u, double v, V3& r, V3& au, V3& av) {
    if (CHEB && O.deg > 0) cheb_patch_eval(cheb_coef(P, O), O.deg, u, v, r, au, av);
    else sphere_patch_eval(P, O, u, v, r, au, av);
}
template <bool CHEB = true>
__device__ inline V3 patch_delta(const PatchDev& P, const ObjDev& O, double u0, double v0, double du, double dv) {
    if (CHEB && O.deg > 0) return cheb_patch_delta(cheb_coef(P, O), O.deg, u0, v0, du, dv);
    return sphere_patch_delta(P, O, u0, v0, du, dv);
}

// MFIE kernel entries K[b][a] (see the library header): with
// g = -(1 + j k R) e^{-j k R} / (4 pi R^3),
//   K[u][a] =  g R.(a_a(src) x a_v(tgt)),  K[v][a] = -g R.(a_a(src) x a_u(tgt)).
__device__ inline void mfie_kernel(double k, V3 R, V3 au_t, V3 av_t, V3 au_s, V3 av_s, zd K[2][2]) {
    const double R2 = dot(R, R);
    const double Rn = sqrt(R2);
    double sn, cs;
    sincos(k * Rn, &sn, &cs);
    const double inv = 1.0 / (4.0 * M_PI * R2 * Rn);
    // -(1 + j kR)(cos - j sin) = -(cos + kR sin) - j(kR cos - sin)
    const double gr = -(cs + k * Rn * sn) * inv;
    const double gi = -(k * Rn * cs - sn) * inv;
    const double t00 = dot(R, cross(au_s, av_t));
    const double t01 = dot(R, cross(av_s, av_t));
    const double t10 = -dot(R, cross(au_s, au_t));
    const double t11 = -dot(R, cross(av_s, au_t));
    K[0][0] = zd{gr * t00, gi * t00};
    K[0][1] = zd{gr * t01, gi * t01};
    K[1][0] = zd{gr * t10, gi * t10};
    K[1][1] = zd{gr * t11, gi * t11};
}

// ----------------------------------------------------------- N-Mueller kernel
// Homogeneous dielectric body in vacuum (Sec. II-A, eqs. 7-9 with
// alpha = -eps_2/eps_1, beta = -mu_2/mu_1; eps_1 = mu_1 = 1, omega = k0).
// Unknowns per node (J^u, J^v, M^u, M^v) sqrt(G); rows per node
// (H_u, H_v, E_u, E_v) tested with t_b: t_b . (n x Y) = s_b T_b . Y,
// (s_u, T_u) = (-1, a_v), (s_v, T_v) = (+1, a_u).  With R = r - r',
// G_k = e^{-jkR}/(4 pi R), g_k = -(1 + jkR) e^{-jkR}/(4 pi R^3):
//   S  = G_1 - mu_2 eps_2 G_2,  C_E = g_1 - eps_2 g_2,  C_H = g_1 - mu_2 g_2,
//   X0[b][a] = s_b j w S (T_b . a_a)     -> rows H_b x M^a and E_b x J^a
//   CH[b][a] = -s_b C_H R . (a_a x T_b)  -> H_b x J^a
//   CE[b][a] =  s_b C_E R . (a_a x T_b)  -> E_b x M^a
//   phi[b]   = (j / w) s_b (g_1 - g_2) (T_b . R), the weight of the surface
//              divergence of the source J (E rows) or M (H rows).
// The interior terms are written as differences G_1 - G_2 and g_1 - g_2,
// evaluated from closed forms that do not cancel at small k R.
struct NmMat {
    double k1, k2, w, e2, m2;
};
__device__ inline NmMat nm_mat(const ObjDev& O) {
    return NmMat{O.k0, O.k0 * sqrt(O.eps_r * O.mu_r), O.k0, O.eps_r, O.mu_r};
}

// x cos x - sin x = sum_{n >= 1} (-1)^n 2n x^{2n+1} / (2n+1)!
__device__ inline double xcos_minus_sin(double x) {
    if (fabs(x) < 0.5) {
        const double x2 = x * x;
        double term = x, s = 0.0;
        for (int n = 1; n <= 9; ++n) {
            term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
            s += 2.0 * n * term;
        }
        return s;
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    return x * cs - sn;
}

struct NmVals {
    zd X0[2][2], CH[2][2], CE[2][2], phi[2];
};

__device__ inline void nm_kernel(const NmMat& M, V3 R, V3 au_t, V3 av_t, V3 au_s, V3 av_s, NmVals& o) {
    const double R2 = dot(R, R);
    const double Rn = sqrt(R2);
    const double x1 = M.k1 * Rn, x2 = M.k2 * Rn;
    const double s1 = sin(x1), s2 = sin(x2);
    const double h1 = sin(0.5 * x1), h2 = sin(0.5 * x2);
    const double m1c = -2.0 * h1 * h1, m2c = -2.0 * h2 * h2;   // cos x - 1 = -2 sin^2(x/2)
    const double inv1 = 1.0 / (4.0 * M_PI * Rn), inv3 = inv1 / R2;
    // G_1 and G_1 - G_2:  e^{-jx} = (cos x - 1) + 1 - j sin x
    const zd G1{(1.0 + m1c) * inv1, -s1 * inv1};
    const zd dG{(m1c - m2c) * inv1, -(s1 - s2) * inv1};
    // (1 + jx) e^{-jx} - 1 = (cos x - 1 + x sin x) + j (x cos x - sin x)
    const double q1r = m1c + x1 * s1, q1i = xcos_minus_sin(x1);
    const double q2r = m2c + x2 * s2, q2i = xcos_minus_sin(x2);
    const zd g1{-(1.0 + q1r) * inv3, -q1i * inv3};
    const zd dg{-(q1r - q2r) * inv3, -(q1i - q2i) * inv3};
    const double em = M.e2 * M.m2;
    const zd S = (1.0 - em) * G1 + em * dG;
    const zd CE = (1.0 - M.e2) * g1 + M.e2 * dg;
    const zd CH = (1.0 - M.m2) * g1 + M.m2 * dg;
    const zd jwS{-M.w * S.im, M.w * S.re};
    const V3 T[2] = {av_t, au_t};
    const V3 A[2] = {au_s, av_s};
    for (int b = 0; b < 2; ++b) {
        const double sb = b ? 1.0 : -1.0;
        const double TR = dot(T[b], R);
        // (j / w) s_b TR dg
        const double f = sb * TR / M.w;
        o.phi[b] = zd{-f * dg.im, f * dg.re};
        for (int a = 0; a < 2; ++a) {
            const double Ta = dot(T[b], A[a]);
            const double cr = dot(R, cross(A[a], T[b]));
            o.X0[b][a] = (sb * Ta) * jwS;
            o.CH[b][a] = (-sb * cr) * CH;
            o.CE[b][a] = (sb * cr) * CE;
        }
    }
}

}  // namespace cbie

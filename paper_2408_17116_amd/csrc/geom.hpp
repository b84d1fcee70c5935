// Patch geometry and the MFIE kernel on the device (FP64).
//
// Equiangular cube-sphere patch on an ellipsoid (the paper gives no map for
// its spheres): xi = (2i+1+u)/s - 1, eta = (2j+1+v)/s - 1,
// c = e_n + tan(pi xi/4) e_1 + tan(pi eta/4) e_2, r = center + diag(axes) c/|c|.
// Covariant basis a_u = dr/du, a_v = dr/dv (eq. 14).
#pragma once
#include "common.hpp"

namespace cbie {

struct PatchDev {
    int face, i, j, split;
    int obj;          // object index
    int node0;        // first node (original order)
    int q;
    int pad;
};

struct ObjDev {
    double axes[3];
    double center[3];
    double k0;
    int q;
    int form;
    double eps_r, mu_r;   // interior material (N-Mueller)
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

// r, a_u, a_v of a patch at (u, v)
__device__ inline void patch_eval(const PatchDev& P, const ObjDev& O, double u, double v,
                                  V3& r, V3& au, V3& av) {
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
__device__ inline V3 patch_delta(const PatchDev& P, const ObjDev& O, double u0, double v0,
                                 double du, double dv) {
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

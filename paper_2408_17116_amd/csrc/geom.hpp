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

}  // namespace cbie

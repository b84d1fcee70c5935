"""Curved patches and their local bases (Sec. II-B, eqs. 11, 14, 17, 18).

The paper gives no parametrization for its spheres; an equiangular
cube-sphere is used.  Patch (f, i, j, s) maps (u, v) in [-1, 1]^2 to

    xi  = (2 i + 1 + u)/s - 1,   eta = (2 j + 1 + v)/s - 1,
    c   = e_n + tan(pi xi / 4) e_1 + tan(pi eta / 4) e_2,
    p   = c / |c|,               r = center + diag(axes) p,

with a right-handed face frame (e_n, e_1, e_2), e_1 x e_2 = e_n, so that
a_u x a_v points outward.  Eq. (14): a_u = dr/du, a_v = dr/dv,
n = a_u x a_v / |a_u x a_v|.  Eq. (18) is circular as printed; it is read
with a_n = n and V = sqrt(G) = |a_u x a_v|, which gives the test vectors
t_u = sqrt(G) a^u = a_v x n and t_v = sqrt(G) a^v = n x a_u satisfying the
duality of eq. (17): t_a . a_b = sqrt(G) delta_ab.

Chebyshev-interpolated patches (generic surfaces, e.g. from CAD input):
patch record (6, p, 0, 0) is patch p of a coefficient table C of shape
(n_patches, 3, deg + 1, deg + 1), passed where an ellipsoid passes its
semi-axes, with r(u, v) = sum_{n,m} C[p, :, n, m] T_n(u) T_m(v),
a_u = sum C T_n'(u) T_m(v), a_v = sum C T_n(u) T_m'(v) (T_n' = n U_{n-1}).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cheb

FACE_FRAMES = np.array([
    [[1, 0, 0], [0, 1, 0], [0, 0, 1]],     # +x
    [[-1, 0, 0], [0, 0, 1], [0, 1, 0]],    # -x
    [[0, 1, 0], [0, 0, 1], [1, 0, 0]],     # +y
    [[0, -1, 0], [1, 0, 0], [0, 0, 1]],    # -y
    [[0, 0, 1], [1, 0, 0], [0, 1, 0]],     # +z
    [[0, 0, -1], [0, 1, 0], [1, 0, 0]],    # -z
], dtype=float)


CHEB_FACE = 6


def _cheb_tables(x, deg):
    """T_n(x) and T_n'(x), n = 0..deg, stacked on a last axis."""
    x = np.asarray(x, dtype=float)
    T = [np.ones_like(x), x]
    U = [np.ones_like(x), 2 * x]          # Chebyshev polynomials of the second kind
    for n in range(2, deg + 1):
        T.append(2 * x * T[-1] - T[-2])
        U.append(2 * x * U[-1] - U[-2])
    dT = [np.zeros_like(x)] + [n * U[n - 1] for n in range(1, deg + 1)]
    return np.stack(T[:deg + 1], axis=-1), np.stack(dT, axis=-1)


def _cheb_patch_map(table, idx, u, v):
    C = np.asarray(table)[np.asarray(idx)]               # (..., 3, d+1, d+1)
    deg = C.shape[-1] - 1
    Tu, dTu = _cheb_tables(u, deg)
    Tv, dTv = _cheb_tables(v, deg)
    r = np.einsum("...cnm,...n,...m->...c", C, Tu, Tv)
    au = np.einsum("...cnm,...n,...m->...c", C, dTu, Tv)
    av = np.einsum("...cnm,...n,...m->...c", C, Tu, dTv)
    return r, au, av


def _cheb_diffs(a, d, deg):
    """T_n(a) - T_n(b) for b = a - d, n = 0..deg, without cancellation: the
    step d is taken as given (never formed as a - b), D_0 = 0, D_1 = d and
    D_{n+1} = 2 a D_n + 2 d T_n(b) - D_{n-1}.  Also returns T_n(b)."""
    a = np.asarray(a, dtype=float)
    d = np.asarray(d, dtype=float)
    Tb, _ = _cheb_tables(a - d, deg)
    D = [np.zeros_like(d), d]
    for n in range(1, deg):
        D.append(2 * a * D[n] + 2 * d * Tb[..., n] - D[n - 1])
    return np.stack(D[:deg + 1], axis=-1), Tb


def patch_map(patch, axes, center, u, v):
    """Position and covariant basis at parameter arrays u, v.

    `patch` is (f, i, j, s); each entry may be a scalar or an integer array
    broadcasting against u and v.  Returns r, a_u, a_v of shape (..., 3)."""
    f, i, j, s = (np.asarray(t) for t in patch)
    if np.all(f == CHEB_FACE):
        return _cheb_patch_map(axes, i, u, v)
    frame = FACE_FRAMES[f]                    # (..., 3, 3)
    e_n, e_1, e_2 = frame[..., 0, :], frame[..., 1, :], frame[..., 2, :]
    u = np.asarray(u, dtype=float)
    v = np.asarray(v, dtype=float)
    xi = (2 * i + 1 + u) / s - 1.0
    eta = (2 * j + 1 + v) / s - 1.0
    tx = np.tan(np.pi * xi / 4)
    ty = np.tan(np.pi * eta / 4)
    c = e_n + tx[..., None] * e_1 + ty[..., None] * e_2
    cn = np.linalg.norm(c, axis=-1, keepdims=True)
    p = c / cn
    dc_du = (np.pi / (4 * s))[..., None] * (1 + tx ** 2)[..., None] * e_1
    dc_dv = (np.pi / (4 * s))[..., None] * (1 + ty ** 2)[..., None] * e_2
    dp_du = (dc_du - p * np.sum(p * dc_du, axis=-1, keepdims=True)) / cn
    dp_dv = (dc_dv - p * np.sum(p * dc_dv, axis=-1, keepdims=True)) / cn
    A = np.asarray(axes, dtype=float)
    r = np.asarray(center, dtype=float) + A * p
    return r, A * dp_du, A * dp_dv


@dataclass
class Nodes:
    """Per-node geometry in the unknown order: node = (p q + k) q + l with
    l the u-index and k the v-index."""
    q: int
    n_patches: int
    patches: list
    axes: tuple          # semi-axes, or the Chebyshev coefficient table
    center: tuple
    u: np.ndarray        # [n] parameter of the node
    v: np.ndarray
    patch: np.ndarray    # [n] patch id
    r: np.ndarray        # [n, 3]
    au: np.ndarray
    av: np.ndarray
    n: np.ndarray        # unit normal
    J: np.ndarray        # sqrt(G) = |a_u x a_v|
    tu: np.ndarray       # a_v x n
    tv: np.ndarray       # n x a_u
    w: np.ndarray        # tensor Fejer weight w_l w_k (on [-1,1]^2)

    @property
    def size(self):
        return self.r.shape[0]


def shape_of(spec):
    """What patch_map takes as `axes`: the semi-axes, or the coefficient
    table of Chebyshev-interpolated patches."""
    coeffs = getattr(spec, "coeffs", None)
    return tuple(spec.axes) if coeffs is None else np.asarray(coeffs, dtype=float)


def build_nodes(spec) -> Nodes:
    q = spec.q
    x, wq = cheb.fejer1(q)
    patches = spec.patches()
    U, V = np.meshgrid(x, x, indexing="xy")   # U[k, l] = x_l, V[k, l] = x_k
    W = np.outer(wq, wq)                      # W[k, l] = w_k w_l
    rs, aus, avs, pid, uu, vv, ww = [], [], [], [], [], [], []
    for p, pt in enumerate(patches):
        r, au, av = patch_map(pt, shape_of(spec), spec.center, U, V)
        rs.append(r.reshape(-1, 3))
        aus.append(au.reshape(-1, 3))
        avs.append(av.reshape(-1, 3))
        pid.append(np.full(q * q, p))
        uu.append(U.reshape(-1))
        vv.append(V.reshape(-1))
        ww.append(W.reshape(-1))
    r = np.concatenate(rs)
    au = np.concatenate(aus)
    av = np.concatenate(avs)
    cr = np.cross(au, av)
    Jac = np.linalg.norm(cr, axis=1)
    n = cr / Jac[:, None]
    return Nodes(q=q, n_patches=len(patches), patches=patches,
                 axes=shape_of(spec), center=tuple(spec.center),
                 u=np.concatenate(uu), v=np.concatenate(vv),
                 patch=np.concatenate(pid), r=r, au=au, av=av, n=n, J=Jac,
                 tu=np.cross(av, n), tv=np.cross(n, au), w=np.concatenate(ww))


def patch_diameter(patch, axes, center) -> float:
    """Patch size used by the near test: the longer corner diagonal."""
    r, _, _ = patch_map(patch, axes, center, np.array([-1.0, 1.0, 1.0, -1.0]),
                        np.array([-1.0, 1.0, -1.0, 1.0]))
    return float(max(np.linalg.norm(r[0] - r[1]), np.linalg.norm(r[2] - r[3])))


def project_to_patches(patches, axes, center, targets, iters=80):
    """Closest points of patches to targets, vectorized over pairs.

    `patches` is an integer array [m, 4] of (f, i, j, s), `targets` [m, 3].
    Gauss-Newton on |r(u,v) - target|^2 from the patch centre, each iterate
    clamped to the square.  Returns (u*, v*, distance) arrays of length m."""
    patches = np.asarray(patches)
    pt = tuple(patches[:, c] for c in range(4))
    m = patches.shape[0]
    u = np.zeros(m)
    v = np.zeros(m)
    for _ in range(iters):
        r, au, av = patch_map(pt, axes, center, u, v)
        d = r - targets
        g0 = np.sum(d * au, axis=1)
        g1 = np.sum(d * av, axis=1)
        h00 = np.sum(au * au, axis=1)
        h01 = np.sum(au * av, axis=1)
        h11 = np.sum(av * av, axis=1)
        det = h00 * h11 - h01 * h01
        du = (h11 * g0 - h01 * g1) / det
        dv = (h00 * g1 - h01 * g0) / det
        un = np.clip(u - du, -1.0, 1.0)
        vn = np.clip(v - dv, -1.0, 1.0)
        done = np.max(np.abs(un - u) + np.abs(vn - v)) < 1e-15
        u, v = un, vn
        if done:
            break
    r, _, _ = patch_map(pt, axes, center, u, v)
    return u, v, np.linalg.norm(r - targets, axis=1)


def patch_diff(patch, axes, center, u0, v0, du, dv):
    """r(u0, v0) - r(u0 + du, v0 + dv) without cancellation: the difference
    of the tangents uses tan a - tan b = sin(a - b) / (cos a cos b), the
    difference of the normalisations uses |c|^2 - |c0|^2 = (c - c0).(c + c0).
    Needed where the self-patch kernel is evaluated very close to its
    singular point.  Shapes broadcast; returns (..., 3).  For a
    Chebyshev-interpolated patch, T_n(u0) T_m(v0) - T_n(u1) T_m(v1) =
    (T_n(u0) - T_n(u1)) T_m(v0) + T_n(u1) (T_m(v0) - T_m(v1)), each
    difference from its own recurrence."""
    f, i, j, s = (np.asarray(t) for t in patch)
    if np.all(f == CHEB_FACE):
        C = np.asarray(axes)[i]
        deg = C.shape[-1] - 1
        du = np.asarray(du, dtype=float)
        dv = np.asarray(dv, dtype=float)
        u0 = np.asarray(u0, dtype=float) + 0.0 * du
        v0 = np.asarray(v0, dtype=float) + 0.0 * dv
        Du, Tu1 = _cheb_diffs(u0, -du, deg)
        Dv, _ = _cheb_diffs(v0, -dv, deg)
        Tv0, _ = _cheb_tables(v0, deg)
        return (np.einsum("...cnm,...n,...m->...c", C, Du, Tv0)
                + np.einsum("...cnm,...n,...m->...c", C, Tu1, Dv))
    frame = FACE_FRAMES[f]
    e_n, e_1, e_2 = frame[..., 0, :], frame[..., 1, :], frame[..., 2, :]
    du = np.asarray(du, dtype=float)
    dv = np.asarray(dv, dtype=float)
    a0 = np.pi / 4 * ((2 * i + 1 + u0) / s - 1.0)
    b0 = np.pi / 4 * ((2 * j + 1 + v0) / s - 1.0)
    a1 = a0 + np.pi / 4 * du / s
    b1 = b0 + np.pi / 4 * dv / s
    # c0 - c1 with c = e_n + tan(a) e_1 + tan(b) e_2
    dtx = -np.sin(np.pi / 4 * du / s) / (np.cos(a0) * np.cos(a1))
    dty = -np.sin(np.pi / 4 * dv / s) / (np.cos(b0) * np.cos(b1))
    dc = dtx[..., None] * e_1 + dty[..., None] * e_2
    c0 = e_n + np.tan(a0)[..., None] * e_1 + np.tan(b0)[..., None] * e_2
    c1 = e_n + np.tan(a1)[..., None] * e_1 + np.tan(b1)[..., None] * e_2
    n0 = np.linalg.norm(c0, axis=-1, keepdims=True)
    n1 = np.linalg.norm(c1, axis=-1, keepdims=True)
    # p0 - p1 = dc/|c0| + c1 (1/|c0| - 1/|c1|),
    # 1/|c0| - 1/|c1| = (|c1|^2 - |c0|^2) / (|c0| |c1| (|c0| + |c1|))
    d2 = -np.sum(dc * (c0 + c1), axis=-1, keepdims=True)
    dp = dc / n0 + c1 * d2 / (n0 * n1 * (n0 + n1))
    return np.asarray(axes, dtype=float) * dp

"""N-Mueller equations of a homogeneous dielectric body discretized by the
CBIE (Sec. II-A eqs. 1, 2, 6-9; Sec. II-B eqs. 15-20) — test
infrastructure, FP64/complex128, no shared code with the GPU path.

Media.  Exterior (1): vacuum, eps_1 = mu_1 = 1, k_1 = k0.  Interior (2):
eps_2 = eps_r, mu_2 = mu_r, k_2 = k0 sqrt(eps_r mu_r).  Normalized units,
omega = k0 (eps0 = mu0 = 1), e^{j w t}.

Equations.  The traces (7) of the exterior and interior representations,
combined by (8) with alpha = -eps_2/eps_1, beta = -mu_2/mu_1 (9), scaled by
eps_1 and mu_1:
  E:  -(eps_1 + eps_2)/2 M + n x Y_E = eps_1 n x E_inc,
      Y_E = jw (mu_1 eps_1 S_1 - mu_2 eps_2 S_2)[J]
            - (1/jw) grad (S_1 - S_2)[div' J] + (eps_1 curl S_1 - eps_2 curl S_2)[M]
  H:  (mu_1 + mu_2)/2 J + n x Y_H = mu_1 n x H_inc,
      Y_H = jw (mu_1 eps_1 S_1 - mu_2 eps_2 S_2)[M]
            - (1/jw) grad (S_1 - S_2)[div' M] - (mu_1 curl S_1 - mu_2 curl S_2)[J]
with S_k[f](r) = int G_k(r - r') f dS', curl S_k[f] = int grad G_k x f dS',
grad G_k = g_k(R) R, g_k = -(1 + j k R) e^{-j k R} / (4 pi R^3), R = r - r'.

Unknowns (eq. 11).  F = (J^u, J^v, M^u, M^v) contravariant components times
sqrt(G) at the Chebyshev nodes: J = (F_J^u a_u + F_J^v a_v)/sqrt(G), so that
J dS' = F^a a_a du dv and div' J dS' = (d_u F^u + d_v F^v) du dv, the
derivatives of the patch's Chebyshev interpolant.  Unknown index 4 node + c,
c = 0..3 for J^u, J^v, M^u, M^v.

Testing (eqs. 17-19).  Rows dotted with t_u = a_v x n, t_v = n x a_u;
t_b . (n x Y) = s_b T_b . Y with (s_u, T_u) = (-1, a_v), (s_v, T_v) = (+1, a_u);
t_b . J = F_J^b.  Rows of a node are ordered (H_u, H_v, E_u, E_v) so the
identity terms sit on the diagonal: (mu_1 + mu_2)/2 twice, then
-(eps_1 + eps_2)/2 twice (the right-hand sides are those of eq. 19).

Entries (eq. 20).  Far pairs: Fejer quadrature at the nodes, the derivative
of the interpolant by the Chebyshev differentiation matrix.  Self and near
pairs: exact integrals of kernel x basis (ell_l(u) ell_k(v) or its u- or
v-derivative) by the same Duffy rule as the conductor's oracle.  The
differences G_1 - G_2 and g_1 - g_2 are formed from series at small k R so
that their cancellation loses no digits.
"""
from __future__ import annotations

import math

import numpy as np

from . import cheb
from .geometry import Nodes, patch_diameter, patch_diff, patch_map, project_to_patches
from .mfie import NEAR_DELTA, default_rule, duffy_rule, near_pairs

UPN = 4


class Media:
    def __init__(self, k0, eps_r, mu_r=1.0):
        self.w = float(k0)
        self.e1, self.m1 = 1.0, 1.0
        self.e2, self.m2 = complex(eps_r), complex(mu_r)
        self.k1 = float(k0)
        self.k2 = k0 * np.sqrt(self.e2 * self.m2)

    @property
    def diag(self):
        h = 0.5 * (self.m1 + self.m2)
        e = -0.5 * (self.e1 + self.e2)
        return np.array([h, h, e, e])


# ------------------------------------------------------ stable kernels ---

def _series(z, coef, n_terms=30):
    out = np.zeros_like(z)
    zn = np.ones_like(z)
    for n in range(1, n_terms + 1):
        zn = zn * z
        out = out + coef(n) * zn
    return out


def em1(z):
    """e^{-z} - 1, accurate for small |z|."""
    z = np.asarray(z, dtype=complex)
    small = np.abs(z) < 0.5
    out = np.exp(-z) - 1.0
    if np.any(small):
        out[small] = _series(z[small], lambda n: (-1.0) ** n / math.factorial(n))
    return out


def hm1(z):
    """(1 + z) e^{-z} - 1 = sum_{n >= 2} (-1)^{n+1} (n - 1) z^n / n!,
    accurate for small |z|."""
    z = np.asarray(z, dtype=complex)
    small = np.abs(z) < 0.5
    out = (1.0 + z) * np.exp(-z) - 1.0
    if np.any(small):
        out[small] = _series(z[small], lambda n: (-1.0) ** (n + 1) * (n - 1) / math.factorial(n))
    return out


def green_terms(md: Media, R):
    """G_1, g_1 and the differences G_1 - G_2, g_1 - g_2 at distances R."""
    R = np.asarray(R, dtype=float)
    z1, z2 = 1j * md.k1 * R, 1j * md.k2 * R
    G1 = np.exp(-z1) / (4 * np.pi * R)
    g1 = -(1.0 + z1) * np.exp(-z1) / (4 * np.pi * R ** 3)
    dG = (em1(z1) - em1(z2)) / (4 * np.pi * R)
    dg = -(hm1(z1) - hm1(z2)) / (4 * np.pi * R ** 3)
    return G1, g1, dG, dg


def kernel_entries(md: Media, r_t, au_t, av_t, r_s, au_s, av_s, Rv=None):
    """Integrand coefficients for broadcast target/source arrays (..., 3).

    Returns (K0, Kd): K0 (..., 4, 4) [row c, column a] multiplies the value
    of the source basis; Kd (..., 4, 2) [row c, J or M] multiplies the
    surface divergence d_u F^u + d_v F^v of the source basis of J or M."""
    if Rv is None:
        Rv = r_t - r_s
    R = np.linalg.norm(Rv, axis=-1)
    G1, g1, dG, dg = green_terms(md, R)
    w = md.w
    e1, e2, m1, m2 = md.e1, md.e2, md.m1, md.m2
    # mu_1 eps_1 G_1 - mu_2 eps_2 G_2, written with the stable difference
    S = (m1 * e1 - m2 * e2) * G1 + m2 * e2 * dG
    CE = (e1 - e2) * g1 + e2 * dg      # eps_1 g_1 - eps_2 g_2
    CH = (m1 - m2) * g1 + m2 * dg      # mu_1 g_1 - mu_2 g_2
    T = (av_t, au_t)
    sgn = (-1.0, 1.0)
    src = (au_s, av_s)
    shape = R.shape
    K0 = np.zeros(shape + (4, 4), dtype=complex)
    Kd = np.zeros(shape + (4, 2), dtype=complex)
    for b in range(2):
        Tb = np.broadcast_to(T[b], Rv.shape)
        sb = sgn[b]
        TR = np.sum(Tb * Rv, axis=-1)
        for a in range(2):
            As = np.broadcast_to(src[a], Rv.shape)
            Ta = np.sum(Tb * As, axis=-1)                   # T_b . a_a
            cr = np.sum(Rv * np.cross(As, Tb), axis=-1)     # T_b . (R x a_a)
            # H row b: M^a single layer, J^a curl
            K0[..., b, 2 + a] = sb * 1j * w * S * Ta
            K0[..., b, a] = -sb * CH * cr
            # E row b: J^a single layer, M^a curl
            K0[..., 2 + b, a] = sb * 1j * w * S * Ta
            K0[..., 2 + b, 2 + a] = sb * CE * cr
        # divergence terms: H rows from div M, E rows from div J
        Kd[..., b, 1] = -sb * (1.0 / (1j * w)) * dg * TR
        Kd[..., 2 + b, 0] = -sb * (1.0 / (1j * w)) * dg * TR
    return K0, Kd


# ---------------------------------------------------------- far blocks ---

def far_patch(nd: Nodes, md: Media, ti, p):
    """Fejer-rule entries of target nodes ti against the nodes of patch p:
    complex (len(ti), 4, q*q, 4) [i, c, j_local, a]."""
    q = nd.q
    q2 = q * q
    sl = slice(p * q2, (p + 1) * q2)
    with np.errstate(divide="ignore", invalid="ignore"):
        K0, Kd = kernel_entries(md, nd.r[ti][:, None], nd.au[ti][:, None], nd.av[ti][:, None],
                                nd.r[sl][None], nd.au[sl][None], nd.av[sl][None])
    w = nd.w[sl][None, :, None, None]
    out = (K0 * w).transpose(0, 2, 1, 3).copy()                     # [i, c, j, a]
    D = cheb.diff_matrix(q)                                          # D[l', l]
    Kw = (Kd * nd.w[sl][None, :, None, None]).reshape(len(ti), q, q, 4, 2)  # [i, k, l', c, s]
    # d_u F^u at (k, l') = sum_l D[l', l] F^u(k, l);  d_v F^v at (k', l) = sum_k D[k', k] F^v(k, l)
    du = np.einsum("iklcs,lm->ickms", Kw, D)     # column (k, m), component u
    dv = np.einsum("iklcs,km->icmls", Kw, D)     # column (m, l), component v
    for s in range(2):
        out[:, :, :, 2 * s] += du[..., s].reshape(len(ti), 4, q2)
        out[:, :, :, 2 * s + 1] += dv[..., s].reshape(len(ti), 4, q2)
    return out


def singular_block(nd: Nodes, md: Media, i, p, xs, ys, rule=None):
    """Exact-integral entries of target node i against patch p with the
    (near-)singular point at (xs, ys): complex (4, q*q, 4) [c, j_local, a]."""
    q = nd.q
    pt = nd.patches[p]
    self_patch = (nd.patch[i] == p)
    if rule is None:
        rule = default_rule(nd, i, p, xs, ys, self_patch)
    X, Wt, D = duffy_rule(xs, ys, **rule)
    r_s, au_s, av_s = patch_map(pt, nd.axes, nd.center, X[:, 0], X[:, 1])
    Rv = patch_diff(pt, nd.axes, nd.center, xs, ys, D[:, 0], D[:, 1]) if self_patch else None
    K0, Kd = kernel_entries(md, nd.r[i], nd.au[i], nd.av[i], r_s, au_s, av_s, Rv)
    Lu = cheb.lagrange_basis(q, X[:, 0])      # [l, x]
    Lv = cheb.lagrange_basis(q, X[:, 1])      # [k, x]
    dLu = cheb.lagrange_deriv(q, X[:, 0])
    dLv = cheb.lagrange_deriv(q, X[:, 1])
    K0w = K0 * Wt[:, None, None]
    Kdw = Kd * Wt[:, None, None]
    out = np.einsum("xca,kx,lx->ckla", K0w, Lv, Lu)
    # basis of F^u: d_u (ell_l(u) ell_k(v)) = ell_l'(u) ell_k(v); of F^v: ell_l(u) ell_k'(v)
    du = np.einsum("xcs,kx,lx->ckls", Kdw, Lv, dLu)
    dv = np.einsum("xcs,kx,lx->ckls", Kdw, dLv, Lu)
    for s in range(2):
        out[..., 2 * s] += du[..., s]
        out[..., 2 * s + 1] += dv[..., s]
    return out.reshape(4, q * q, 4)


# ------------------------------------------------------------ assembly ---

def _singular_chunk(args):
    nd, md, chunk, rule = args
    return [singular_block(nd, md, t, p, u, v, rule) for (t, p, u, v, _s) in chunk]


def dense_matrix(nd: Nodes, k0, eps_r, mu_r=1.0, delta=NEAR_DELTA, rule=None, pairs=None, workers=1):
    """Dense complex128 N-Mueller matrix (4n x 4n), original unknown order.
    `workers` > 1 spreads the singular integrals over a pool of spawned
    processes."""
    md = Media(k0, eps_r, mu_r)
    n = nd.size
    q2 = nd.q * nd.q
    A = np.empty((n, 4, n, 4), dtype=complex)
    idx = np.arange(n)
    for p in range(nd.n_patches):
        for a0 in range(0, n, 512):
            ti = idx[a0:a0 + 512]
            A[a0:a0 + 512, :, p * q2:(p + 1) * q2, :] = far_patch(nd, md, ti, p)
    if pairs is None:
        pairs = near_pairs(nd, delta)
    if workers > 1:
        import multiprocessing
        size = max(1, len(pairs) // (8 * workers))
        chunks = [pairs[i:i + size] for i in range(0, len(pairs), size)]
        with multiprocessing.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_singular_chunk, [(nd, md, ch, rule) for ch in chunks])
        blocks = [b for r in res for b in r]
    else:
        blocks = (singular_block(nd, md, t, p, u, v, rule) for (t, p, u, v, _s) in pairs)
    for (t, p, _u, _v, _self), blk in zip(pairs, blocks):
        A[t, :, p * q2:(p + 1) * q2, :] = blk
    A = A.reshape(4 * n, 4 * n)
    A[np.arange(4 * n), np.arange(4 * n)] += np.tile(md.diag, n)
    return A


def matrix_rows(nd: Nodes, k0, eps_r, mu_r=1.0, rows=(), delta=NEAR_DELTA, rule=None):
    """Selected rows (unknown indices) of the same matrix, one by one."""
    md = Media(k0, eps_r, mu_r)
    rows = np.asarray(rows)
    n = nd.size
    q2 = nd.q * nd.q
    pats = np.array(nd.patches)
    diam = np.array([patch_diameter(pt, nd.axes, nd.center) for pt in nd.patches])
    out = np.empty((rows.size, 4 * n), dtype=complex)
    for ri, row in enumerate(rows):
        t, c = divmod(int(row), 4)
        us, vs, dist = project_to_patches(pats, nd.axes, nd.center, np.repeat(nd.r[t][None], nd.n_patches, axis=0))
        blk = np.empty((n, 4), dtype=complex)
        for p in range(nd.n_patches):
            self_p = (p == nd.patch[t])
            if self_p or dist[p] < delta * diam[p]:
                u, v = (nd.u[t], nd.v[t]) if self_p else (us[p], vs[p])
                blk[p * q2:(p + 1) * q2] = singular_block(nd, md, t, p, u, v, rule)[c]
            else:
                blk[p * q2:(p + 1) * q2] = far_patch(nd, md, np.array([t]), p)[0, c]
        r = blk.reshape(-1)
        r[row] += md.diag[c]
        out[ri] = r
    return out


def rhs_planewave(nd: Nodes, k0, khat, pol):
    """Right-hand sides of eq. (19) (eps_1 = mu_1 = 1), rows (H_u, H_v, E_u,
    E_v) per node: (-a_v . H_inc, a_u . H_inc, -a_v . E_inc, a_u . E_inc),
    E_inc = pol e^{-j k0 khat . r}, H_inc = khat x E_inc.  (4n, n_waves)."""
    khat = np.atleast_2d(khat)
    pol = np.atleast_2d(pol)
    n = nd.size
    B = np.empty((4 * n, khat.shape[0]), dtype=complex)
    for w in range(khat.shape[0]):
        ph = np.exp(-1j * k0 * (nd.r @ khat[w]))
        E = pol[w][None, :] * ph[:, None]
        H = np.cross(khat[w], pol[w])[None, :] * ph[:, None]
        B[0::4, w] = -np.sum(nd.av * H, axis=1)
        B[1::4, w] = np.sum(nd.au * H, axis=1)
        B[2::4, w] = -np.sum(nd.av * E, axis=1)
        B[3::4, w] = np.sum(nd.au * E, axis=1)
    return B


def currents(nd: Nodes, x):
    """(J, M) at the nodes from unknowns x (4n,)."""
    x = np.asarray(x)
    J = (x[0::4, None] * nd.au + x[1::4, None] * nd.av) / nd.J[:, None]
    M = (x[2::4, None] * nd.au + x[3::4, None] * nd.av) / nd.J[:, None]
    return J, M


def far_field(nd: Nodes, k0, x, rhat):
    """r e^{j k r} E_s in the far zone from J and M (eta_1 = 1):
    -j k / (4 pi) (N_perp - rhat x L), N = int J e^{j k rhat . r'} dS',
    L = int M e^{j k rhat . r'} dS'."""
    x = np.asarray(x)
    rhat = np.atleast_2d(rhat)
    ph = np.exp(1j * k0 * (rhat @ nd.r.T))
    CJ = nd.w[:, None] * (x[0::4, None] * nd.au + x[1::4, None] * nd.av)
    CM = nd.w[:, None] * (x[2::4, None] * nd.au + x[3::4, None] * nd.av)
    N = ph @ CJ
    L = ph @ CM
    Np = N - rhat * np.sum(rhat * N, axis=1, keepdims=True)
    return -1j * k0 / (4 * np.pi) * (Np - np.cross(rhat, L))


def rcs(nd: Nodes, k0, x, rhat):
    E = far_field(nd, k0, x, rhat)
    return 4 * np.pi * np.sum(np.abs(E) ** 2, axis=1)

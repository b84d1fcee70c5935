"""PEC MFIE discretized by the CBIE (Secs. II-A, II-B).

Equation.  Eqs. (1), (2), (5) and (6) with M = 0 give, on the surface,
    1/2 J - n x curl S[J] = n x H_inc                          (MFIE)
where curl S[J](r) = int grad G(r - r') x J(r') dS' and
grad G = -(1 + j k R) e^{-j k R} / (4 pi R^3) R,  R = r - r'  (eq. 4,
e^{j w t} convention).  Eq. (10) prints "+ n x curl S"; eqs. (2), (5), (6)
fix the sign used here.  The uniform mu_1 row factor of eq. (22) is dropped
on both sides.  Units are normalized (eps0 = mu0 = 1, eta0 = 1).

Unknowns.  J = (F^u a_u + F^v a_v)/sqrt(G) (eq. 11) with F^a sampled at the
Chebyshev nodes; unknown index = 2 node + a (a = 0: u, 1: v).  Then
J dS' = (F^u a_u + F^v a_v) du dv, the Jacobian cancels.

Testing.  Dot with t_u = a_v x n, t_v = n x a_u (eqs. 17, 18): since
t_u . (n x Y) = -a_v . Y and t_v . (n x Y) = a_u . Y,
    row (i,u):  1/2 F^u_i + a_v(i) . curl S[J](r_i) = -a_v(i) . H_inc(r_i)
    row (i,v):  1/2 F^v_i - a_u(i) . curl S[J](r_i) =  a_u(i) . H_inc(r_i)
With a_v(i).(grad G x a) = grad G . (a x a_v(i)) the kernel entries are
    K[u,a] =  g R . (a_a(r') x a_v(i)),   K[v,a] = -g R . (a_a(r') x a_u(i)),
    g = -(1 + j k R) e^{-j k R} / (4 pi R^3).

Entries (eq. 20).  Far pairs: plain Fejer quadrature, A = w_j K(r_j).
Self and near pairs (target i, source patch p): the exact integral
    A[(i,b),(j,a)] = int int K[b,a](u,v) ell_l(u) ell_k(v) du dv
over the Chebyshev interpolant, node j = (p, k, l).  The paper computes these
by a singularity-cancelling change of variables whose details it omits; the
oracle evaluates the same integrals by an independent rule: Duffy (polar)
triangles around the singular point, a sinh map in the angular variable and
geometrically graded Gauss-Legendre panels in the radial variable.

Near test: patch p is near target i iff dist(r_i, p) < delta diam(p),
delta = 1, dist by projection onto the patch, diam = longer corner diagonal;
the patch that owns node i is always "self".
"""
from __future__ import annotations

import numpy as np

from . import cheb
from .geometry import (Nodes, patch_diameter, patch_diff, patch_map,
                       project_to_patches)

NEAR_DELTA = 1.0


# ---------------------------------------------------------------- kernel ---

def kernel_entries(k, r_t, au_t, av_t, r_s, au_s, av_s, Rv=None):
    """K[b, a] for broadcast target/source arrays (..., 3): returns complex
    array (..., 2, 2) indexed [b, a].  Rv = r_t - r_s may be passed in when
    it has been computed without cancellation."""
    if Rv is None:
        Rv = r_t - r_s
    R = np.linalg.norm(Rv, axis=-1)
    g = -(1.0 + 1j * k * R) * np.exp(-1j * k * R) / (4 * np.pi * R ** 3)
    out = np.empty(R.shape + (2, 2), dtype=complex)
    out[..., 0, 0] = g * np.sum(Rv * np.cross(au_s, av_t), axis=-1)
    out[..., 0, 1] = g * np.sum(Rv * np.cross(av_s, av_t), axis=-1)
    out[..., 1, 0] = -g * np.sum(Rv * np.cross(au_s, au_t), axis=-1)
    out[..., 1, 1] = -g * np.sum(Rv * np.cross(av_s, au_t), axis=-1)
    return out


def far_block(nd: Nodes, k, ti, sj):
    """Plain-quadrature entries for target nodes ti and source nodes sj:
    complex (len(ti), 2, len(sj), 2) indexed [i, b, j, a]."""
    K = kernel_entries(k, nd.r[ti][:, None], nd.au[ti][:, None],
                       nd.av[ti][:, None], nd.r[sj][None], nd.au[sj][None],
                       nd.av[sj][None])
    K *= nd.w[sj][None, :, None, None]
    return K.transpose(0, 2, 1, 3)


# ------------------------------------------------ singular quadrature ---

def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def duffy_rule(xs, ys, n_ang=24, n_rad=20, grade=0.2, levels=0):
    """Points and weights on [-1, 1]^2 for integrands with a (near-)
    singularity at or next to (xs, ys).

    The square is cut into triangles with apex (xs, ys) and each edge as
    base, each triangle split at the foot of the perpendicular from the apex.
    On a triangle (apex, A, B): x = apex + s (A + t (B - A) - apex), whose
    Jacobian s |det(A - apex, B - A)| cancels a 1/R singularity at the apex;
    t is mapped by t = t_F + (h / L) sinh(sigma) (h: apex-to-edge distance,
    L = |B - A|, t_F: foot), which flattens the angular peak of width h / L;
    s runs over geometrically graded panels [g^{m+1}, g^m] and [0, g^levels]
    with Gauss-Legendre points on each.  Returns points X, weights W and the
    offsets D = X - apex (formed without subtraction)."""
    P = np.array([xs, ys], dtype=float)
    C = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
    ga, gwa = _gauss(n_ang)
    gr, gwr = _gauss(n_rad)
    # radial panels
    edges = [0.0] + [grade ** m for m in range(levels, 0, -1)] + [1.0]
    s_pts, s_w = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        s_pts.append(0.5 * (b - a) * gr + 0.5 * (b + a))
        s_w.append(0.5 * (b - a) * gwr)
    s_pts = np.concatenate(s_pts)
    s_w = np.concatenate(s_w)
    pts, wts = [], []
    for e in range(4):
        A, B = C[e], C[(e + 1) % 4]
        L = np.linalg.norm(B - A)
        d = (B - A) / L
        tF = np.dot(P - A, d) / L
        h = abs((P - A)[0] * d[1] - (P - A)[1] * d[0])
        if h < 1e-13:
            continue  # apex on this edge: zero-area triangle
        pieces = []
        if 0.0 < tF < 1.0:
            F = A + tF * (B - A)
            pieces = [(A, F), (F, B)]
        else:
            pieces = [(A, B)]
        for (A2, B2) in pieces:
            L2 = np.linalg.norm(B2 - A2)
            if L2 < 1e-15:
                continue
            d2 = (B2 - A2) / L2
            tF2 = np.dot(P - A2, d2) / L2
            area2 = abs((A2 - P)[0] * (B2 - A2)[1] - (A2 - P)[1] * (B2 - A2)[0])
            lo = np.arcsinh((0.0 - tF2) * L2 / h)
            hi = np.arcsinh((1.0 - tF2) * L2 / h)
            sig = 0.5 * (hi - lo) * ga + 0.5 * (hi + lo)
            t = tF2 + (h / L2) * np.sinh(sig)
            wt = 0.5 * (hi - lo) * gwa * (h / L2) * np.cosh(sig)
            E = A2[None, :] + t[:, None] * (B2 - A2)[None, :]    # edge points
            D = s_pts[None, :, None] * (E - P)[:, None, :]       # x - apex
            W = wt[:, None] * s_w[None, :] * s_pts[None, :] * area2
            pts.append(D.reshape(-1, 2))
            wts.append(W.reshape(-1))
    D = np.concatenate(pts)
    return P[None, :] + D, np.concatenate(wts), D


def default_rule(nd: Nodes, i, p, xs, ys, self_patch):
    """Rule size: the self rule needs no radial grading (the Duffy integrand
    is smooth in s); a near target at distance d gets graded panels down to
    about d/4 in parameter units."""
    if self_patch:
        return dict(n_ang=32, n_rad=24, levels=0)
    r, au, av = patch_map(nd.patches[p], nd.axes, nd.center, np.array(xs),
                          np.array(ys))
    d = np.linalg.norm(r - nd.r[i]) / max(np.linalg.norm(au),
                                           np.linalg.norm(av))
    lev = int(np.clip(np.ceil(np.log(max(d, 1e-12) / 4) / np.log(0.2)), 0, 12))
    return dict(n_ang=32, n_rad=16, levels=lev)


def singular_block(nd: Nodes, k, i, p, xs, ys, rule=None):
    """Exact-integral entries for target node i against source patch p with
    the (near-)singular point at parameter (xs, ys): complex (2, q*q, 2)
    indexed [b, j_local, a] with j_local = k q + l."""
    q = nd.q
    pt = nd.patches[p]
    self_patch = (nd.patch[i] == p)
    if rule is None:
        rule = default_rule(nd, i, p, xs, ys, self_patch)
    X, Wt, D = duffy_rule(xs, ys, **rule)
    r_s, au_s, av_s = patch_map(pt, nd.axes, nd.center, X[:, 0], X[:, 1])
    Rv = None
    if self_patch:
        # the target is the apex: form r_i - r(x) without cancellation
        Rv = patch_diff(pt, nd.axes, nd.center, xs, ys, D[:, 0], D[:, 1])
    K = kernel_entries(k, nd.r[i], nd.au[i], nd.av[i], r_s, au_s, av_s, Rv)
    Lu = cheb.lagrange_basis(q, X[:, 0])   # [l, pts]
    Lv = cheb.lagrange_basis(q, X[:, 1])   # [k, pts]
    KW = K * Wt[:, None, None]             # [pts, b, a]
    out = np.einsum("xba,kx,lx->bkla", KW, Lv, Lu)
    return out.reshape(2, q * q, 2)


# ------------------------------------------------------ near structure ---

def near_pairs(nd: Nodes, delta=NEAR_DELTA):
    """List of (target node, patch, u*, v*, self_flag) for every target and
    every patch that is self or within delta * diam of it."""
    q2 = nd.q * nd.q
    P = nd.n_patches
    pats = np.array(nd.patches)
    diam = np.array([patch_diameter(pt, nd.axes, nd.center)
                     for pt in nd.patches])
    cen = np.array([nd.r[p * q2:(p + 1) * q2].mean(axis=0) for p in range(P)])
    rad = np.array([np.max(np.linalg.norm(nd.r[p * q2:(p + 1) * q2] - cen[p],
                                          axis=1)) for p in range(P)])
    out = []
    ti_all, pp_all = [], []
    for p in range(P):
        d = np.linalg.norm(nd.r - cen[p], axis=1)
        # any point of the patch lies within ~1.5 rad of its centroid
        cand = np.nonzero(d < delta * diam[p] + 1.5 * rad[p] + 1e-12)[0]
        cand = cand[nd.patch[cand] != p]
        ti_all.append(cand)
        pp_all.append(np.full(cand.size, p))
    ti = np.concatenate(ti_all)
    pp = np.concatenate(pp_all)
    us, vs, dist = project_to_patches(pats[pp], nd.axes, nd.center, nd.r[ti])
    keep = dist < delta * diam[pp]
    for t, p, u, v in zip(ti[keep], pp[keep], us[keep], vs[keep]):
        out.append((int(t), int(p), float(u), float(v), False))
    for t in range(nd.size):
        out.append((t, int(nd.patch[t]), float(nd.u[t]), float(nd.v[t]), True))
    out.sort(key=lambda e: (e[0], e[1]))
    return out


# ----------------------------------------------------------- assembly ---

def _singular_chunk(args):
    nd, k, chunk, rule = args
    return [singular_block(nd, k, t, p, u, v, rule) for (t, p, u, v, _s) in chunk]


def dense_matrix(nd: Nodes, k, delta=NEAR_DELTA, rule=None, pairs=None, workers=1):
    """Dense complex128 MFIE matrix (2n x 2n) in the original unknown order.
    `workers` > 1 spreads the singular integrals over a pool of spawned
    processes (safe in a process that has initialised a GPU)."""
    n = nd.size
    q2 = nd.q * nd.q
    A = np.empty((n, 2, n, 2), dtype=complex)
    step = 256
    idx = np.arange(n)
    for a0 in range(0, n, step):
        ti = idx[a0:a0 + step]
        with np.errstate(divide="ignore", invalid="ignore"):
            A[a0:a0 + step] = far_block(nd, k, ti, idx)
    if pairs is None:
        pairs = near_pairs(nd, delta)
    if workers > 1:
        import multiprocessing
        size = max(1, len(pairs) // (8 * workers))
        chunks = [pairs[i:i + size] for i in range(0, len(pairs), size)]
        with multiprocessing.get_context("spawn").Pool(workers) as pool:
            results = pool.map(_singular_chunk, [(nd, k, ch, rule) for ch in chunks])
        blocks = [b for r in results for b in r]
    else:
        blocks = (singular_block(nd, k, t, p, u, v, rule) for (t, p, u, v, _s) in pairs)
    for (t, p, u, v, _self), blk in zip(pairs, blocks):
        A[t, :, p * q2:(p + 1) * q2, :] = blk
    A = A.reshape(2 * n, 2 * n)
    A[np.arange(2 * n), np.arange(2 * n)] += 0.5
    return A


def matrix_rows(nd: Nodes, k, rows, delta=NEAR_DELTA, rule=None):
    """Selected rows (unknown indices) of the same matrix, computed one by
    one: far entries for every source node, exact integrals for near ones."""
    rows = np.asarray(rows)
    n = nd.size
    q2 = nd.q * nd.q
    pats = np.array(nd.patches)
    diam = np.array([patch_diameter(pt, nd.axes, nd.center)
                     for pt in nd.patches])
    out = np.empty((rows.size, 2 * n), dtype=complex)
    for ri, row in enumerate(rows):
        t, b = divmod(int(row), 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            blk = far_block(nd, k, np.array([t]), np.arange(n))[0, b]  # [j, a]
        P = nd.n_patches
        us, vs, dist = project_to_patches(
            pats, nd.axes, nd.center, np.repeat(nd.r[t][None], P, axis=0))
        for p in range(P):
            self_p = (p == nd.patch[t])
            if not self_p and not dist[p] < delta * diam[p]:
                continue
            u, v = (nd.u[t], nd.v[t]) if self_p else (us[p], vs[p])
            blk[p * q2:(p + 1) * q2] = singular_block(nd, k, t, p, u, v,
                                                      rule)[b]
        r = blk.reshape(-1)
        r[row] += 0.5
        out[ri] = r
    return out


def rhs_planewave(nd: Nodes, k, khat, pol):
    """Eq. (22) right-hand side (mu_1 dropped): b_u = -a_v . H_inc,
    b_v = a_u . H_inc with E_inc = pol e^{-j k khat . r},
    H_inc = khat x E_inc (eta = 1).  Returns (2n, n_waves)."""
    khat = np.atleast_2d(khat)
    pol = np.atleast_2d(pol)
    n = nd.size
    B = np.empty((2 * n, khat.shape[0]), dtype=complex)
    for w in range(khat.shape[0]):
        ph = np.exp(-1j * k * (nd.r @ khat[w]))
        H = np.cross(khat[w], pol[w])[None, :] * ph[:, None]
        B[0::2, w] = -np.sum(nd.av * H, axis=1)
        B[1::2, w] = np.sum(nd.au * H, axis=1)
    return B


# ------------------------------------------------- scalar layer checks ---

def layer_of_one(nd: Nodes, k, i, kind="S", delta=NEAR_DELTA, pairs=None):
    """int_S K(r_i, r') dS' over the whole surface for the scalar kernels
    K = G (kind 'S', single layer of eq. 3) or K = n' . grad' G (kind 'D',
    double layer), with the same near/far split and singular rule as the
    matrix.  Used only to pin the quadrature machinery to closed forms."""
    q2 = nd.q * nd.q
    r_i = nd.r[i]
    near = {}
    if pairs is None:
        pairs = [e for e in near_pairs(nd, delta) if e[0] == i]
    for (t, p, u, v, _s) in pairs:
        if t == i:
            near[p] = (u, v)

    def kern(Rv, au, av):
        R = np.linalg.norm(Rv, axis=-1)
        if kind == "S":
            return np.exp(-1j * k * R) / (4 * np.pi * R) * np.linalg.norm(np.cross(au, av), axis=-1)
        # n' dS' = (a_u x a_v) du dv ; grad' G = (1 + j k R) e^{-jkR} R / (4 pi R^3)
        g = (1 + 1j * k * R) * np.exp(-1j * k * R) / (4 * np.pi * R ** 3)
        return g * np.sum(Rv * np.cross(au, av), axis=-1)

    total = 0.0 + 0.0j
    for p in range(nd.n_patches):
        sl = slice(p * q2, (p + 1) * q2)
        if p in near:
            u, v = near[p]
            self_patch = (nd.patch[i] == p)
            rule = default_rule(nd, i, p, u, v, self_patch)
            X, Wt, D = duffy_rule(u, v, **rule)
            r_s, au_s, av_s = patch_map(nd.patches[p], nd.axes, nd.center, X[:, 0], X[:, 1])
            Rv = (patch_diff(nd.patches[p], nd.axes, nd.center, u, v, D[:, 0], D[:, 1])
                  if self_patch else r_i - r_s)
            total += np.sum(Wt * kern(Rv, au_s, av_s))
        else:
            total += np.sum(nd.w[sl] * kern(r_i - nd.r[sl], nd.au[sl], nd.av[sl]))
    return total

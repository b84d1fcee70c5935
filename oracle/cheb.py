"""Chebyshev tools of the CBIE discretization (Sec. II-B).

- Fejer's first quadrature rule on [-1, 1]: the nodes are the q zeros of
  T_q (first-kind Chebyshev points, all interior), the weights follow
  Fejer's formula.  The paper's remark that the nodes "include the endpoints"
  does not hold for the first rule; the interior first-kind points are used.
- The nodal -> Chebyshev coefficient map of eq. (13), read with
  alpha_0 = 1, alpha_n = 2 (n > 0), i.e. the discrete orthogonality of
  T_n at first-kind points, and with the second sample coordinate read as
  v_k (eq. 13 prints u_k).
- The nodal (Lagrange) basis ell_l(u) of the interpolant of eq. (12):
  F(u) = sum_l F(u_l) ell_l(u), ell_l(u) = sum_n alpha_n/q T_n(u_l) T_n(u).

Nodes are stored in ascending order.
"""
from __future__ import annotations

import numpy as np


def fejer1(q: int):
    """Fejer-1 nodes (ascending) and weights on [-1, 1].

    x_l = -cos(theta_l), theta_l = (2l+1) pi / (2q);
    w_l = (2/q) [1 - 2 sum_{m=1}^{floor(q/2)} cos(2 m theta_l) / (4 m^2 - 1)].
    (Since cos(2m(pi - theta)) = cos(2m theta) the weights are symmetric and
    the reflection x -> -x used for the ascending order leaves them unchanged.)
    """
    l = np.arange(q)
    theta = (2 * l + 1) * np.pi / (2 * q)
    x = -np.cos(theta)
    w = np.ones(q)
    for m in range(1, q // 2 + 1):
        w -= 2.0 * np.cos(2 * m * theta) / (4 * m * m - 1)
    w *= 2.0 / q
    return x, w


def cheb_T(n_max: int, x):
    """T_0..T_{n_max-1} at x by the three-term recurrence; shape (n_max, *x)."""
    x = np.asarray(x, dtype=float)
    T = np.empty((n_max,) + x.shape)
    T[0] = 1.0
    if n_max > 1:
        T[1] = x
    for n in range(2, n_max):
        T[n] = 2 * x * T[n - 1] - T[n - 2]
    return T


def alpha(q: int) -> np.ndarray:
    a = np.full(q, 2.0)
    a[0] = 1.0
    return a


def coeffs_from_nodal(F: np.ndarray) -> np.ndarray:
    """Eq. (13): gamma[n, m] from nodal values F[k, l] = F(u_l, v_k) on the
    q_u x q_v grid (v index first).  Returns gamma indexed [m, n] to match the
    (v, u) layout: gamma[m, n] multiplies T_n(u) T_m(v)."""
    qv, qu = F.shape
    xu, _ = fejer1(qu)
    xv, _ = fejer1(qv)
    Tu = cheb_T(qu, xu)  # [n, l]
    Tv = cheb_T(qv, xv)  # [m, k]
    au, av = alpha(qu), alpha(qv)
    g = np.einsum("kl,nl,mk->mn", F, Tu, Tv)
    return g * (av[:, None] * au[None, :]) / (qu * qv)


def eval_expansion(gamma: np.ndarray, u, v):
    """Eq. (12): sum_{m,n} gamma[m, n] T_n(u) T_m(v) at scalar or array u, v
    of equal shape."""
    qv, qu = gamma.shape
    Tu = cheb_T(qu, u)
    Tv = cheb_T(qv, v)
    return np.einsum("mn,n...,m...->...", gamma, Tu, Tv)


def lagrange_basis(q: int, u) -> np.ndarray:
    """ell_l(u) for l = 0..q-1 at points u; shape (q, *u)."""
    x, _ = fejer1(q)
    a = alpha(q)
    Tn_nodes = cheb_T(q, x)          # [n, l]
    Tn_u = cheb_T(q, u)              # [n, ...]
    return np.einsum("n,nl,n...->l...", a / q, Tn_nodes, Tn_u)


def lagrange_deriv(q: int, u) -> np.ndarray:
    """ell_l'(u) for l = 0..q-1 at points u in (-1, 1); shape (q, *u).
    Uses T_n'(x) = n U_{n-1}(x)."""
    x, _ = fejer1(q)
    a = alpha(q)
    Tn_nodes = cheb_T(q, x)          # [n, l]
    u = np.asarray(u, dtype=float)
    U = np.empty((q + 1,) + u.shape)
    U[0] = 1.0
    U[1] = 2 * u
    for n in range(2, q + 1):
        U[n] = 2 * u * U[n - 1] - U[n - 2]
    dT = np.zeros((q,) + u.shape)
    for n in range(1, q):
        dT[n] = n * U[n - 1]
    return np.einsum("n,nl,n...->l...", a / q, Tn_nodes, dT)


def diff_matrix(q: int) -> np.ndarray:
    """D[l', l] = ell_l'(u_l'): derivative of the interpolant at the nodes.
    Uses T_n'(x) = n U_{n-1}(x)."""
    x, _ = fejer1(q)
    a = alpha(q)
    Tn_nodes = cheb_T(q, x)               # [n, l]
    # U_{n-1}(x) by recurrence
    U = np.empty((q + 1, q))
    U[0] = 1.0
    U[1] = 2 * x
    for n in range(2, q + 1):
        U[n] = 2 * x * U[n - 1] - U[n - 2]
    dT = np.zeros((q, q))                 # [n, l'] = T_n'(x_l')
    for n in range(1, q):
        dT[n] = n * U[n - 1]
    return np.einsum("n,nl,nm->ml", a / q, Tn_nodes, dT)

"""Adaptive cross approximation with partial pivoting (Sec. III; the paper
compresses admissible blocks "for example" by ACA, its ref. [22], Bebendorf).

A block M (m x n) is approximated by sum_k u_k v_k^T from O(k (m + n))
entries:
  1. take the first unused row i_k (initially row 0), form the residual row
     r = M[i_k, :] - sum_{l<k} u_l[i_k] v_l;
  2. column pivot j_k = argmax |r_j| (lowest index on ties); if |r_j| is
     zero, mark the row used and try the next unused row;
  3. v_k = r / r[j_k]; u_k = M[:, j_k] - sum_{l<k} v_l[j_k] u_l;
  4. update |S_k|_F^2 = |S_{k-1}|_F^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k)
     + |u_k|^2 |v_k|^2 with S_k = sum u v^T;
  5. stop when |u_k| |v_k| <= eps |S_k|_F, else next row i_{k+1} =
     argmax |u_k| over unused rows.
The factors are not unique; compare products and error bounds, not U, V.
"""
from __future__ import annotations

import numpy as np


def aca(row_fn, col_fn, m, n, eps, max_rank=None):
    if max_rank is None:
        max_rank = min(m, n)
    U, V = [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    s2 = 0.0
    while len(U) < max_rank:
        r = np.array(row_fn(i), dtype=complex)
        for u, v in zip(U, V):
            r -= u[i] * v
        used[i] = True
        j = int(np.argmax(np.abs(r)))
        if abs(r[j]) == 0.0:
            free = np.nonzero(~used)[0]
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = np.array(col_fn(j), dtype=complex)
        for uu, vv in zip(U, V):
            u -= vv[j] * uu
        nu, nv = np.linalg.norm(u), np.linalg.norm(v)
        cross = 0.0
        for uu, vv in zip(U, V):
            cross += np.real(np.vdot(uu, u) * np.vdot(vv, v))
        s2 += 2 * cross + (nu * nv) ** 2
        U.append(u)
        V.append(v)
        if nu * nv <= eps * np.sqrt(abs(s2)):
            break
        cand = np.abs(u).copy()
        cand[used] = -1.0
        if np.all(used):
            break
        i = int(np.argmax(cand))
    if not U:
        return np.zeros((m, 0), complex), np.zeros((n, 0), complex)
    return np.array(U).T, np.array(V).T


def svd_rank(M, eps):
    """Smallest rank r with |M - M_r|_F <= eps |M|_F (truncated SVD)."""
    s = np.linalg.svd(M, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]   # tail[r] = |s_r..|
    tot = np.sqrt(np.sum(s ** 2))
    for r in range(len(s) + 1):
        if r == len(s) or tail[r] <= eps * tot:
            return r
    return len(s)

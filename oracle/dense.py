"""Dense direct solve: the plain method the H-matrix solver accelerates.

The paper's comparison point is the uncompressed system solved by LU
decomposition (Sec. I; Sec. IV-A, Fig. 4).  LAPACK's partial-pivot LU
(scipy.linalg.lu_factor / lu_solve) is the solver; a hand-written
right-looking partial-pivot LU for small systems cross-checks it.  LU
factors are not unique under pivot ties, so solutions are compared, never
factors.  component_block_solve is the component-wise approach of
Sec. III-A (eqs. 22-28) with dense blocks.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def solve(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    lu, piv = sla.lu_factor(A, check_finite=False)
    return sla.lu_solve((lu, piv), B, check_finite=False)


def lu_partial_pivot(A: np.ndarray):
    """Textbook Doolittle LU with row partial pivoting, P A = L U.
    Returns (LU packed, perm) with perm[i] = original row at position i."""
    A = np.array(A, dtype=complex)
    n = A.shape[0]
    perm = np.arange(n)
    for j in range(n):
        p = j + int(np.argmax(np.abs(A[j:, j])))
        if p != j:
            A[[j, p]] = A[[p, j]]
            perm[[j, p]] = perm[[p, j]]
        if A[j, j] == 0:
            raise np.linalg.LinAlgError("singular pivot")
        A[j + 1:, j] /= A[j, j]
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
    return A, perm


def lu_solve_small(LU: np.ndarray, perm: np.ndarray, b: np.ndarray):
    n = LU.shape[0]
    y = np.array(b, dtype=complex)[perm]
    for i in range(n):
        y[i] -= LU[i, :i] @ y[:i]
    for i in range(n - 1, -1, -1):
        y[i] = (y[i] - LU[i, i + 1:] @ y[i + 1:]) / LU[i, i]
    return y


def component_order(n_nodes: int, upn: int) -> np.ndarray:
    """Component-wise ordering of one object's unknowns (Sec. III-A,
    eq. 22): entry k of the result is the interleaved index (upn i + a) of
    the unknown at position k = a n_nodes + i, so A[np.ix_(p, p)] is the
    block matrix of the component interaction blocks [K_ab]."""
    a, i = np.divmod(np.arange(upn * n_nodes), n_nodes)
    return upn * i + a


def _leaf_perm(piv):
    """LAPACK's row interchanges as a permutation: (P^T A)[k] = A[perm[k]]."""
    perm = np.arange(piv.size)
    for k, p in enumerate(piv):
        perm[[k, p]] = perm[[p, k]]
    return perm


def _block_factor(K, parts):
    """Block LU of eq. 23 over `parts` diagonal blocks (a power of two):
    K11 = L11 U11; L21 = K21 U11^-1; U12 = L11^-1 K12;
    K22 - L21 U12 = L22 U22, each half factored the same way; a single block
    by partial-pivot LU (row interchanges inside it only)."""
    if parts == 1:
        lu, piv = sla.lu_factor(K, check_finite=False)
        return ("leaf", lu, _leaf_perm(piv))
    n1 = K.shape[0] * (parts // 2) // parts
    F11 = _block_factor(K[:n1, :n1], parts // 2)
    U12 = _lower(F11, K[:n1, n1:])
    L21 = _upper_right(F11, K[n1:, :n1])
    F22 = _block_factor(K[n1:, n1:] - L21 @ U12, parts // 2)
    return ("node", F11, F22, L21, U12, n1)


def _lower(F, B):
    """L^-1 B (forward substitution, eqs. 26-27)."""
    if F[0] == "leaf":
        _, lu, perm = F
        return sla.solve_triangular(lu, B[perm], lower=True, unit_diagonal=True, check_finite=False)
    _, F11, F22, L21, _U12, n1 = F
    X1 = _lower(F11, B[:n1])
    return np.concatenate([X1, _lower(F22, B[n1:] - L21 @ X1)])


def _upper(F, X):
    """U^-1 X (back substitution, eq. 28)."""
    if F[0] == "leaf":
        return sla.solve_triangular(F[1], X, lower=False, check_finite=False)
    _, F11, F22, _L21, U12, n1 = F
    J2 = _upper(F22, X[n1:])
    return np.concatenate([_upper(F11, X[:n1] - U12 @ J2), J2])


def _upper_right(F, C):
    """C U^-1 (the rows of L21 in eq. 23)."""
    if F[0] == "leaf":
        return sla.solve_triangular(F[1], C.T, trans="T", lower=False, check_finite=False).T
    _, F11, F22, _L21, U12, n1 = F
    Y1 = _upper_right(F11, C[:, :n1])
    return np.concatenate([Y1, _upper_right(F22, C[:, n1:] - Y1 @ U12)], axis=1)


def component_block_solve(A: np.ndarray, B: np.ndarray, upn: int) -> np.ndarray:
    """Solve A x = B for one object (interleaved unknowns, upn per node) by
    the component-wise approach of Sec. III-A: reorder to the component
    blocks (eq. 22), block LU (eq. 23, nested for upn = 4), forward
    substitution L X = b (eqs. 24, 26-27), back substitution U x = X
    (eqs. 25, 28), and return x in the interleaved order.  Dense blocks stand
    in for the H-matrices; pivoting stays inside the single-component
    diagonal blocks."""
    p = component_order(A.shape[0] // upn, upn)
    K = np.asarray(A, dtype=complex)[np.ix_(p, p)]
    F = _block_factor(K, upn)
    Bp = np.asarray(B, dtype=complex)[p]
    x = np.empty_like(Bp)
    x[p] = _upper(F, _lower(F, Bp))
    return x


def backward_error(A, x, b):
    r = A @ x - b
    return np.linalg.norm(r) / (np.linalg.norm(A, 2) * np.linalg.norm(x) + np.linalg.norm(b))

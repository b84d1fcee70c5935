"""Dense direct solve: the plain method the H-matrix solver accelerates.

The paper's comparison point is the uncompressed system solved by LU
decomposition (Sec. I; Sec. IV-A, Fig. 4).  LAPACK's partial-pivot LU
(scipy.linalg.lu_factor / lu_solve) is the solver; a hand-written
right-looking partial-pivot LU for small systems cross-checks it.  LU
factors are not unique under pivot ties, so solutions are compared, never
factors.
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


def backward_error(A, x, b):
    r = A @ x - b
    return np.linalg.norm(r) / (np.linalg.norm(A, 2) * np.linalg.norm(x) + np.linalg.norm(b))

"""Incident fields of a point electric dipole and the right-hand sides they
give (test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline use the oracle).

The paper excites its spiral antenna with an x-polarized dipole at the
origin (Sec. IV-A, Fig. 6); the right-hand sides take the dipole's fields
in place of the plane wave's in eq. 22 (MFIE) and eq. 19 (N-Mueller, exterior
vacuum).  Units as everywhere in the oracle: eps = mu = 1, omega = k, time
factor e^{j omega t}.  A current moment m (I l) at r0 has the vector
potential A = m G with G = e^{-jkR} / (4 pi R), R = |r - r0|, so

    H = curl A = grad G x m,
    E = curl H / (j k) = -j k (G m + (grad grad G) m / k^2),

with grad G = G' Rhat, G' = -(1/R + j k) G, and
grad grad G = G'' Rhat Rhat^T + (G' / R) (I - Rhat Rhat^T),
G'' = (2/R^2 + 2 j k / R - k^2) G.
"""
from __future__ import annotations

import numpy as np

from .geometry import Nodes


def fields(r, r0, m, k):
    """E and H (n, 3) complex at points r (n, 3) of a dipole of moment m
    (3,) at r0 (3,) in free space of wavenumber k."""
    r = np.atleast_2d(np.asarray(r, dtype=float))
    m = np.asarray(m, dtype=complex)
    Rv = r - np.asarray(r0, dtype=float)[None, :]
    R = np.linalg.norm(Rv, axis=1)
    Rh = Rv / R[:, None]
    G = np.exp(-1j * k * R) / (4 * np.pi * R)
    G1 = -(1.0 / R + 1j * k) * G
    G2 = (2.0 / R ** 2 + 2j * k / R - k ** 2) * G
    H = np.cross(G1[:, None] * Rh, m[None, :])
    mr = Rh @ m                                   # Rhat . m
    ggm = G2[:, None] * mr[:, None] * Rh + (G1 / R)[:, None] * (m[None, :] - mr[:, None] * Rh)
    E = -1j * k * (G[:, None] * m[None, :] + ggm / k ** 2)
    return E, H


def _tangential(nd: Nodes, F):
    """(-a_v . F, a_u . F) per node."""
    return -np.sum(nd.av * F, axis=1), np.sum(nd.au * F, axis=1)


def rhs_mfie(nd: Nodes, k, pos, mom):
    """Eq. (22) right-hand sides (mu_1 dropped) for dipoles at pos (nd, 3)
    with moments mom (nd, 3): b_u = -a_v . H_inc, b_v = a_u . H_inc.
    Returns (2 n, n_dipoles)."""
    pos, mom = np.atleast_2d(pos), np.atleast_2d(mom)
    B = np.empty((2 * nd.size, pos.shape[0]), dtype=complex)
    for w in range(pos.shape[0]):
        _E, H = fields(nd.r, pos[w], mom[w], k)
        B[0::2, w], B[1::2, w] = _tangential(nd, H)
    return B


def rhs_nmuller(nd: Nodes, k0, pos, mom):
    """Eq. (19) right-hand sides (eps_1 = mu_1 = 1), rows (H_u, H_v, E_u,
    E_v) per node.  Returns (4 n, n_dipoles)."""
    pos, mom = np.atleast_2d(pos), np.atleast_2d(mom)
    B = np.empty((4 * nd.size, pos.shape[0]), dtype=complex)
    for w in range(pos.shape[0]):
        E, H = fields(nd.r, pos[w], mom[w], k0)
        B[0::4, w], B[1::4, w] = _tangential(nd, H)
        B[2::4, w], B[3::4, w] = _tangential(nd, E)
    return B

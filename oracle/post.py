"""Post-processing of the CBIE solution (Secs. II-B, IV).

Surface current from the contravariant unknowns, eq. (11):
J = (F^u a_u + F^v a_v) / sqrt(G).

Far field.  With E_s = -L_E{J} (eq. 1) the far zone gives
E_s ~ -j k e^{-j k r} / (4 pi r) N_perp,  N(r_hat) = int J e^{j k r_hat . r'} dS'
(normalized units), evaluated by the Fejer rule of each patch:
N = sum_nodes w (F^u a_u + F^v a_v) e^{j k r_hat . r}.
Bistatic RCS sigma = 4 pi r^2 |E_s|^2 / |E_0|^2 = k^2 |N_perp|^2 / (4 pi).
"""
from __future__ import annotations

import numpy as np


def surface_current(nd, x):
    """J at the nodes from unknowns x (2n,) or (2n, m)."""
    x = np.asarray(x)
    Fu, Fv = x[0::2], x[1::2]
    if x.ndim == 1:
        return (Fu[:, None] * nd.au + Fv[:, None] * nd.av) / nd.J[:, None]
    return (Fu[:, None, :] * nd.au[:, :, None] + Fv[:, None, :] * nd.av[:, :, None]) / nd.J[:, None, None]


def nodal_unknowns(nd, J):
    """F^a = t_a . J: the unknowns of a given tangential current field J at
    the nodes (t_a . a_b = sqrt(G) delta_ab)."""
    x = np.empty(2 * nd.size, dtype=complex)
    x[0::2] = np.sum(nd.tu * J, axis=1)
    x[1::2] = np.sum(nd.tv * J, axis=1)
    return x


def radiation_vector(nd, k, x, rhat):
    """N(r_hat) for unknowns x (2n,) at directions rhat (m, 3): (m, 3)."""
    Fu, Fv = x[0::2], x[1::2]
    C = nd.w[:, None] * (Fu[:, None] * nd.au + Fv[:, None] * nd.av)   # (n, 3)
    ph = np.exp(1j * k * (rhat @ nd.r.T))                              # (m, n)
    return ph @ C


def rcs(nd, k, x, rhat):
    N = radiation_vector(nd, k, x, rhat)
    Np = N - rhat * np.sum(rhat * N, axis=1, keepdims=True)
    return k ** 2 * np.sum(np.abs(Np) ** 2, axis=1) / (4 * np.pi)


def far_field(nd, k, x, rhat):
    """r e^{j k r} E_s in the far zone: -j k N_perp / (4 pi)."""
    N = radiation_vector(nd, k, x, rhat)
    Np = N - rhat * np.sum(rhat * N, axis=1, keepdims=True)
    return -1j * k * Np / (4 * np.pi)


def plane_cut(theta_deg, phi_deg):
    th = np.deg2rad(np.asarray(theta_deg, dtype=float))
    ph = np.deg2rad(phi_deg)
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)


def weighted_rel_l2(nd, J, Jref):
    """Relative L2 of a surface current, quadrature-weighted
    (sum w sqrt(G) |.|^2)."""
    wt = nd.w * nd.J
    num = np.sum(wt[:, None] * np.abs(J - Jref) ** 2)
    den = np.sum(wt[:, None] * np.abs(Jref) ** 2)
    return float(np.sqrt(num / den))

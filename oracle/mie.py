"""Mie series for a sphere (validation of the MFIE solution, Sec. IV).

Written in the e^{-i w t} convention of Bohren & Huffman (chapter 4) and
converted to the paper's e^{j w t} convention (Sec. I, last paragraph) by
complex conjugation of the phasors, which leaves |.| (RCS) unchanged.

Incident field x-polarised, propagating along +z, unit amplitude, normalized
units (k / (w mu) = 1):  E_i = sum_n E_n (M_o1n^(1) - i N_e1n^(1)),
H_i = -sum_n E_n (M_e1n^(1) + i N_o1n^(1)),  E_n = i^n (2n+1)/(n(n+1)),
scattered  E_s = sum_n E_n (i a_n N_e1n^(3) - b_n M_o1n^(3)),
           H_s = sum_n E_n (i b_n N_o1n^(3) + a_n M_e1n^(3)).
Perfect conductor: tangential E vanishes at r = a, which gives
a_n = psi_n'(x) / xi_n'(x), b_n = psi_n(x) / xi_n(x) with
psi_n = rho j_n, xi_n = rho h_n^(1), x = k a.
Homogeneous dielectric sphere (relative eps_r, mu_r, index m = sqrt(eps_r mu_r)):
continuity of tangential E and H at r = a (B&H eq. 4.53 written with psi, xi)
a_n = (m psi_n(mx) psi_n'(x) - mu_r psi_n(x) psi_n'(mx))
      / (m psi_n(mx) xi_n'(x) - mu_r xi_n(x) psi_n'(mx)),
b_n = (mu_r psi_n(mx) psi_n'(x) - m psi_n(x) psi_n'(mx))
      / (mu_r psi_n(mx) xi_n'(x) - m xi_n(x) psi_n'(mx)),
which tend to the conductor's as m -> infinity.
Surface currents J = r_hat x H and M = E x r_hat at r = a (outside).
Truncation after n_max = x + 4 x^(1/3) + 2 terms (Wiscombe), plus a margin.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def n_terms(x: float) -> int:
    return int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0)) + 8


def riccati(n_max, rho):
    """psi_n, psi_n', xi_n, xi_n' for n = 1..n_max at real rho (scalar or
    array); the n index comes first."""
    rho = np.asarray(rho, dtype=float)
    n = np.arange(1, n_max + 1).reshape((n_max,) + (1,) * rho.ndim)
    j = spherical_jn(n, rho)
    jd = spherical_jn(n, rho, derivative=True)
    y = spherical_yn(n, rho)
    yd = spherical_yn(n, rho, derivative=True)
    h = j + 1j * y
    hd = jd + 1j * yd
    return rho * j, j + rho * jd, rho * h, h + rho * hd


def pec_coefficients(x: float):
    nmax = n_terms(x)
    psi, dpsi, xi, dxi = riccati(nmax, x)
    return dpsi / dxi, psi / xi


def dielectric_coefficients(x: float, eps_r, mu_r=1.0):
    nmax = n_terms(x)
    m = np.sqrt(complex(eps_r) * complex(mu_r))
    if abs(m.imag) < 1e-15:
        m = m.real
    mu_r = complex(mu_r).real if abs(complex(mu_r).imag) < 1e-15 else complex(mu_r)
    psi, dpsi, xi, dxi = riccati(nmax, x)
    n = np.arange(1, nmax + 1)
    pm = m * x * spherical_jn(n, m * x)
    dpm = spherical_jn(n, m * x) + m * x * spherical_jn(n, m * x, derivative=True)
    an = (m * pm * dpsi - mu_r * psi * dpm) / (m * pm * dxi - mu_r * xi * dpm)
    bn = (mu_r * pm * dpsi - m * psi * dpm) / (mu_r * pm * dxi - m * xi * dpm)
    return an, bn


def pi_tau(n_max, mu):
    """Angular functions pi_n, tau_n (n = 1..n_max) at mu = cos(theta)."""
    mu = np.asarray(mu, dtype=float)
    pi = np.zeros((n_max + 1,) + mu.shape)
    tau = np.zeros((n_max + 1,) + mu.shape)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, n_max + 1):
        pi[n] = ((2 * n - 1) / (n - 1)) * mu * pi[n - 1] - (n / (n - 1)) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def _sph(r):
    x, y, z = r[..., 0], r[..., 1], r[..., 2]
    rr = np.linalg.norm(r, axis=-1)
    th = np.arccos(np.clip(z / rr, -1, 1))
    ph = np.arctan2(y, x)
    return rr, th, ph


def _basis(th, ph):
    er = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], -1)
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(th)], -1)
    return er, et, ep


def _fields_bh(k, a, r, which, coef=None):
    """Total E and H (B&H convention) at points r, outside or on the sphere.
    which = 'H' or 'E'; coef = (a_n, b_n), the conductor's by default.
    Returns complex (..., 3)."""
    x = k * a
    an, bn = pec_coefficients(x) if coef is None else coef
    nmax = an.size
    n = np.arange(1, nmax + 1)
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    rr, th, ph = _sph(r)
    rho = k * rr
    er, et, ep = _basis(th, ph)
    pi, tau = pi_tau(nmax, np.cos(th))
    psi, dpsi, xi, dxi = riccati(nmax, rho)
    # radial factors: z_n = psi/rho, [rho z_n]'/rho = psi'/rho
    z1, d1 = psi / rho, dpsi / rho
    z3, d3 = xi / rho, dxi / rho
    cp, sp = np.cos(ph), np.sin(ph)
    st = np.sin(th)
    nn = (n * (n + 1)).reshape((nmax,) + (1,) * np.ndim(th))

    def M_o(z):
        return (cp * pi * z)[..., None] * et - (sp * tau * z)[..., None] * ep

    def M_e(z):
        return -(sp * pi * z)[..., None] * et - (cp * tau * z)[..., None] * ep

    def N_o(z, d):
        return ((sp * nn * st * pi * z / rho)[..., None] * er
                + (sp * tau * d)[..., None] * et + (cp * pi * d)[..., None] * ep)

    def N_e(z, d):
        return ((cp * nn * st * pi * z / rho)[..., None] * er
                + (cp * tau * d)[..., None] * et - (sp * pi * d)[..., None] * ep)

    Ex = En.reshape((nmax,) + (1,) * np.ndim(th))
    A = an.reshape(Ex.shape)
    B = bn.reshape(Ex.shape)
    if which == "E":
        inc = Ex[..., None] * (M_o(z1) - 1j * N_e(z1, d1))
        sca = Ex[..., None] * (1j * A[..., None] * N_e(z3, d3) - B[..., None] * M_o(z3))
    else:
        inc = -Ex[..., None] * (M_e(z1) + 1j * N_o(z1, d1))
        sca = Ex[..., None] * (1j * B[..., None] * N_o(z3, d3) + A[..., None] * M_e(z3))
    return np.sum(inc + sca, axis=0)


def pec_surface_current(k, a, r):
    """J = n x H_total on the sphere |r| = a at points r (..., 3), in the
    paper's e^{j w t} convention."""
    r = np.asarray(r, dtype=float)
    H = _fields_bh(k, a, r, "H")
    rr = np.linalg.norm(r, axis=-1, keepdims=True)
    J = np.cross(r / rr, H)
    return np.conj(J)


def dielectric_surface_currents(k, a, eps_r, mu_r, r):
    """(J, M) = (n x H_1, E_1 x n) on the sphere |r| = a at points r
    (..., 3), exterior total fields, e^{j w t} convention."""
    r = np.asarray(r, dtype=float)
    coef = dielectric_coefficients(k * a, eps_r, mu_r)
    H = _fields_bh(k, a, r, "H", coef)
    E = _fields_bh(k, a, r, "E", coef)
    n = r / np.linalg.norm(r, axis=-1, keepdims=True)
    return np.conj(np.cross(n, H)), np.conj(np.cross(E, n))


def dielectric_amplitudes(k, a, eps_r, mu_r, theta):
    an, bn = dielectric_coefficients(k * a, eps_r, mu_r)
    return _amplitudes(an, bn, theta)


def dielectric_rcs(k, a, eps_r, mu_r, theta):
    """Bistatic RCS (phi = 0, phi = 90 deg) of the dielectric sphere."""
    S1, S2 = dielectric_amplitudes(k, a, eps_r, mu_r, theta)
    return 4 * np.pi * np.abs(S2) ** 2 / k ** 2, 4 * np.pi * np.abs(S1) ** 2 / k ** 2


def pec_total_field(k, a, r, which="E"):
    """Total E or H (e^{j w t} convention) at points r with |r| >= a."""
    return np.conj(_fields_bh(k, a, np.asarray(r, dtype=float), which))


def pec_amplitudes(k, a, theta):
    """S1, S2 at scattering angles theta (B&H eq. 4.74)."""
    an, bn = pec_coefficients(k * a)
    return _amplitudes(an, bn, theta)


def _amplitudes(an, bn, theta):
    nmax = an.size
    n = np.arange(1, nmax + 1)
    pi, tau = pi_tau(nmax, np.cos(theta))
    f = ((2 * n + 1) / (n * (n + 1)))[:, None]
    S1 = np.sum(f * (an[:, None] * pi + bn[:, None] * tau), axis=0)
    S2 = np.sum(f * (an[:, None] * tau + bn[:, None] * pi), axis=0)
    return S1, S2


def pec_rcs(k, a, theta):
    """Bistatic RCS for x-polarised +z incidence: (sigma_E at phi = 0,
    sigma_H at phi = 90 deg), sigma = 4 pi |S|^2 / k^2."""
    S1, S2 = pec_amplitudes(k, a, theta)
    return 4 * np.pi * np.abs(S2) ** 2 / k ** 2, 4 * np.pi * np.abs(S1) ** 2 / k ** 2


def efficiencies(an, bn, x):
    n = np.arange(1, an.size + 1)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(an + bn))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(an) ** 2 + np.abs(bn) ** 2))
    return qext, qsca

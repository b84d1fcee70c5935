"""Pins of the N-Mueller oracle (Secs. II-A, II-B): the dielectric Mie
series (optical theorem, Rayleigh limit, vanishing contrast), the dense
CBIE solution converging to the Mie surface currents J and M and the RCS,
the exactly diagonal matrix of a scatterer with the exterior's material, the
cancellation-free kernel differences, and the row-by-row assembly."""
import numpy as np
import pytest

from oracle import geometry as G, mie, muller as Mu, post
from synth import workloads as W

KH, POL = np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]])


def test_dielectric_mie_coefficients():
    for x, er in ((2.0, 4.0), (5.0, 16.0), (0.7, 50.0)):
        an, bn = mie.dielectric_coefficients(x, er)
        qe, qs = mie.efficiencies(an, bn, x)
        assert abs(qe - qs) < 1e-10 * qe          # lossless: extinction = scattering
    an, bn = mie.dielectric_coefficients(2.0, 1.0)
    assert np.abs(an).max() == 0.0 and np.abs(bn).max() == 0.0
    # Rayleigh limit (electric dipole): a_1 = -(2i/3) x^3 (m^2 - 1)/(m^2 + 2) (1 + O(x^2)),
    # b_1 = O(x^5), in the e^{-iwt} convention the coefficients are written in
    for x, er in ((0.01, 4.0), (0.003, 16.0)):
        an, bn = mie.dielectric_coefficients(x, er)
        ref = -(2j / 3) * x ** 3 * (er - 1) / (er + 2)
        assert abs(an[0] - ref) < 5 * x ** 2 * abs(ref)
        assert abs(bn[0]) < 5 * x ** 2 * abs(ref)


def test_kernel_differences_have_no_cancellation():
    z = 1j * np.array([0.3, 0.45, 0.49])
    assert np.abs(Mu.hm1(z) - ((1 + z) * np.exp(-z) - 1)).max() < 1e-14
    assert np.abs(Mu.em1(z) - np.expm1(-z.imag * 1j)).max() < 1e-15
    # leading Taylor terms at tiny argument, where the direct forms lose
    # all digits: (1 + z) e^{-z} - 1 = -z^2/2 + z^3/3 - z^4/8 + ..., e^{-z} - 1 = -z + z^2/2 - z^3/6 + ...
    z = 1j * np.array([1e-7, 1e-4])
    assert np.allclose(Mu.hm1(z), -z ** 2 / 2 + z ** 3 / 3 - z ** 4 / 8, rtol=1e-12, atol=0)
    assert np.allclose(Mu.em1(z), -z + z ** 2 / 2 - z ** 3 / 6, rtol=1e-12, atol=0)


def test_matching_materials_give_a_diagonal_matrix():
    """eps_r = mu_r = 1: the interior and exterior operators cancel, the
    matrix is the identity terms, and the solution is the incident traces
    J = n x H_inc, M = E_inc x n."""
    spec = W.tiny_sphere(s=1, q=3, k0=1.3)
    nd = G.build_nodes(spec)
    A = Mu.dense_matrix(nd, spec.k0, 1.0, 1.0, workers=4)
    d = np.diag(A).copy()
    assert np.abs(A - np.diag(d)).max() == 0.0
    assert np.allclose(d, np.tile([1.0, 1.0, -1.0, -1.0], nd.size))
    b = Mu.rhs_planewave(nd, spec.k0, KH, POL)[:, 0]
    J, M = Mu.currents(nd, b / d)
    ph = np.exp(-1j * spec.k0 * nd.r[:, 2])[:, None]
    E = POL[0][None] * ph
    H = np.cross(KH[0], POL[0])[None] * ph
    assert np.abs(J - np.cross(nd.n, H)).max() < 1e-14
    assert np.abs(M - np.cross(E, nd.n)).max() < 1e-14


def _mie_errors(s, q, k0=1.0, er=4.0):
    spec = W.ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=s, q=q, k0=k0)
    nd = G.build_nodes(spec)
    A = Mu.dense_matrix(nd, k0, er, 1.0, workers=8)
    x = np.linalg.solve(A, Mu.rhs_planewave(nd, k0, KH, POL)[:, 0])
    J, M = Mu.currents(nd, x)
    Jm, Mm = mie.dielectric_surface_currents(k0, 1.0, er, 1.0, nd.r)
    th = np.arange(0, 181, 10)
    sE, sH = mie.dielectric_rcs(k0, 1.0, er, 1.0, np.deg2rad(th))
    s0 = Mu.rcs(nd, k0, x, post.plane_cut(th, 0.0))
    s90 = Mu.rcs(nd, k0, x, post.plane_cut(th, 90.0))
    return (np.linalg.norm(J - Jm) / np.linalg.norm(Jm), np.linalg.norm(M - Mm) / np.linalg.norm(Mm),
            max(np.abs(s0 - sE).max() / sE.max(), np.abs(s90 - sH).max() / sH.max()))


def test_dense_solution_converges_to_dielectric_mie():
    """eps_r = 4, ka = 1: a sign or factor error in any of the sixteen
    kernel entries, the divergence terms or the identity gives an O(1) gap."""
    e1 = _mie_errors(1, 4)
    e2 = _mie_errors(2, 4)
    print(f"s=1 q=4: J {e1[0]:.2e} M {e1[1]:.2e} RCS {e1[2]:.2e}; s=2 q=4: J {e2[0]:.2e} M {e2[1]:.2e} RCS {e2[2]:.2e}")
    assert max(e2) < 1e-3
    assert e2[0] < 0.2 * e1[0] and e2[1] < 0.2 * e1[1]


@pytest.mark.slow
def test_dense_solution_converges_spectrally_in_q():
    e5 = _mie_errors(2, 5)
    e6 = _mie_errors(2, 6)
    assert max(e6) < 5e-6 and e6[0] < 0.2 * e5[0]


def test_rows_match_dense_assembly():
    spec = W.ObjectSpec(axes=(1.0, 0.8, 0.6), center=(0.0, 0.0, 0.0), s=1, q=4, k0=2.0)
    nd = G.build_nodes(spec)
    A = Mu.dense_matrix(nd, spec.k0, 9.0, 1.0, workers=4)
    rows = np.array([0, 5, 66, 4 * nd.size - 1])
    R = Mu.matrix_rows(nd, spec.k0, 9.0, 1.0, rows)
    assert np.abs(R - A[rows]).max() < 1e-13 * np.abs(A).max()

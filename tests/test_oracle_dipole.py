"""Pins of the oracle's point-dipole excitation (Sec. IV-A: the spiral
antenna's x-polarized dipole source) to what fixes a radiating dipole:
Maxwell's curl equations (by central differences), the radiated power of a
Hertzian dipole, the transverse far zone, and the plane wave a distant
dipole becomes, whose right-hand sides must approach the plane-wave ones of
eqs. 19 and 22."""
import numpy as np
import pytest

from oracle import dipole, geometry as G, mfie, muller
from synth import workloads as W


def _curl(f, r, h):
    """Curl of a complex vector field f (points (n, 3) -> (n, 3)) by central
    differences."""
    J = np.empty((r.shape[0], 3, 3), dtype=complex)   # J[:, i, j] = d f_i / d x_j
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, :, j] = (f(r + e) - f(r - e)) / (2 * h)
    return np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], axis=1)


def test_fields_satisfy_maxwell():
    # curl E = -j k H and curl H = j k E away from the source (e^{j w t},
    # eps = mu = 1, omega = k)
    rng = np.random.default_rng(2)
    k = 2.3
    r0 = np.array([0.2, -0.1, 0.4])
    m = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    d = rng.standard_normal((20, 3))
    r = r0 + d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(0.3, 3.0, 20)[:, None]
    E, H = dipole.fields(r, r0, m, k)
    cE = _curl(lambda x: dipole.fields(x, r0, m, k)[0], r, 1e-5)
    cH = _curl(lambda x: dipole.fields(x, r0, m, k)[1], r, 1e-5)
    assert np.abs(cE + 1j * k * H).max() < 1e-7 * np.abs(H).max()
    assert np.abs(cH - 1j * k * E).max() < 1e-7 * np.abs(E).max()


@pytest.mark.parametrize("radius", [0.7, 5.0])
def test_radiated_power_of_a_hertzian_dipole(radius):
    # Re of the Poynting flux through any sphere around the dipole is
    # k^2 |m|^2 / (12 pi) (eta = 1); the reactive near fields carry none
    k = 3.1
    m = np.array([0.3, -1.2j, 0.5 + 0.4j])
    x, wx = np.polynomial.legendre.leggauss(48)            # cos(theta)
    ph = np.arange(96) * 2 * np.pi / 96
    ct, P = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    n = np.stack([st * np.cos(P), st * np.sin(P), ct], axis=-1).reshape(-1, 3)
    w = (np.outer(wx, np.full(96, 2 * np.pi / 96)) * radius ** 2).ravel()
    E, H = dipole.fields(radius * n, np.zeros(3), m, k)
    S = 0.5 * np.real(np.sum(np.cross(E, np.conj(H)) * n, axis=1))
    power = np.sum(w * S)
    exact = k ** 2 * np.vdot(m, m).real / (12 * np.pi)
    assert abs(power - exact) < 1e-10 * exact


def test_far_zone_is_transverse():
    k = 2.0
    m = np.array([1.0, 0.5, -0.3])
    d = np.array([[0.3, 0.4, 0.866], [-0.6, 0.8, 0.0]])
    d /= np.linalg.norm(d, axis=1)[:, None]
    R = 1e6 / k
    E, H = dipole.fields(R * d, np.zeros(3), m, k)
    for i in range(2):
        assert abs(np.dot(E[i], d[i])) < 1e-5 * np.linalg.norm(E[i])
        assert np.linalg.norm(H[i] - np.cross(d[i], E[i])) < 1e-5 * np.linalg.norm(H[i])
        # amplitude: |E| = k |m_perp| / (4 pi R)
        mt = m - np.dot(m, d[i]) * d[i]
        assert abs(np.linalg.norm(E[i]) - k * np.linalg.norm(mt) / (4 * np.pi * R)) < 1e-5 * np.linalg.norm(E[i])


def test_distant_dipole_gives_the_plane_wave_right_hand_sides():
    # an x-directed dipole at (0, 0, -D) is, near the origin, the plane wave
    # propagating +z polarized +x, scaled by c = -j k e^{-jkD} / (4 pi D):
    # the right-hand sides of both formulations converge to the plane-wave
    # ones as 1/D
    spec = W.tiny_sphere(s=2, q=4, k0=3.0)
    nd = G.build_nodes(spec)
    k = spec.k0
    kh, pol = W.axial_wave()
    ref = {"mfie": mfie.rhs_planewave(nd, k, kh, pol), "nm": muller.rhs_planewave(nd, k, kh, pol)}
    errs = {"mfie": [], "nm": []}
    for D in (1e4, 1e5):
        c = -1j * k * np.exp(-1j * k * D) / (4 * np.pi * D)
        pos, mom = np.array([[0.0, 0.0, -D]]), np.array([[1.0, 0.0, 0.0]])
        for name, b in (("mfie", dipole.rhs_mfie(nd, k, pos, mom)), ("nm", dipole.rhs_nmuller(nd, k, pos, mom))):
            errs[name].append(np.linalg.norm(b / c - ref[name]) / np.linalg.norm(ref[name]))
    for name in errs:
        e4, e5 = errs[name]
        assert e5 < 1e-4 and e4 / e5 > 5, (name, e4, e5)

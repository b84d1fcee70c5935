"""Pins of the oracle's Chebyshev-interpolated patches (generic surface
input, the form a CAD surface is handed over in; Sec. II-B, eqs. 11-14 on
patches of any shape) to what fixes them: a flat patch is represented
exactly; the interpolant reproduces the surface at its Chebyshev points;
a sphere's radius and area and a torus's area converge to their closed
forms; the cancellation-free difference equals the direct one and its
first-order limit; the layer potentials of one on the interpolated sphere
take their closed forms, the static double layer on the torus is -1/2
(Gauss), and the MFIE current on the interpolated sphere converges to the
Mie series."""
import numpy as np
import pytest

from oracle import dense, geometry as G, mfie, mie, post
from synth import workloads as W


def test_flat_patch_is_exact():
    # degree 1: r = c + alpha u e1 + beta v e2, area 4 alpha beta by the
    # Fejer rule exactly, constant basis and normal
    c, e1, e2 = np.array([0.3, -1.0, 2.0]), np.array([0.6, 0.8, 0.0]), np.array([0.0, 0.0, 1.0])
    alpha, beta = 0.7, 1.9
    C = np.zeros((1, 3, 2, 2))
    C[0, :, 0, 0], C[0, :, 1, 0], C[0, :, 0, 1] = c, alpha * e1, beta * e2
    spec = W.ObjectSpec(axes=(1, 1, 1), center=(0, 0, 0), s=0, q=5, k0=1.0, coeffs=C)
    nd = G.build_nodes(spec)
    assert abs(np.sum(nd.w * nd.J) - 4 * alpha * beta) < 1e-14
    assert np.abs(nd.au - alpha * e1).max() < 1e-15 and np.abs(nd.av - beta * e2).max() < 1e-15
    assert np.abs(nd.n - np.cross(e1, e2)).max() < 1e-15
    assert np.abs(nd.r - (c + alpha * np.outer(nd.u, e1) + beta * np.outer(nd.v, e2))).max() < 1e-15


def test_interpolant_reproduces_the_surface_at_its_points():
    deg = 9
    spec = W.torus_cheb(6, 3, 4, 1.0, deg, R=1.3, rho=0.5)
    x = np.cos(np.pi * (np.arange(deg + 1) + 0.5) / (deg + 1))
    U, V = np.meshgrid(x, x, indexing="ij")
    for p in (0, 7, 17):
        a, b = divmod(p, 3)
        th = 2 * np.pi * (a + 0.5 * (U + 1)) / 6
        ph = 2 * np.pi * (b + 0.5 * (V + 1)) / 3
        ex = np.stack([(1.3 + 0.5 * np.cos(ph)) * np.cos(th), (1.3 + 0.5 * np.cos(ph)) * np.sin(th),
                       0.5 * np.sin(ph)], axis=-1)
        r, _, _ = G.patch_map((G.CHEB_FACE, p, 0, 0), spec.coeffs, None, U, V)
        assert np.abs(r - ex).max() < 1e-14


def test_sphere_radius_and_area_converge():
    errs = []
    for deg in (6, 10, 14):
        nd = G.build_nodes(W.gnomonic_sphere_cheb(2, 11, 1.0, deg))
        rad = np.abs(np.linalg.norm(nd.r, axis=1) - 1.0).max()
        area = abs(np.sum(nd.w * nd.J) - 4 * np.pi)
        errs.append((rad, area))
    assert errs[0][0] < 2e-5 and errs[2][0] < 1e-10
    assert errs[0][1] < 1e-3 and errs[2][1] < 1e-7 and errs[2][1] < errs[0][1] / 1e3
    # the outward normal of the sphere is its position
    nd = G.build_nodes(W.gnomonic_sphere_cheb(2, 8, 1.0, 14))
    assert np.abs(np.sum(nd.n * nd.r, axis=1) - 1.0).max() < 1e-8


def test_torus_area():
    nd = G.build_nodes(W.torus_cheb(8, 4, 6, 1.0, 12, R=1.0, rho=0.4))
    assert abs(np.sum(nd.w * nd.J) - 4 * np.pi ** 2 * 1.0 * 0.4) < 1e-11


def test_cancellation_free_difference():
    nd = G.build_nodes(W.torus_cheb(8, 4, 6, 1.0, 12))
    for p in (3, 20):
        pt = nd.patches[p]
        u0, v0 = 0.3, -0.7
        for h in (1e-1, 1e-3):
            d = G.patch_diff(pt, nd.axes, nd.center, u0, v0, h, -0.5 * h)
            r0, _, _ = G.patch_map(pt, nd.axes, nd.center, u0, v0)
            r1, _, _ = G.patch_map(pt, nd.axes, nd.center, u0 + h, v0 - 0.5 * h)
            assert np.abs(d - (r0 - r1)).max() < 1e-14
        # first-order limit: r(u0) - r(u0 + du) -> -(a_u du + a_v dv)
        _, au, av = G.patch_map(pt, nd.axes, nd.center, u0, v0)
        for h in (1e-9, 1e-13):
            d = G.patch_diff(pt, nd.axes, nd.center, u0, v0, h, -0.5 * h)
            assert np.abs(d / h + (au - 0.5 * av)).max() < 5 * h + 1e-13


def test_layer_potentials_of_one_on_the_interpolated_sphere():
    # S[1] and D[1] on a sphere of radius a (closed forms), here through
    # Chebyshev patches of degree 14 of the gnomonic cube sphere
    nd = G.build_nodes(W.gnomonic_sphere_cheb(1, 8, 1.0, 14))
    pairs = mfie.near_pairs(nd)
    k, a = 1.0, 1.0
    Sx = np.exp(-1j * k * a) * np.sin(k * a) / k
    Dx = -(1 / (4 * a)) * (2 * (1 - np.exp(-2j * k * a)) / (1j * k) - 2 * a * np.exp(-2j * k * a))
    for i in (0, 37, 200):
        pi = [e for e in pairs if e[0] == i]
        assert abs(mfie.layer_of_one(nd, k, i, "S", pairs=pi) - Sx) < 2e-6
        assert abs(mfie.layer_of_one(nd, k, i, "D", pairs=pi) - Dx) < 2e-6


def test_static_double_layer_on_the_torus_is_minus_half():
    nd = G.build_nodes(W.torus_cheb(8, 4, 6, 1e-9, 12))
    pairs = mfie.near_pairs(nd)
    for i in (0, 100, 700):
        pi = [e for e in pairs if e[0] == i]
        assert abs(mfie.layer_of_one(nd, 1e-9, i, "D", pairs=pi) + 0.5) < 1e-6


@pytest.mark.slow
def test_mfie_current_on_the_interpolated_sphere_converges_to_mie():
    errs = []
    for q in (4, 6):
        nd = G.build_nodes(W.gnomonic_sphere_cheb(1, q, 1.0, 14))
        A = mfie.dense_matrix(nd, 1.0, workers=4)
        b = mfie.rhs_planewave(nd, 1.0, *W.axial_wave())[:, 0]
        x = dense.solve(A, b)
        Jm = mie.pec_surface_current(1.0, 1.0, nd.r)
        errs.append(post.weighted_rel_l2(nd, post.surface_current(nd, x), Jm))
    assert errs[0] < 1e-2 and errs[1] < 1e-3 and errs[1] < errs[0] / 8

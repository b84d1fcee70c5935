"""Pins of the oracle's building blocks to closed forms (not the GPU path).

Fejer-1 rule, Chebyshev maps (eqs. 12-13), geometry and bases (eqs. 11, 14,
17, 18), the cancellation-free patch difference, the Duffy rule against the
closed-form integral of 1/R over rectangles, dense LU against LAPACK, the
component-wise block LU (Sec. III-A, eqs. 22-28) against LAPACK.
"""
import numpy as np
import pytest
from scipy.special import ellipeinc, ellipkinc

from oracle import cheb, dense, geometry as G
from oracle import mfie
from synth import workloads as W


@pytest.mark.parametrize("q", [3, 4, 6, 8, 11])
def test_fejer_moments(q):
    x, w = cheb.fejer1(q)
    assert np.all(np.diff(x) > 0) and np.all(np.abs(x) < 1)
    # exact for all polynomials of degree <= q-1
    for m in range(q):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(w * x ** m) - exact) < 1e-14
    # first-kind nodes are the zeros of T_q
    assert np.max(np.abs(np.cos(q * np.arccos(x)))) < 1e-13


@pytest.mark.parametrize("q", [4, 8])
def test_chebyshev_round_trip_and_exactness(q):
    x, _ = cheb.fejer1(q)
    rng = np.random.default_rng(0)
    F = rng.standard_normal((q, q))
    g = cheb.coeffs_from_nodal(F)
    U, V = np.meshgrid(x, x, indexing="xy")
    assert np.max(np.abs(cheb.eval_expansion(g, U, V) - F)) < 1e-13
    # a known polynomial of degree < q in each variable is reproduced
    p = lambda u, v: 1 + 2 * u ** (q - 1) - 3 * u * v ** 2 + v ** (q - 1)
    g = cheb.coeffs_from_nodal(p(U, V))
    uu, vv = rng.uniform(-1, 1, 20), rng.uniform(-1, 1, 20)
    assert np.max(np.abs(cheb.eval_expansion(g, uu, vv) - p(uu, vv))) < 1e-12
    # Lagrange basis: partition of unity, cardinality, derivative matrix
    L = cheb.lagrange_basis(q, uu)
    assert np.max(np.abs(L.sum(axis=0) - 1)) < 1e-13
    assert np.max(np.abs(cheb.lagrange_basis(q, x) - np.eye(q))) < 1e-13
    D = cheb.diff_matrix(q)
    f = x ** (q - 1) + x ** 2
    df = (q - 1) * x ** (q - 2) + 2 * x
    assert np.max(np.abs(D @ f - df)) < 1e-11


def test_sphere_geometry_pins():
    spec = W.sphere_pec_small()
    nd = G.build_nodes(spec)
    assert np.max(np.abs(np.linalg.norm(nd.r, axis=1) - 1)) < 1e-14
    assert np.max(np.abs(np.sum(nd.n * nd.r, axis=1) - 1)) < 1e-14   # outward
    # eq. (17) duality of the test vectors
    assert np.max(np.abs(np.sum(nd.tu * nd.au, 1) - nd.J)) < 1e-14
    assert np.max(np.abs(np.sum(nd.tv * nd.av, 1) - nd.J)) < 1e-14
    assert np.max(np.abs(np.sum(nd.tu * nd.av, 1))) < 1e-14
    assert np.max(np.abs(np.sum(nd.tv * nd.au, 1))) < 1e-14


def test_sphere_area_converges_spectrally():
    errs = []
    for q in (4, 6, 8):
        nd = G.build_nodes(W.tiny_sphere(s=2, q=q))
        errs.append(abs(np.sum(nd.w * nd.J) - 4 * np.pi))
    assert errs[2] < 1e-7 and errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20


def test_ellipsoid_area_legendre():
    # Legendre's closed form with incomplete elliptic integrals (a > b > c)
    a, b, c = 2.0, 1.3, 0.7
    spec = W.ObjectSpec(axes=(a, b, c), center=(0.3, -0.2, 0.1), s=3, q=10, k0=1.0)
    nd = G.build_nodes(spec)
    phi = np.arccos(c / a)
    m = a * a * (b * b - c * c) / (b * b * (a * a - c * c))
    S = 2 * np.pi * c * c + 2 * np.pi * a * b / np.sin(phi) * (
        ellipeinc(phi, m) * np.sin(phi) ** 2 + ellipkinc(phi, m) * np.cos(phi) ** 2)
    assert abs(np.sum(nd.w * nd.J) - S) / S < 1e-7
    # normals point away from the centre
    assert np.all(np.sum(nd.n * (nd.r - np.array(spec.center)), axis=1) > 0)


def test_patch_diff_matches_direct_difference():
    pt = (3, 1, 0, 2)
    u0, v0 = 0.37, -0.81
    du = np.array([0.2, -1e-3, 0.5])
    dv = np.array([-0.1, 2e-3, 0.3])
    d = G.patch_diff(pt, (1.2, 1.0, 0.8), (0, 0, 0), u0, v0, du, dv)
    r0, _, _ = G.patch_map(pt, (1.2, 1.0, 0.8), (0, 0, 0), u0, v0)
    r1, _, _ = G.patch_map(pt, (1.2, 1.0, 0.8), (0, 0, 0), u0 + du, v0 + dv)
    assert np.max(np.abs(d - (r0 - r1))) < 1e-15
    # tiny offsets: the difference is first order in the offset, d ~ -(a_u du + a_v dv)
    _, au, av = G.patch_map(pt, (1.2, 1.0, 0.8), (0, 0, 0), u0, v0)
    h = 1e-9
    d = G.patch_diff(pt, (1.2, 1.0, 0.8), (0, 0, 0), u0, v0, h, -h)
    assert np.max(np.abs(d + (au * h - av * h))) < 1e-16


def _rect_one_over_R(a, b, h):
    """int_0^a int_0^b 1/sqrt(x^2 + y^2 + h^2) dx dy (closed form)."""
    d = np.sqrt(a * a + b * b + h * h)
    v = a * np.log((b + d) / np.sqrt(a * a + h * h)) + b * np.log((a + d) / np.sqrt(b * b + h * h))
    if h > 0:
        v -= h * np.arctan(a * b / (h * d))
    return v


@pytest.mark.parametrize("x0,y0,h", [(0.0, 0.0, 0.0), (0.3, -0.7, 0.0), (0.98, 0.1, 0.0),
                                     (0.999, 0.999, 0.0), (0.5, 0.5, 1e-3), (1.0, 0.3, 0.02)])
def test_duffy_rule_closed_forms(x0, y0, h):
    X, W_, D = mfie.duffy_rule(x0, y0, n_ang=32, n_rad=20, levels=10)
    assert abs(W_.sum() - 4.0) < 1e-13
    assert np.max(np.abs(X - (np.array([x0, y0]) + D))) < 1e-15
    num = np.sum(W_ / np.sqrt((X[:, 0] - x0) ** 2 + (X[:, 1] - y0) ** 2 + h * h))
    ex = 0.0
    for a in (1 - x0, 1 + x0):
        for b in (1 - y0, 1 + y0):
            if a > 0 and b > 0:
                ex += _rect_one_over_R(a, b, h)
    if x0 == 0 and y0 == 0 and h == 0:
        assert abs(ex - 8 * np.arcsinh(1.0)) < 1e-14   # the centred square
    assert abs(num - ex) < 1e-10 * ex


def test_hand_lu_matches_lapack():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))
    b = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    LU, perm = dense.lu_partial_pivot(A)
    x1 = dense.lu_solve_small(LU, perm, b)
    x2 = dense.solve(A, b)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-12
    assert dense.backward_error(A, x2, b) < 1e-15


def test_component_order_gathers_the_component_blocks():
    # position a n + i holds unknown (node i, component a): the blocks of the
    # reordered matrix are the strided component interactions of eq. 22
    rng = np.random.default_rng(5)
    for upn, n in ((2, 7), (4, 5)):
        A = rng.standard_normal((upn * n, upn * n))
        p = dense.component_order(n, upn)
        assert sorted(p) == list(range(upn * n))
        K = A[np.ix_(p, p)]
        for a in range(upn):
            for b in range(upn):
                assert np.array_equal(K[a * n:(a + 1) * n, b * n:(b + 1) * n], A[a::upn, b::upn])


@pytest.mark.parametrize("upn,n", [(2, 37), (4, 19)])
def test_component_block_solve_matches_lapack(upn, n):
    # eqs. 23-28 with dense blocks reproduce the plain solve; the component
    # diagonal blocks are made dominant so that no pivoting across them is
    # needed (the H-LU pivots inside diagonal leaves only)
    rng = np.random.default_rng(upn)
    N = upn * n
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 4.0 * np.sqrt(N) * np.eye(N)
    B = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
    x = dense.component_block_solve(A, B, upn)
    xr = dense.solve(A, B)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-12


def test_component_block_solve_on_the_cbie_matrices():
    # the MFIE (2 components) and N-Mueller (4) matrices of a small sphere:
    # the component-wise solve equals the interleaved LAPACK solve
    from oracle import muller
    spec = W.tiny_sphere(s=1, q=4, k0=2.0)
    nd = G.build_nodes(spec)
    A = mfie.dense_matrix(nd, spec.k0)
    b = mfie.rhs_planewave(nd, spec.k0, *W.axial_wave())
    xr = dense.solve(A, b)
    assert np.linalg.norm(dense.component_block_solve(A, b, 2) - xr) / np.linalg.norm(xr) < 1e-11
    A4 = muller.dense_matrix(nd, spec.k0, 4.0)
    b4 = muller.rhs_planewave(nd, spec.k0, *W.axial_wave())
    xr4 = dense.solve(A4, b4)
    assert np.linalg.norm(dense.component_block_solve(A4, b4, 4) - xr4) / np.linalg.norm(xr4) < 1e-11

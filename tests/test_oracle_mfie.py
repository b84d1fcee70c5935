"""Pins of the oracle's MFIE system (eqs. 10, 11, 19-22) and Mie series.

The MFIE pins are end-to-end: a dropped term, a wrong sign or a transposed
index anywhere in the far kernel, the singular rule, the right-hand side or
the post-processing breaks the spectral convergence towards the Mie surface
current and RCS, the closed-form layer potentials, or reciprocity.
"""
import numpy as np
import pytest

from oracle import dense, geometry as G, mfie, mie, post
from synth import workloads as W


# ------------------------------------------------------------------ Mie ---

def test_mie_optical_theorem_and_rayleigh():
    for x in (0.3, 2 * np.pi, 20.0):
        an, bn = mie.pec_coefficients(x)
        qe, qs = mie.efficiencies(an, bn, x)
        assert abs(qe - qs) < 1e-12 * qe
    # Rayleigh limit of the PEC backscatter efficiency: 9 x^4
    x = 0.01
    sE, _ = mie.pec_rcs(x, 1.0, np.array([np.pi]))
    assert abs(sE[0] / np.pi - 9 * x ** 4) < 1e-3 * 9 * x ** 4


def test_mie_boundary_condition_and_tangential_current():
    k = 2 * np.pi
    rng = np.random.default_rng(0)
    p = rng.standard_normal((12, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    E = mie.pec_total_field(k, 1.0, p, "E")
    assert np.max(np.abs(np.cross(p, E))) < 1e-13 * np.max(np.abs(E))
    J = mie.pec_surface_current(k, 1.0, p)
    assert np.max(np.abs(np.sum(J * p, axis=1))) < 1e-14
    # physical optics on the lit pole for a large sphere: J ~ 2 n x H_inc
    k = 60.0
    Jp = mie.pec_surface_current(k, 1.0, np.array([[1e-9, 0.0, -1.0]]))[0]
    po = 2 * np.exp(1j * k) * np.array([1.0, 0.0, 0.0])
    assert np.linalg.norm(Jp - po) < 0.02 * 2


# -------------------------------------------------- singular machinery ---

@pytest.mark.parametrize("s,q,k", [(1, 8, 1.0), (2, 8, 2 * np.pi)])
def test_layer_potentials_of_one_on_sphere(s, q, k):
    nd = G.build_nodes(W.tiny_sphere(s, q, k))
    pairs = mfie.near_pairs(nd)
    a = 1.0
    Sx = np.exp(-1j * k * a) * np.sin(k * a) / k
    Dx = -(1 / (4 * a)) * (2 * (1 - np.exp(-2j * k * a)) / (1j * k) - 2 * a * np.exp(-2j * k * a))
    for i in (0, 37, 200):
        pi = [e for e in pairs if e[0] == i]
        S = mfie.layer_of_one(nd, k, i, "S", pairs=pi)
        D = mfie.layer_of_one(nd, k, i, "D", pairs=pi)
        tol = 1e-12 if k == 1.0 else 2e-6      # discretization error at ka = 2 pi, q = 8
        assert abs(S - Sx) < tol and abs(D - Dx) < tol


def test_static_double_layer_is_minus_half():
    # Gauss: the static double layer of 1 on a closed surface is -1/2
    nd = G.build_nodes(W.ObjectSpec(axes=(1.5, 1.0, 0.7), center=(0, 0, 0), s=2, q=8, k0=1e-9))
    pairs = mfie.near_pairs(nd)
    for i in (3, 300):
        pi = [e for e in pairs if e[0] == i]
        D = mfie.layer_of_one(nd, 1e-9, i, "D", pairs=pi)
        assert abs(D + 0.5) < 1e-6


def test_singular_rule_self_consistency():
    nd = G.build_nodes(W.sphere_pec_small())
    k = 2 * np.pi
    for i in (0, 5, 27):
        p, u, v = nd.patch[i], nd.u[i], nd.v[i]
        b1 = mfie.singular_block(nd, k, i, p, u, v)
        b2 = mfie.singular_block(nd, k, i, p, u, v, rule=dict(n_ang=48, n_rad=36, levels=0))
        assert np.max(np.abs(b1 - b2)) < 1e-12 * np.max(np.abs(b2))
    # the closest near pair of this mesh (target 0.0054 m off the patch)
    b1 = mfie.singular_block(nd, k, 7, 2, -1.0, -0.9807852804032301)
    b2 = mfie.singular_block(nd, k, 7, 2, -1.0, -0.9807852804032301,
                             rule=dict(n_ang=48, n_rad=24, levels=12))
    assert np.max(np.abs(b1 - b2)) < 1e-11 * np.max(np.abs(b2))


def test_far_and_exact_entries_agree_on_smooth_densities():
    # Beyond the near threshold the plain Fejer entries differ from the exact
    # integrals against the Chebyshev basis entry by entry (the rule is not
    # exact for ell_l times the kernel), but applied to a smooth current they
    # agree to the discretization level.  The near/far split is therefore
    # part of the matrix definition and both implementations must classify
    # pairs identically.
    nd = G.build_nodes(W.sphere_pec_ka20())
    k = 20.0
    pats = np.array(nd.patches)
    diam = G.patch_diameter(nd.patches[0], nd.axes, nd.center)
    ti = np.arange(64, 64 * 60)
    us, vs, dist = G.project_to_patches(np.repeat(pats[[0]], ti.size, 0), nd.axes, nd.center, nd.r[ti])
    Jm = mie.pec_surface_current(k, 1.0, nd.r[:64])
    F = np.stack([np.sum(nd.tu[:64] * Jm, 1), np.sum(nd.tv[:64] * Jm, 1)], 1)
    sel = np.nonzero((dist > diam) & (dist < 1.1 * diam))[0][:3]
    assert sel.size > 0
    for s_ in sel:
        i = ti[s_]
        ex = mfie.singular_block(nd, k, i, 0, us[s_], vs[s_])
        far = mfie.far_block(nd, k, np.array([i]), np.arange(64))[0]
        a = np.einsum("bja,ja->b", ex, F)
        b = np.einsum("bja,ja->b", far, F)
        assert np.max(np.abs(a - b)) < 1e-6 * np.max(np.abs(a))
        assert np.max(np.abs(ex - far)) > 1e-4 * np.max(np.abs(ex))


# ------------------------------------------------------ MFIE vs Mie ---

@pytest.fixture(scope="module")
def small_systems():
    out = {}
    for q in (4, 6):
        spec = W.tiny_sphere(s=1, q=q, k0=1.0)
        nd = G.build_nodes(spec)
        A = mfie.dense_matrix(nd, spec.k0)
        kh, pol = W.axial_wave()
        b = mfie.rhs_planewave(nd, spec.k0, kh, pol)[:, 0]
        out[q] = (nd, A, b, dense.solve(A, b))
    return out


def test_mfie_current_converges_to_mie(small_systems):
    errs = []
    for q in (4, 6):
        nd, A, b, x = small_systems[q]
        Jm = mie.pec_surface_current(1.0, 1.0, nd.r)
        errs.append(post.weighted_rel_l2(nd, post.surface_current(nd, x), Jm))
        # the Mie current satisfies the discrete equations to the same order
        xm = post.nodal_unknowns(nd, Jm)
        assert np.linalg.norm(A @ xm - b) / np.linalg.norm(b) < 3 * errs[-1]
    assert errs[0] < 2e-3 and errs[1] < 6e-5 and errs[1] < errs[0] / 15


def test_mfie_rcs_matches_mie(small_systems):
    nd, A, b, x = small_systems[6]
    th = np.linspace(0, 180, 181)
    sE, sH = mie.pec_rcs(1.0, 1.0, np.deg2rad(th))
    rE = post.rcs(nd, 1.0, x, post.plane_cut(th, 0.0))
    rH = post.rcs(nd, 1.0, x, post.plane_cut(th, 90.0))
    assert np.linalg.norm(rE - sE) / np.linalg.norm(sE) < 1e-3
    assert np.linalg.norm(rH - sH) / np.linalg.norm(sH) < 1e-3


def test_dense_solution_backward_error(small_systems):
    nd, A, b, x = small_systems[6]
    assert dense.backward_error(A, x, b) < 1e-14


def test_reciprocity_on_ellipsoid():
    spec = W.ObjectSpec(axes=(1.2, 0.8, 0.6), center=(0.1, 0.0, -0.1), s=1, q=5, k0=1.5)
    nd = G.build_nodes(spec)
    k = spec.k0
    A = mfie.dense_matrix(nd, k)
    ki = np.array([0.3, -0.5, 0.81]); ki /= np.linalg.norm(ki)
    ks = np.array([-0.7, 0.2, 0.4]); ks /= np.linalg.norm(ks)
    ei = np.cross(ki, [0, 1.0, 0]); ei /= np.linalg.norm(ei)
    es = np.cross(ks, [1.0, 0, 0]); es /= np.linalg.norm(es)
    b1 = mfie.rhs_planewave(nd, k, ki, ei)[:, 0]
    b2 = mfie.rhs_planewave(nd, k, -ks, es)[:, 0]
    x1, x2 = dense.solve(A, b1), dense.solve(A, b2)
    f1 = post.far_field(nd, k, x1, ks[None])[0] @ es
    f2 = post.far_field(nd, k, x2, -ki[None])[0] @ ei
    # converges with q (5e-3, 1.8e-3, 5.8e-4 at q = 4, 5, 6); a sign or
    # transposition error in the RHS or far field gives an O(1) mismatch
    assert abs(f1 - f2) < 3e-3 * abs(f1)


@pytest.mark.slow
def test_mfie_converges_spectrally_beyond_order_eight():
    """The oracle at q = 10 (the paper's 10 x 10 points per patch): a sphere
    of one wavelength radius (ka = 2 pi), one patch per cube face of 1.57
    wavelengths; the surface current against Mie falls from 4.1e-3 at q = 8
    to 2.3e-4 at q = 10."""
    errs = {}
    for q in (8, 10):
        spec = W.ObjectSpec(axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), s=1, q=q, k0=2 * np.pi)
        nd = G.build_nodes(spec)
        kh, pol = W.axial_wave()
        x = dense.solve(mfie.dense_matrix(nd, spec.k0, workers=4), mfie.rhs_planewave(nd, spec.k0, kh, pol)[:, 0])
        Jm = mie.pec_surface_current(spec.k0, 1.0, nd.r)
        errs[q] = post.weighted_rel_l2(nd, post.surface_current(nd, x), Jm)
    assert errs[8] < 6e-3 and errs[10] < 4e-4 and errs[10] < errs[8] / 8


@pytest.mark.parametrize("spec", [W.ObjectSpec(axes=(1.0, 0.8, 0.6), center=(0.1, 0.0, 0.0), s=1, q=4, k0=2.0),
                                  W.tiny_sphere(s=2, q=3, k0=3.0)], ids=["ellipsoid_s1q4", "sphere_s2q3"])
def test_rows_match_dense_assembly(spec):
    """The row routine (the checker of every full-size sampled-row test) and
    the dense assembly reach their entries by different loops (per row: a
    projection onto every patch; dense: the near-pair list): both must give
    the same matrix, first, last and interior rows of both components."""
    nd = G.build_nodes(spec)
    A = mfie.dense_matrix(nd, spec.k0, workers=4)
    n2 = 2 * nd.size
    rows = np.array([0, 1, 7, n2 // 2, n2 // 2 + 1, n2 - 2, n2 - 1])
    R = mfie.matrix_rows(nd, spec.k0, rows)
    assert np.abs(R - A[rows]).max() < 1e-13 * np.abs(A).max()
